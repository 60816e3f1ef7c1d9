"""The launches bench.py times, at their full shapes and batch sizes: the
batched multiply gives every job the bits of that job's plain multiply, and
a sampled job matches the oracle's multiply bit for bit.

Inputs are uniform residues per limb from a seeded torch generator (not
from the library); the sampled job is copied to the host for the oracle.
"""
import numpy as np
import pytest
import torch

from oracle import keys as okeys, mult, params as oparams
from paper_2601_15401_amd import mick

pytestmark = pytest.mark.gpu

# the bench workloads: (log_n, L, K, dnum, k, level, batch)
CONFIGS = {
    "n16_k8_b8": (16, 32, 8, 4, 8, 32, 8),
    "n15_k4_b16": (15, 16, 4, 4, 4, 16, 16),
    "paper3": (16, 24, 24, 1, 3, 24, 8),
}


def _uniform_cts(prm, jobs, k, level, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    q = torch.tensor(prm.q[:level], dtype=torch.int64, device="cuda").view(level, 1)
    out = torch.empty(jobs, k, 2, level, prm.N, dtype=torch.int32, device="cuda")
    for j in range(jobs):
        r = torch.randint(0, 1 << 62, (k, 2, level, prm.N), generator=g, dtype=torch.int64, device="cuda")
        out[j] = (r % q).to(torch.int32)
    return out


@pytest.mark.parametrize("name", list(CONFIGS))
def test_batched_launch_at_full_size(name):
    log_n, L, K, dnum, k, level, jobs = CONFIGS[name]
    seed = 60 + list(CONFIGS).index(name)
    prm = mick.Params(log_n, L, K, dnum)
    gk = mick.Keys(prm, seed, k)
    cts = _uniform_cts(prm, jobs, k, level, seed)
    out = mick.mul_relin_rescale_batch(prm, gk, cts, level)
    assert out.shape == (jobs, 2, level - k + 1, prm.N)
    for j in range(jobs):
        plain = mick.mul_relin_rescale(prm, gk, [cts[j, u] for u in range(k)], level)
        assert torch.equal(out[j], plain), "%s: job %d differs from its plain multiply" % (name, j)
    j = jobs - 1
    host = mick.to_numpy_u32(cts[j]).astype(np.uint64)
    op = oparams.make_params(log_n, L, K, dnum)
    ok = okeys.keygen(op, seed, k)
    want = mult.mul_relin_rescale(op, ok, [host[u] for u in range(k)], level)
    got = mick.to_numpy_u32(out[j]).astype(np.uint64)
    bad = np.argwhere(got != want)
    assert bad.size == 0, "%s job %d: %d residues differ from the oracle, first at %s" % (
        name, j, len(bad), bad[0].tolist())
