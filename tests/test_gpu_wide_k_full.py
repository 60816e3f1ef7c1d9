"""GPU parity at the widths and ring degrees where the oracle takes minutes:
k = 9..12 at N = 2^16 (32 + 8 primes, dnum 4), N = 2^15 (16 + 4, dnum 4) and
N = 2^14 (12 + 2, dnum 4), covering the fused tensor kernel's widest
instantiations (eleven d_t tiles in LDS with 128- and 256-row pass-B blocks)
and the heavy requests of the mixed and served workloads (N = 2^16, k = 12).

The expected values are per-limb SHA-256 digests of the oracle's multiply on
the same seeded inputs, written by tests/golden/make_wide_k_digests.py (which
calls only the oracle); every output limb of the library must hash to the
oracle's digest, i.e. match it bit for bit.

The job-table path (one launch per stage for mixed k and level), its graph
replay, and the work queue run the same inputs plus further shapes at
N = 2^15 and 2^16; every job must equal its plain multiply and the digest
cases also the oracle.
"""
import os

import numpy as np
import pytest
import torch

from paper_2601_15401_amd import mick
from seeded_inputs import limb_digests, uniform_cts

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DIGESTS = os.path.join(HERE, "golden", "wide_k_digests.txt")


def _load_digests():
    cases = {}
    if not os.path.exists(DIGESTS):  # checked by test_golden_digests.py
        return cases
    with open(DIGESTS) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            vals = [int(v) for v in parts[1:10]]
            cases[parts[0]] = (tuple(vals), parts[10:])
    return cases


CASES = _load_digests()
_sets = {}


def _set(log_n, L, K, dnum, key_seed, k_max):
    key = (log_n, L, K, dnum, key_seed, k_max)
    if key not in _sets:
        prm = mick.Params(log_n, L, K, dnum)
        _sets[key] = (prm, mick.Keys(prm, key_seed, k_max))
    return _sets[key]


def _case_inputs(name):
    (log_n, L, K, dnum, ks, kmax, k, level, iseed), digests = CASES[name]
    prm, keys = _set(log_n, L, K, dnum, ks, kmax)
    cts = [mick.from_numpy_u32(c) for c in uniform_cts(iseed, prm.q[:level], prm.N, k)]
    return prm, keys, cts, level, digests


def _check_digests(out, digests, what):
    got = limb_digests(mick.to_numpy_u32(out))
    assert len(got) == len(digests), (what, len(got), len(digests))
    bad = [i for i, (g, w) in enumerate(zip(got, digests)) if g != w]
    n_limbs = len(got) // 2
    assert not bad, "%s: %d of %d output limbs differ from the oracle, first poly %d limb %d" % (
        what, len(bad), len(got), bad[0] // n_limbs, bad[0] % n_limbs)


@pytest.mark.parametrize("name", sorted(CASES))
def test_wide_k_multiply_matches_oracle(name):
    prm, keys, cts, level, digests = _case_inputs(name)
    print("case", name, flush=True)
    out = mick.mul_relin_rescale(prm, keys, cts, level)
    _check_digests(out, digests, name)
    # the same job in a same-shape batch of two
    k = len(cts)
    batch = torch.stack([torch.stack(cts), torch.stack(cts)])
    outb = mick.mul_relin_rescale_batch(prm, keys, batch, level)
    assert torch.equal(outb[0], out) and torch.equal(outb[1], out), name


def _random_ct(rng, prm, level):
    return mick.from_numpy_u32(np.stack([np.stack([rng.integers(0, q, prm.N, dtype=np.int64).astype(np.uint32)
                                                   for q in prm.q[:level]]) for _ in range(2)]))


# extra (k, level) shapes per ring degree besides the digest cases
EXTRA = {16: [(2, 32), (7, 20), (12, 12), (5, 9), (3, 4)], 15: [(3, 16), (8, 10), (12, 12), (2, 2), (6, 15)]}


@pytest.mark.parametrize("log_n", [15, 16])
def test_job_table_wide_k_equals_plain_and_oracle(log_n):
    names = sorted(n for n in CASES if CASES[n][0][0] == log_n)
    specs, digests = [], []
    for n in names:
        prm, keys, cts, level, dg = _case_inputs(n)
        specs.append((cts, level, None))
        digests.append((n, dg))
    rng = np.random.default_rng(4000 + log_n)
    for k, level in EXTRA[log_n]:
        specs.append(([_random_ct(rng, prm, level) for _ in range(k)], level, None))
    print("job table N=2^%d, %d jobs" % (log_n, len(specs)), flush=True)
    outs = mick.mul_relin_rescale_jobs(prm, keys, specs)
    for (n, dg), out in zip(digests, outs):
        _check_digests(out, dg, "job-table " + n)
    for i, ((cts, level, _), out) in enumerate(zip(specs, outs)):
        plain = mick.mul_relin_rescale(prm, keys, cts, level)
        assert torch.equal(out, plain), "N=2^%d job %d (k=%d, level=%d)" % (log_n, i, len(cts), level)
    # the planned form captured into a graph and replayed twice
    plan = mick.Plan(prm, keys, specs)
    eager = [o.clone() for o in plan.run()]
    torch.cuda.synchronize()
    for o, want in zip(eager, outs):
        assert torch.equal(o, want)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.run()
    for rep in range(2):
        for o in plan.outs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, (o, want) in enumerate(zip(plan.outs, outs)):
            assert torch.equal(o, want), (rep, i)


def test_queue_over_wide_sets_equals_plain():
    n16 = _set(16, 32, 8, 4, 81, 12)
    n15 = _set(15, 16, 4, 4, 82, 12)
    sets = [n15, n16]
    rng = np.random.default_rng(4100)
    shapes = [(1, 12, 32), (0, 12, 16), (1, 2, 32), (0, 11, 13), (1, 9, 12), (0, 4, 16), (1, 12, 20), (0, 2, 5)]
    jobs = []
    for i, (st, k, level) in enumerate(shapes):
        prm = sets[st][0]
        cts = [_random_ct(rng, prm, level) for _ in range(k)]
        out = torch.empty(2, level - k + 1, prm.N, dtype=torch.int32, device="cuda")
        jobs.append((7000 + i, st, cts, level, out))
    probe = mick.Queue(sets, capacity=256)
    biggest = max(probe.job_bytes(st, k, lv) for st, k, lv in shapes)
    probe.close()
    q = mick.Queue(sets, capacity=2 * biggest)  # admission has to wait for space
    q.push(jobs)
    print("queue: %d jobs over N=2^15 and 2^16" % len(jobs), flush=True)
    q.drain()
    assert q.info() == (0, 0, 0)
    for jid, st, cts, level, out in jobs:
        prm, keys = sets[st]
        assert torch.equal(out, mick.mul_relin_rescale(prm, keys, cts, level)), jid
    q.close()
