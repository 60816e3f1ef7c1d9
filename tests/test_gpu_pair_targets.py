"""GPU parity of the two-target ModUp kernels (digits of 5 to 8 primes):
target pairs that straddle the digit's own limbs, an odd number of q
targets or of special primes (a pair with one member), ragged last digits
and digits padded to eight rows, through the plain, batched and job-table
launches, against the oracle bit for bit.
"""
import zlib

import numpy as np
import pytest
import torch

from oracle import keys as okeys, mult, params as oparams
from paper_2601_15401_amd import mick

pytestmark = pytest.mark.gpu

# (log_n, L, K, dnum, seed, k_max): digit widths 7 (L=14, dnum=2), 5 (L=10,
# dnum=2) and 8 (L=16, dnum=2; L=8, dnum=1); K odd and even, down to 1
SETS = {
    "L14K3d2": (13, 14, 3, 2, 51, 4),
    "L10K5d2": (13, 10, 5, 2, 52, 3),
    "L16K2d2": (13, 16, 2, 2, 53, 3),
    "L8K1d1": (13, 8, 1, 1, 54, 3),
}
_cache = {}


class Ctx:
    def __init__(self, log_n, L, K, dnum, seed, k_max):
        self.op = oparams.make_params(log_n, L, K, dnum)
        self.ok = okeys.keygen(self.op, seed, k_max)
        self.prm = mick.Params(log_n, L, K, dnum)
        self.gk = mick.Keys(self.prm, seed, k_max)


def ctx(name):
    if name not in _cache:
        _cache[name] = Ctx(*SETS[name])
    return _cache[name]


def _eq(got_t, want, what):
    got = mick.to_numpy_u32(got_t).astype(np.uint64)
    want = np.asarray(want, dtype=np.uint64)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    bad = np.argwhere(got != want)
    assert bad.size == 0, "%s: %d residues differ, first at %s" % (what, len(bad), bad[0].tolist())


def _rand_ct(rng, qs, n):
    return np.stack([np.stack([rng.integers(0, q, n, dtype=np.int64).astype(np.uint64) for q in qs])
                     for _ in range(2)])


def _seed(*parts):
    return zlib.crc32("-".join(map(str, parts)).encode())


def test_sets_take_the_two_target_kernel():
    for name, (log_n, L, K, dnum, _, _) in SETS.items():
        alpha = oparams.make_params(log_n, L, K, dnum).alpha
        assert 5 <= alpha <= 8, name


@pytest.mark.parametrize("name,k,level", [
    ("L14K3d2", 3, 14),   # two digits of 7: 7 q targets each (odd), K = 3 (odd)
    ("L14K3d2", 4, 11),   # ragged last digit (4 primes): 7 and 4 q targets
    ("L14K3d2", 2, 8),    # the first digit's own limbs split the q targets 0 | 7
    ("L10K5d2", 3, 10),   # digits of 5, padded to eight rows
    ("L10K5d2", 2, 6),    # ragged: 5 and 1 primes
    ("L16K2d2", 3, 16),   # digits of 8, even counts
    ("L16K2d2", 2, 9),
    ("L16K2d2", 2, 2),    # one digit holds every active q limb: no q targets
    ("L14K3d2", 2, 3),    # no q targets, three special primes (one alone)
    ("L8K1d1", 3, 8),     # a single special prime: its pair has one member
    ("L8K1d1", 2, 5),
])
def test_multiply_parity(name, k, level):
    c = ctx(name)
    rng = np.random.default_rng(_seed("pair", name, k, level))
    cts = [_rand_ct(rng, c.op.q[:level], c.op.N) for _ in range(k)]
    out = mick.mul_relin_rescale(c.prm, c.gk, [mick.from_numpy_u32(x) for x in cts], level)
    _eq(out, mult.mul_relin_rescale(c.op, c.ok, cts, level), "%s k=%d level=%d" % (name, k, level))


def test_relin_parity():
    c = ctx("L14K3d2")
    rng = np.random.default_rng(_seed("pair-relin"))
    k, level = 4, 13
    D = np.stack([np.stack([rng.integers(0, q, c.op.N, dtype=np.int64).astype(np.uint64) for q in c.op.q[:level]])
                  for _ in range(k + 1)])
    out = mick.relin_k(c.prm, c.gk, mick.from_numpy_u32(D), k, level)
    _eq(out, np.stack(mult.relin_textbook(c.op, c.ok, D, level)), "relin k=%d level=%d" % (k, level))


def test_batched_and_job_table_match_plain():
    """Same-shape batch and a job table mixing k and level: every job equals
    its plain multiply; two jobs are checked against the oracle."""
    c = ctx("L14K3d2")
    rng = np.random.default_rng(_seed("pair-batch"))
    k, level, jobs = 3, 12, 3
    host = [[_rand_ct(rng, c.op.q[:level], c.op.N) for _ in range(k)] for _ in range(jobs)]
    batch = torch.stack([torch.stack([mick.from_numpy_u32(x) for x in h]) for h in host])
    out = mick.mul_relin_rescale_batch(c.prm, c.gk, batch, level)
    for j in range(jobs):
        assert torch.equal(out[j], mick.mul_relin_rescale(c.prm, c.gk, [batch[j, u] for u in range(k)], level)), j
    _eq(out[jobs - 1], mult.mul_relin_rescale(c.op, c.ok, host[jobs - 1], level), "batched job %d" % (jobs - 1))
    shapes = [(4, 14), (2, 9), (3, 7), (2, 2)]
    specs, hs = [], []
    for kk, lv in shapes:
        cts = [_rand_ct(rng, c.op.q[:lv], c.op.N) for _ in range(kk)]
        hs.append(cts)
        specs.append(([mick.from_numpy_u32(x) for x in cts], lv, None))
    outs = mick.mul_relin_rescale_jobs(c.prm, c.gk, specs)
    for (cts_d, lv, _), o in zip(specs, outs):
        assert torch.equal(o, mick.mul_relin_rescale(c.prm, c.gk, cts_d, lv)), lv
    _eq(outs[1], mult.mul_relin_rescale(c.op, c.ok, hs[1], shapes[1][1]), "job table job 1")
