"""GPU parity at wide key-switching digits and many special primes: the
single-digit setting of the paper's evaluation (dnum = 1, K >= L; Sec. VI,
L = K = 24) and its neighbours, against the oracle, bit for bit.

The digit widths cover the ModUp kernel's wide instantiations: 16 and 24
(exact), 20 (padded to 24 rows, last chunk ragged) and 12 (two digits,
padded to 16); K = 12..24 runs the 24-prime ModDown kernel.
"""
import zlib

import numpy as np
import pytest
import torch

from oracle import ckks, keys as okeys, mult, params as oparams
from paper_2601_15401_amd import mick

pytestmark = pytest.mark.gpu

SCALE = 2.0 ** 30


def _eq(got_t, want, what):
    got = mick.to_numpy_u32(got_t).astype(np.uint64) if isinstance(got_t, torch.Tensor) else got_t.astype(np.uint64)
    want = np.asarray(want, dtype=np.uint64)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    bad = np.argwhere(got != want)
    assert bad.size == 0, "%s: %d residues differ, first at %s" % (what, len(bad), bad[0].tolist())


def _rand_ct(rng, qs, n):
    return np.stack([np.stack([rng.integers(0, q, n, dtype=np.int64).astype(np.uint64) for q in qs])
                     for _ in range(2)])


def _seed(*parts):
    return zlib.crc32("-".join(map(str, parts)).encode())


class Ctx:
    def __init__(self, log_n, L, K, dnum, seed, k_max):
        self.op = oparams.make_params(log_n, L, K, dnum)
        self.ok = okeys.keygen(self.op, seed, k_max)
        self.prm = mick.Params(log_n, L, K, dnum)
        self.gk = mick.Keys(self.prm, seed, k_max)
        self.seed = seed


SETS = {
    "L24K24d1": (13, 24, 24, 1, 21, 4),
    "L16K16d1": (13, 16, 16, 1, 22, 3),
    "L20K12d1": (13, 20, 12, 1, 23, 3),
    "L24K12d2": (13, 24, 12, 2, 24, 3),
}
_cache = {}


def ctx(name):
    if name not in _cache:
        _cache[name] = Ctx(*SETS[name])
    return _cache[name]


@pytest.mark.parametrize("name", list(SETS))
def test_params_and_keys(name):
    c = ctx(name)
    assert c.prm.q == c.op.q and c.prm.p == c.op.p and c.prm.alpha == c.op.alpha
    t = c.ok.k_max
    for b in range(c.op.dnum):
        ev = c.gk.export_evk(t, b)
        _eq(ev[0], c.ok.evk[(t, b)][0], "%s evk t=%d b=%d" % (name, t, b))


@pytest.mark.parametrize("name,k,level", [
    ("L24K24d1", 3, 24), ("L24K24d1", 2, 9), ("L24K24d1", 4, 5),
    ("L16K16d1", 3, 16), ("L20K12d1", 2, 20), ("L20K12d1", 3, 11), ("L24K12d2", 3, 24), ("L24K12d2", 2, 13),
])
def test_relin_parity(name, k, level):
    c = ctx(name)
    rng = np.random.default_rng(_seed("relin", name, k, level))
    D = np.stack([np.stack([rng.integers(0, q, c.op.N, dtype=np.int64).astype(np.uint64) for q in c.op.q[:level]])
                  for _ in range(k + 1)])
    out = mick.relin_k(c.prm, c.gk, mick.from_numpy_u32(D), k, level)
    _eq(out, np.stack(mult.relin_textbook(c.op, c.ok, D, level)), "%s relin k=%d level=%d" % (name, k, level))


@pytest.mark.parametrize("name,k,level", [
    ("L24K24d1", 3, 24), ("L24K24d1", 4, 24), ("L24K24d1", 3, 17), ("L24K24d1", 2, 2),
    ("L16K16d1", 3, 16), ("L16K16d1", 2, 7), ("L20K12d1", 3, 20), ("L24K12d2", 3, 24), ("L24K12d2", 3, 12),
])
def test_multiply_parity(name, k, level):
    c = ctx(name)
    rng = np.random.default_rng(_seed("mul", name, k, level))
    cts = [_rand_ct(rng, c.op.q[:level], c.op.N) for _ in range(k)]
    out = mick.mul_relin_rescale(c.prm, c.gk, [mick.from_numpy_u32(x) for x in cts], level)
    _eq(out, mult.mul_relin_rescale(c.op, c.ok, cts, level), "%s k=%d level=%d" % (name, k, level))


def test_unfused_composition_is_the_textbook_path():
    """mul_k, then relinearisation with its own ModDown, then the mu-level
    rescale: the oracle's textbook order (ModDown, then mu rescales)."""
    c = ctx("L24K24d1")
    rng = np.random.default_rng(31)
    level, k = 24, 3
    cts = [_rand_ct(rng, c.op.q[:level], c.op.N) for _ in range(k)]
    d = mick.mul_k(c.prm, [mick.from_numpy_u32(x) for x in cts], level)
    y = mick.relin_k(c.prm, c.gk, d, k, level)
    out = mick.rescale_multi(c.prm, y, level, k - 1)
    _eq(out, mult.mul_relin_rescale(c.op, c.ok, cts, level, path="textbook"), "unfused L=K=24")


def test_mixed_jobs_match_plain_and_oracle():
    """One job-table batch over several k and levels at L = K = 24, dnum = 1."""
    c = ctx("L24K24d1")
    rng = np.random.default_rng(32)
    shapes = [(3, 24), (2, 24), (4, 19), (3, 5), (2, 3)]
    specs, host = [], []
    for k, level in shapes:
        cts = [_rand_ct(rng, c.op.q[:level], c.op.N) for _ in range(k)]
        host.append(cts)
        specs.append(([mick.from_numpy_u32(x) for x in cts], level, None))
    outs = mick.mul_relin_rescale_jobs(c.prm, c.gk, specs)
    for (cts_d, level, _), out in zip(specs, outs):
        assert torch.equal(out, mick.mul_relin_rescale(c.prm, c.gk, cts_d, level))
    for i in (0, 2, 4):
        _eq(outs[i], mult.mul_relin_rescale(c.op, c.ok, host[i], shapes[i][1]), "job %d" % i)


def test_three_input_n16_paper_parameters():
    """The paper's three-input multiply (N = 2^16, L = K = 24, dnum = 1):
    bit for bit the oracle on encryptions, and decoding to the product of
    the three messages."""
    op = oparams.make_params(16, 24, 24, 1)
    ok = okeys.keygen(op, 41, 3)
    prm = mick.Params(16, 24, 24, 1)
    gk = mick.Keys(prm, 41, 3)
    level = 24
    cts_o, cts_g, want = [], [], np.ones(op.N // 2, dtype=np.complex128)
    for u in range(3):
        r, i, m = ckks.message(op, 41, u, SCALE)
        want = want * (r + 1j * i)
        cts_o.append(ckks.encrypt(op, ok, m, level, 41, u))
        cts_g.append(mick.encrypt(prm, gk, m, level, 41, u))
    out = mick.mul_relin_rescale(prm, gk, cts_g, level)
    _eq(out, mult.mul_relin_rescale(op, ok, cts_o, level), "N=2^16 L=K=24 k=3")
    scale_out = SCALE ** 3 / (op.q[22] * op.q[23])
    re, im = mick.decode(prm, mick.decrypt(prm, gk, out, 22), scale_out)
    # the fresh public-key encryption noise dominates: about sigma sqrt(2N/3)
    # per coefficient, sqrt(N) times that in a slot, over Delta = 2^30, i.e.
    # ~2e-4 per slot before the other factors multiply it (max ~1.3e-3 seen)
    err = np.abs((re + 1j * im) - want)
    assert err.max() < 1e-2, err.max()
