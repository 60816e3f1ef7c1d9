"""GPU parity of the tensor product fused with pass B of the INTT of
d_2..d_k (the fused multiply's first kernel): pass-B blocks of 64 (N = 2^13),
128 (N = 2^14, 2^15) and 256 rows (N = 2^16), k from 5 to 12 (1024-residue
tiles; k <= 4 takes larger tiles and runs in every other multiply test),
plain and batched launches, against the oracle bit for bit.  The unfused
composition (plain tensor kernel, both INTT passes) runs on the same inputs
against the oracle's textbook path.
"""
import zlib

import numpy as np
import pytest
import torch

from oracle import keys as okeys, mult, params as oparams
from paper_2601_15401_amd import mick

pytestmark = pytest.mark.gpu

_cache = {}


def ctx(log_n, k_max):
    key = (log_n, k_max)
    if key not in _cache:
        op = oparams.preset(log_n)
        seed = 70 + log_n
        prm = mick.Params(log_n, op.L, op.K, op.dnum)
        _cache[key] = (op, okeys.keygen(op, seed, k_max), prm, mick.Keys(prm, seed, k_max))
    return _cache[key]


def _rand_ct(rng, qs, n):
    return np.stack([np.stack([rng.integers(0, q, n, dtype=np.int64).astype(np.uint64) for q in qs])
                     for _ in range(2)])


def _eq(got_t, want, what):
    got = mick.to_numpy_u32(got_t).astype(np.uint64)
    want = np.asarray(want, dtype=np.uint64)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    bad = np.argwhere(got != want)
    assert bad.size == 0, "%s: %d residues differ, first at %s" % (what, len(bad), bad[0].tolist())


@pytest.mark.parametrize("log_n,k,level", [
    (14, 5, 8), (14, 6, 7), (15, 5, 16), (15, 7, 11), (16, 5, 9), (16, 8, 10),
])
def test_fused_multiply_parity(log_n, k, level):
    op, ok, prm, gk = ctx(log_n, 8)
    rng = np.random.default_rng(zlib.crc32(b"tib-%d-%d-%d" % (log_n, k, level)))
    cts = [_rand_ct(rng, op.q[:level], op.N) for _ in range(k)]
    dev = [mick.from_numpy_u32(x) for x in cts]
    out = mick.mul_relin_rescale(prm, gk, dev, level)
    _eq(out, mult.mul_relin_rescale(op, ok, cts, level), "N=2^%d k=%d level=%d" % (log_n, k, level))
    # the unfused composition (plain tensor kernel, both INTT passes, the
    # textbook order) on the same inputs
    d = mick.mul_k(prm, dev, level)
    y = mick.relin_k(prm, gk, d, k, level)
    _eq(mick.rescale_multi(prm, y, level, k - 1), mult.mul_relin_rescale(op, ok, cts, level, path="textbook"),
        "unfused N=2^%d k=%d level=%d" % (log_n, k, level))


@pytest.mark.parametrize("log_n,k,level,jobs", [(14, 6, 8, 3), (16, 5, 6, 2)])
def test_fused_batch_matches_plain(log_n, k, level, jobs):
    op, ok, prm, gk = ctx(log_n, 8)
    rng = np.random.default_rng(zlib.crc32(b"tib-batch-%d-%d" % (log_n, k)))
    host = [[_rand_ct(rng, op.q[:level], op.N) for _ in range(k)] for _ in range(jobs)]
    batch = torch.stack([torch.stack([mick.from_numpy_u32(x) for x in h]) for h in host])
    out = mick.mul_relin_rescale_batch(prm, gk, batch, level)
    for j in range(jobs):
        assert torch.equal(out[j], mick.mul_relin_rescale(prm, gk, [batch[j, u] for u in range(k)], level)), j
    _eq(out[0], mult.mul_relin_rescale(op, ok, host[0], level), "batched job 0")


_wide = {}


@pytest.mark.parametrize("log_n,L,K,dnum,k,level", [
    (13, 12, 3, 3, 12, 12),  # 64-row pass-B blocks, eleven d_t tiles in LDS
    (13, 12, 3, 3, 9, 10),
    (14, 12, 2, 4, 10, 11),  # 128-row blocks
])
def test_fused_wide_k_parity(log_n, L, K, dnum, k, level):
    key = (log_n, L, K, dnum)
    if key not in _wide:
        op = oparams.make_params(log_n, L, K, dnum)
        prm = mick.Params(log_n, L, K, dnum)
        _wide[key] = (op, okeys.keygen(op, 90 + log_n, 12), prm, mick.Keys(prm, 90 + log_n, 12))
    op, ok, prm, gk = _wide[key]
    rng = np.random.default_rng(zlib.crc32(b"tib-wide-%d-%d-%d" % (log_n, k, level)))
    cts = [_rand_ct(rng, op.q[:level], op.N) for _ in range(k)]
    out = mick.mul_relin_rescale(prm, gk, [mick.from_numpy_u32(x) for x in cts], level)
    _eq(out, mult.mul_relin_rescale(op, ok, cts, level), "N=2^%d k=%d level=%d" % (log_n, k, level))


def test_profiled_sites_of_the_fused_multiply():
    """The launch sites bench.py prices: the fused tensor kernel reports as
    tensor_inttB, the INTT of d_2..d_k as its pass A only; a selection keeps
    the other sites out."""
    op, ok, prm, gk = ctx(14, 8)
    rng = np.random.default_rng(5)
    k, level = 3, 8
    dev = [mick.from_numpy_u32(_rand_ct(rng, op.q[:level], op.N)) for _ in range(k)]
    mick.mul_relin_rescale(prm, gk, dev, level)  # warm
    torch.cuda.synchronize()
    mick.profile_enable(True)
    try:
        mick.profile_collect()
        mick.mul_relin_rescale(prm, gk, dev, level)
        sites = mick.profile_collect()
        mick.profile_select(["tensor_inttB"])
        mick.mul_relin_rescale(prm, gk, dev, level)
        only = mick.profile_collect()
    finally:
        mick.profile_select(None)
        mick.profile_enable(False)
    for s in ("tensor_inttB", "intt_d.passA", "modup_bconv_passA", "passB_kip", "intt_acc.passA",
              "moddown_rescale", "ntt_out.passA", "ntt_out.passB"):
        assert s in sites and sites[s][1] == 1, (s, sites)
    assert "tensor" not in sites and "intt_d.passB" not in sites, sites
    assert set(only) == {"tensor_inttB"}, only
