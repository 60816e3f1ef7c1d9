"""GPU parity of the three ways the fused multiply forms d_0..d_k (a chain of
linear factors; a balanced product tree with exact-sum nodes; the same tree
with Karatsuba and 3-parallel fast-filter nodes): every method must give the
oracle's residues bit for bit, in plain, same-shape batched and job-table
launches.  k = 2..8 at N = 2^13 against the oracle directly; k = 9..12 at
N = 2^14..2^16 against the oracle digests of tests/golden/wide_k_digests.txt.
"""
import os
import zlib

import numpy as np
import pytest
import torch

from oracle import keys as okeys, mult, params as oparams
from paper_2601_15401_amd import mick
from seeded_inputs import limb_digests, uniform_cts

pytestmark = pytest.mark.gpu

METHODS = [mick.TENSOR_TREE, mick.TENSOR_FILTER]


@pytest.fixture(scope="module")
def n13():
    op = oparams.make_params(13, 8, 2, 4)
    prm = mick.Params(13, 8, 2, 4)
    return op, okeys.keygen(op, 23, 8), prm, mick.Keys(prm, 23, 8)


def _eq(got_t, want, what):
    got = mick.to_numpy_u32(got_t).astype(np.uint64)
    bad = np.argwhere(got != np.asarray(want, dtype=np.uint64))
    assert bad.size == 0, "%s: %d residues differ, first at %s" % (what, len(bad), bad[0].tolist())


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("k,level", [(2, 8), (3, 8), (4, 7), (5, 6), (6, 8), (7, 8), (8, 8), (2, 2)])
def test_tensor_method_matches_oracle(n13, method, k, level):
    op, ok, prm, gk = n13
    seed = zlib.crc32(b"tm-%d-%d" % (k, level))
    host = uniform_cts(seed, op.q[:level], op.N, k)
    dev = [mick.from_numpy_u32(c) for c in host]
    want = mult.mul_relin_rescale(op, ok, host, level)
    mick.set_tensor_method(prm, method)
    try:
        assert mick.tensor_method(prm) == method
        _eq(mick.mul_relin_rescale(prm, gk, dev, level), want, "method %d k=%d level=%d" % (method, k, level))
        out = mick.mul_relin_rescale_batch(prm, gk, torch.stack([torch.stack(dev)] * 2), level)
        _eq(out[1], want, "batched")
        outs = mick.mul_relin_rescale_jobs(prm, gk, [(dev, level, None), (dev[:2], level, None)])
        _eq(outs[0], want, "job table")
    finally:
        mick.set_tensor_method(prm, mick.TENSOR_CHAIN)


def _digest_cases():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "wide_k_digests.txt")
    cases = {}
    if os.path.exists(path):
        for line in open(path):
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            cases[p[0]] = ([int(v) for v in p[1:10]], p[10:])
    return cases


CASES = _digest_cases()
_sets = {}


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("name", sorted(CASES))
def test_tensor_method_wide_k_matches_oracle_digests(method, name):
    (log_n, L, K, dnum, ks, kmax, k, level, iseed), digests = CASES[name]
    key = (log_n, L, K, dnum, ks, kmax)
    if key not in _sets:
        prm = mick.Params(log_n, L, K, dnum)
        _sets[key] = (prm, mick.Keys(prm, ks, kmax))
    prm, keys = _sets[key]
    dev = [mick.from_numpy_u32(c) for c in uniform_cts(iseed, prm.q[:level], prm.N, k)]
    print("case", name, "method", method, flush=True)
    mick.set_tensor_method(prm, method)
    try:
        out = mick.mul_relin_rescale(prm, keys, dev, level)
        got = limb_digests(mick.to_numpy_u32(out))
        bad = [i for i, (g, w) in enumerate(zip(got, digests)) if g != w]
        assert len(got) == len(digests) and not bad, "%s method %d: %d limbs differ" % (name, method, len(bad))
    finally:
        mick.set_tensor_method(prm, mick.TENSOR_CHAIN)


def test_tensor_method_argument_checks(n13):
    _, _, prm, _ = n13
    with pytest.raises(mick.MickError):
        mick.set_tensor_method(prm, 3)
    assert mick.tensor_method(prm) == mick.TENSOR_CHAIN
