"""GPU parity of the standalone fast basis conversion (eq. (basis
conversion)) in both forms, 64-bit multiply-adds on the vector ALUs and int8
matrix cores with exact recombination, against the oracle's conversion, bit
for bit: full digits and a truncated last digit, 30-bit q targets and 31-bit
special-prime targets, digits of 1, 2, 4 and 8 primes."""
import numpy as np
import pytest

from oracle import mult, params as oparams
from paper_2601_15401_amd import mick

pytestmark = pytest.mark.gpu

_sets = {}


def _set(log_n, L, K, dnum):
    key = (log_n, L, K, dnum)
    if key not in _sets:
        _sets[key] = (oparams.make_params(log_n, L, K, dnum), mick.Params(log_n, L, K, dnum))
    return _sets[key]


@pytest.mark.parametrize("log_n,L,K,dnum,level,digit", [
    (16, 32, 8, 4, 32, 0),   # eight-prime digit, 32 targets
    (16, 32, 8, 4, 32, 3),
    (16, 32, 8, 4, 20, 2),   # truncated last digit: 4 primes
    (15, 16, 4, 4, 16, 1),   # four-prime digits
    (14, 8, 2, 4, 7, 3),     # a single prime left in the last digit
    (13, 3, 1, 3, 3, 1),     # one prime per digit
])
@pytest.mark.parametrize("method", [mick.BCONV_VALU, mick.BCONV_MFMA])
def test_bconv_matches_oracle(log_n, L, K, dnum, level, digit, method):
    op, prm = _set(log_n, L, K, dnum)
    lo = digit * op.alpha
    src_primes = op.q[lo:min(lo + op.alpha, level)]
    dst_primes = [q for i, q in enumerate(op.q[:level]) if not lo <= i < lo + len(src_primes)] + op.p
    rng = np.random.default_rng(level * 100 + digit)
    polys = 3
    x = np.stack([np.stack([rng.integers(0, q, op.N, dtype=np.int64).astype(np.uint64) for q in src_primes])
                  for _ in range(polys)])
    out = mick.bconv(prm, mick.from_numpy_u32(x), level, digit, method)
    got = mick.to_numpy_u32(out).astype(np.uint64)
    for p in range(polys):
        want = mult.bconv(x[p], src_primes, dst_primes)
        bad = np.argwhere(got[p] != want)
        assert bad.size == 0, "method %d poly %d: %d residues differ, first at %s" % (
            method, p, len(bad), bad[0].tolist())


def test_bconv_extreme_inputs_agree():
    """Residues at 0 and q - 1 (the largest signed-byte digits) in both forms."""
    op, prm = _set(16, 32, 8, 4)
    src_primes = op.q[8:16]
    x = np.stack([np.full(op.N, q - 1, dtype=np.uint64) for q in src_primes])
    x[:, ::3] = 0
    dev = mick.from_numpy_u32(x[None])
    a = mick.to_numpy_u32(mick.bconv(prm, dev, 32, 1, mick.BCONV_VALU))
    b = mick.to_numpy_u32(mick.bconv(prm, dev, 32, 1, mick.BCONV_MFMA))
    dst_primes = op.q[:8] + op.q[16:32] + op.p
    assert np.array_equal(a[0].astype(np.uint64), mult.bconv(x, src_primes, dst_primes))
    assert np.array_equal(a, b)
