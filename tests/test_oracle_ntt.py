"""Pins for the oracle's negacyclic NTT (CPU only).

The NTT is pinned to its definition (direct evaluation at the roots
psi^(2 brv(k) + 1)), to schoolbook negacyclic convolution, and to the
inverse property at every workload shape.
"""
import numpy as np
import pytest

from oracle import ntt, params, prng


def _rand_limbs(moduli, n, seed):
    return np.stack([prng.uniform_mod(prng.stream_key(seed, "TEST", i), q, n) for i, q in enumerate(moduli)])


@pytest.mark.parametrize("log_n", [1, 2, 3, 5, 8])
def test_ntt_matches_definition_small(log_n):
    n = 1 << log_n
    qs = params.primes_below(30, 2 * n, 2) + params.primes_below(31, 2 * n, 1)
    psis = [params.min_psi(q, n) for q in qs]
    a = _rand_limbs(qs, n, 1)
    A = ntt.ntt(a, qs, psis)
    for i, (q, psi) in enumerate(zip(qs, psis)):
        assert [int(x) for x in A[i]] == ntt.ntt_direct(a[i], q, psi, range(n))


@pytest.mark.parametrize("log_n", [13, 16])
def test_ntt_matches_definition_sampled(log_n):
    prm = params.preset(log_n)
    qs = [prm.q[0], prm.q[-1], prm.p[-1]]
    psis = [prm.psi_q[0], prm.psi_q[-1], prm.psi_p[-1]]
    a = _rand_limbs(qs, prm.N, 2)
    A = ntt.ntt(a, qs, psis)
    rng = np.random.default_rng(5)
    ks = [0, 1, prm.N - 1] + rng.integers(0, prm.N, 5).tolist()
    for i, (q, psi) in enumerate(zip(qs, psis)):
        assert [int(A[i][k]) for k in ks] == ntt.ntt_direct(a[i], q, psi, ks)


@pytest.mark.parametrize("log_n", [2, 4, 6, 9, 10])
def test_ntt_convolution_matches_schoolbook(log_n):
    n = 1 << log_n
    qs = params.primes_below(30, 2 * n, 1) + params.primes_below(31, 2 * n, 1)
    psis = [params.min_psi(q, n) for q in qs]
    a = _rand_limbs(qs, n, 3)
    b = _rand_limbs(qs, n, 4)
    qc = np.array(qs, dtype=np.uint64).reshape(-1, 1)
    c = ntt.intt((ntt.ntt(a, qs, psis) * ntt.ntt(b, qs, psis)) % qc, qs, psis)
    for i, q in enumerate(qs):
        assert [int(x) for x in c[i]] == ntt.negacyclic_schoolbook(a[i], b[i], q)


def test_negacyclic_wrap_sign():
    # x^(N-1) * x = x^N = -1 in Z_q[x]/(x^N + 1)
    n, q = 8, 17
    a = [0] * n
    a[n - 1] = 1
    b = [0] * n
    b[1] = 1
    assert ntt.negacyclic_schoolbook(a, b, q) == [q - 1] + [0] * (n - 1)


@pytest.mark.parametrize("log_n", [13, 14, 15, 16])
def test_intt_inverts_ntt_at_workload_shapes(log_n):
    prm = params.preset(log_n)
    qs = prm.q + prm.p
    psis = prm.psi_q + prm.psi_p
    a = _rand_limbs(qs, prm.N, 6)
    A = ntt.ntt(a, qs, psis)
    assert np.array_equal(ntt.intt(A, qs, psis), a)
    assert np.array_equal(ntt.ntt(ntt.intt(a, qs, psis), qs, psis), a)


def test_ntt_of_constant_and_monomial():
    # NTT(1) is all ones; NTT(x)[k] = psi^(2 brv(k) + 1)
    log_n = 5
    n = 1 << log_n
    q = params.primes_below(30, 2 * n, 1)[0]
    psi = params.min_psi(q, n)
    one = np.zeros((1, n), dtype=np.uint64)
    one[0, 0] = 1
    assert np.all(ntt.ntt(one, [q], [psi]) == 1)
    x = np.zeros((1, n), dtype=np.uint64)
    x[0, 1] = 1
    X = ntt.ntt(x, [q], [psi])[0]
    for k in range(n):
        assert int(X[k]) == pow(psi, 2 * ntt.brv(k, log_n) + 1, q)
