"""Negacyclic NTT over Z_q[x]/(x^N + 1) (oracle side).

Test infrastructure only (see ``oracle/__init__``).

The paper turns polynomial products into coefficient-wise products with the
NTT (Sec. I, Sec. II) but fixes no ordering.  Reading used on both sides:

    NTT(a)[k] = a(psi^(2*brv(k) + 1)) mod q,     k = 0..N-1,

with brv the log2(N)-bit reversal and psi the smallest primitive 2N-th root
of unity (oracle/params).  `ntt_direct` evaluates this definition; `ntt` is
the standard radix-2 Cooley-Tukey factorisation of the same map with merged
psi twiddles (twiddle of block b at stage s = psi^brv(2^s + b)), and `intt`
its Gentleman-Sande inverse followed by the factor N^-1.  The fast forms are
checked against the definition and against schoolbook negacyclic convolution.
"""
from __future__ import annotations

import numpy as np

from . import counts


def brv(x: int, bits: int) -> int:
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


def _brv_table(log_n: int) -> np.ndarray:
    n = 1 << log_n
    return np.array([brv(i, log_n) for i in range(n)], dtype=np.int64)


_BRV_CACHE = {}
_TW_CACHE = {}


def brv_table(log_n: int) -> np.ndarray:
    if log_n not in _BRV_CACHE:
        _BRV_CACHE[log_n] = _brv_table(log_n)
    return _BRV_CACHE[log_n]


def _powers(base: int, q: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    v = 1
    for i in range(n):
        out[i] = v
        v = v * base % q
    return out


def twiddles(q: int, psi: int, log_n: int):
    """(psi^brv(k), psi^-brv(k)) for k < N, as uint64 arrays."""
    key = (q, psi, log_n)
    if key not in _TW_CACHE:
        n = 1 << log_n
        r = brv_table(log_n)
        fw = _powers(psi, q, n)[r]
        bw = _powers(pow(psi, -1, q), q, n)[r]
        _TW_CACHE[key] = (fw, bw)
    return _TW_CACHE[key]


def _stack(qs, psis, log_n):
    fw = np.stack([twiddles(q, p, log_n)[0] for q, p in zip(qs, psis)])
    bw = np.stack([twiddles(q, p, log_n)[1] for q, p in zip(qs, psis)])
    return fw, bw


def ntt(a: np.ndarray, qs, psis) -> np.ndarray:
    """Forward NTT of each row of `a` ([limbs, N], canonical residues)."""
    a = np.array(a, dtype=np.uint64, copy=True)
    limbs, n = a.shape
    log_n = n.bit_length() - 1
    counts.add("ntt", limbs)
    fw, _ = _stack(qs, psis, log_n)
    qv = np.array(qs, dtype=np.uint64).reshape(limbs, 1, 1)
    for s in range(log_n):
        m = 1 << s
        half = n // (2 * m)
        v = a.reshape(limbs, m, 2, half)
        w = fw[:, m:2 * m].reshape(limbs, m, 1)
        x = v[:, :, 0, :].copy()
        t = (v[:, :, 1, :] * w) % qv
        v[:, :, 0, :] = (x + t) % qv
        v[:, :, 1, :] = (x + qv - t) % qv
    return a


def intt(A: np.ndarray, qs, psis) -> np.ndarray:
    """Inverse of `ntt` row by row."""
    a = np.array(A, dtype=np.uint64, copy=True)
    limbs, n = a.shape
    log_n = n.bit_length() - 1
    counts.add("intt", limbs)
    _, bw = _stack(qs, psis, log_n)
    qv = np.array(qs, dtype=np.uint64).reshape(limbs, 1, 1)
    for s in reversed(range(log_n)):
        m = 1 << s
        half = n // (2 * m)
        v = a.reshape(limbs, m, 2, half)
        w = bw[:, m:2 * m].reshape(limbs, m, 1)
        x = v[:, :, 0, :].copy()
        y = v[:, :, 1, :].copy()
        v[:, :, 0, :] = (x + y) % qv
        v[:, :, 1, :] = ((x + qv - y) % qv * w) % qv
    ninv = np.array([pow(n, -1, q) for q in qs], dtype=np.uint64).reshape(limbs, 1)
    return (a * ninv) % np.array(qs, dtype=np.uint64).reshape(limbs, 1)


def ntt_direct(a, q: int, psi: int, ks) -> list:
    """The defining sum NTT(a)[k] = sum_i a_i psi^((2 brv(k) + 1) i) mod q."""
    n = len(a)
    log_n = n.bit_length() - 1
    out = []
    coeffs = [int(x) for x in a]
    for k in ks:
        root = pow(psi, 2 * brv(k, log_n) + 1, q)
        acc = 0
        for c in reversed(coeffs):       # Horner
            acc = (acc * root + c) % q
        out.append(acc)
    return out


def negacyclic_schoolbook(a, b, q: int) -> list:
    """c = a * b mod (x^N + 1, q) by the textbook double loop (Python ints)."""
    n = len(a)
    c = [0] * n
    for i in range(n):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(n):
            k = i + j
            if k < n:
                c[k] += ai * int(b[j])
            else:
                c[k - n] -= ai * int(b[j])
    return [x % q for x in c]
