"""RNS parameters: primes, negacyclic roots and digit structure (oracle side).

Test infrastructure only (see ``oracle/__init__``).

Follows Sec. II (RNS decomposition of Q into pairwise co-prime q_j, the key
switching modulus P = prod p_i) with these readings where the paper is silent:

* q_i is the (i+1)-th largest prime below 2^30 with q = 1 (mod 2N); p_i the
  same rule below 2^31.  q_0 is the largest, so rescaling drops the smallest
  remaining primes first (Sec. II, eq. (1-rs) drops q_{L-1}).
* psi_q is the smallest x in [2, q) with x^N = -1 (mod q).
* Hybrid key switching with dnum digits: alpha = ceil(L / dnum) primes per
  digit; digit b holds q_{b*alpha} .. q_{min((b+1)*alpha, level)-1} at a level.
  With dnum = 1 and K >= L this is the single-digit form of Sec. II.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

# Deterministic Miller-Rabin: these bases are exact for all n < 3.3e24.
_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def primes_below(bits: int, two_n: int, count: int) -> List[int]:
    """The `count` largest primes p < 2^bits with p = 1 (mod two_n), descending."""
    out = []
    x = ((2 ** bits - 2) // two_n) * two_n + 1
    while len(out) < count:
        if x < two_n:
            raise ValueError("not enough NTT-friendly primes")
        if is_prime(x):
            out.append(x)
        x -= two_n
    return out


def min_psi(q: int, n: int) -> int:
    """Smallest x >= 2 with x^n = -1 (mod q): a primitive 2n-th root of unity.

    The solutions of x^n = -1 are exactly the odd powers psi0^(2i+1), i < n,
    of any one of them, so the smallest is found among those n values (a
    linear search from 2 would take ~q/n steps for small n)."""
    if (q - 1) % (2 * n):
        raise ValueError("q is not 1 mod 2n")
    e = (q - 1) // (2 * n)
    g = 2
    while pow(pow(g, e, q), n, q) != q - 1:
        g += 1
    psi0 = pow(g, e, q)
    sq = psi0 * psi0 % q
    best, x = q, psi0
    for _ in range(n):
        best = min(best, x)
        x = x * sq % q
    return best


@dataclass
class Params:
    log_n: int
    L: int
    K: int
    dnum: int
    q: List[int] = field(default_factory=list)
    p: List[int] = field(default_factory=list)
    psi_q: List[int] = field(default_factory=list)
    psi_p: List[int] = field(default_factory=list)
    h: int = 64          # Hamming weight of s
    sigma: float = 3.2   # error standard deviation

    @property
    def N(self) -> int:
        return 1 << self.log_n

    @property
    def alpha(self) -> int:
        return -(-self.L // self.dnum)

    @property
    def P(self) -> int:
        out = 1
        for x in self.p:
            out *= x
        return out

    def Q(self, level: int) -> int:
        out = 1
        for x in self.q[:level]:
            out *= x
        return out

    def digits(self, level: int) -> List[List[int]]:
        """Active q-limb indices of each digit at `level` (hybrid key switching)."""
        a = self.alpha
        out = []
        for b in range(self.dnum):
            lo, hi = b * a, min((b + 1) * a, level)
            if lo < hi:
                out.append(list(range(lo, hi)))
        return out

    def ext_moduli(self, level: int) -> List[int]:
        """Moduli of the extended basis Q_level * P: q_0..q_{level-1}, p_0..p_{K-1}."""
        return list(self.q[:level]) + list(self.p)

    def ext_psi(self, level: int) -> List[int]:
        return list(self.psi_q[:level]) + list(self.psi_p)


def make_params(log_n: int, L: int, K: int, dnum: int, h: int = 64, sigma: float = 3.2) -> Params:
    n = 1 << log_n
    q = primes_below(30, 2 * n, L)
    p = primes_below(31, 2 * n, K)
    prm = Params(log_n=log_n, L=L, K=K, dnum=dnum, q=q, p=p, h=h, sigma=sigma)
    prm.psi_q = [min_psi(x, n) for x in q]
    prm.psi_p = [min_psi(x, n) for x in p]
    return prm


# The parameter sets of the workloads (N, L, K, dnum).  N = 2^14 has no stated
# prime counts; L = 8, K = 2, dnum = 4 interpolates the 2^13 and 2^15 sets.
PRESETS = {
    13: (3, 1, 3),
    14: (8, 2, 4),
    15: (16, 4, 4),
    16: (32, 8, 4),
}


def preset(log_n: int) -> Params:
    L, K, dnum = PRESETS[log_n]
    return make_params(log_n, L, K, dnum)
