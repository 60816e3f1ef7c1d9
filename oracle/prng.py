"""Counter-based random streams and samplers (oracle side).

Test infrastructure only (see ``oracle/__init__``).

The paper draws a ternary secret of Hamming weight h, uniform polynomials
(U_q, Table I; U_PQ in the evaluation keys of Sec. V-A), Gaussian errors
N(0, sigma^2) and a ternary v of weight N/2 for encryption (Sec. II), but
fixes no generator.  Readings used on both sides of the parity check:

* Generator: the SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014)
  in counter mode.  draw(key, n) = mix64(key + (n + 1) * GAMMA mod 2^64), which
  is the n-th output of SplitMix64 started from state `key`.
* Stream key: h = mix64(seed + GAMMA); then for each word w of
  (tag, a, b, c): h = mix64((h ^ w) + GAMMA).  `tag` is an ASCII name packed
  little-endian into a u64; a, b, c are small indices (0 when unused).
* Uniform mod q: draw(key, n) mod q for coefficient n.  Uniform polynomials
  are drawn directly as NTT-domain values (uniform in either domain).
* Ternary of weight h: partial Fisher-Yates over positions 0..N-1; selection i
  takes position j = i + (draw(key, 2i) mod (N - i)), swaps it to slot i, and
  gives it sign +1 if draw(key, 2i + 1) is even, else -1.
* Gaussian: inversion of a cumulative table over x in [-B, B], B = floor(6
  sigma).  rho(x) = exp(-x^2 / (2 sigma^2)) in FP64, summed sequentially from
  x = -B; T[x] = floor(2^64 * C(x) / S) for x < B.  Sample n is the smallest x
  with draw(key, n) < T[x], else B.
* Slot values: re_j from draw 2j, im_j from draw 2j + 1, each
  2 * (u >> 11) * 2^-53 - 1, i.e. uniform in [-1, 1).
"""
from __future__ import annotations

import math
import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB


def tag(name: str) -> int:
    b = name.encode("ascii")
    assert len(b) <= 8
    return int.from_bytes(b, "little")


def mix64(z: int) -> int:
    z &= MASK
    z = ((z ^ (z >> 30)) * M1) & MASK
    z = ((z ^ (z >> 27)) * M2) & MASK
    return z ^ (z >> 31)


def stream_key(seed: int, name: str, a: int = 0, b: int = 0, c: int = 0) -> int:
    h = mix64(seed + GAMMA)
    for w in (tag(name), a, b, c):
        h = mix64(((h ^ w) + GAMMA) & MASK)
    return h


def draw(key: int, n: int) -> int:
    return mix64(key + (n + 1) * GAMMA)


def draws(key: int, count: int, start: int = 0) -> np.ndarray:
    """draw(key, n) for n in [start, start + count) as uint64 (vectorised)."""
    n = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + n * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_mod(key: int, q: int, count: int) -> np.ndarray:
    return draws(key, count) % np.uint64(q)


def ternary_hw(key: int, n: int, h: int) -> np.ndarray:
    """int64 array with exactly h entries in {+1, -1}, the rest 0."""
    d = draws(key, 2 * h)
    idx = list(range(n))
    out = np.zeros(n, dtype=np.int64)
    for i in range(h):
        j = i + int(d[2 * i]) % (n - i)
        idx[i], idx[j] = idx[j], idx[i]
        out[idx[i]] = 1 if (int(d[2 * i + 1]) & 1) == 0 else -1
    return out


def cdt_table(sigma: float):
    """(B, T) with T[x + B] for x in [-B, B): the cumulative thresholds."""
    B = int(math.floor(6.0 * sigma))
    xs = list(range(-B, B + 1))
    rho = [math.exp(-(x * x) / (2.0 * sigma * sigma)) for x in xs]
    S = 0.0
    for r in rho:
        S += r
    T = []
    c = 0.0
    for r in rho[:-1]:
        c += r
        T.append(int((c / S) * 18446744073709551616.0))
    return B, T


def gaussian(key: int, n: int, sigma: float) -> np.ndarray:
    B, T = cdt_table(sigma)
    Ta = np.array(T, dtype=np.uint64)
    u = draws(key, n)
    # count of thresholds <= u is the index of the first threshold above u
    k = np.searchsorted(Ta, u, side="right")
    return k.astype(np.int64) - B


def slots(key: int, n_slots: int):
    d = draws(key, 2 * n_slots)
    v = (d >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    v = 2.0 * v - 1.0
    return v[0::2].copy(), v[1::2].copy()
