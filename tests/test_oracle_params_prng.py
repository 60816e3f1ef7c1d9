"""Pins for the oracle's primes, roots and random streams (CPU only)."""
import math

import numpy as np
import pytest

from oracle import params, prng

pytestmark = pytest.mark.filterwarnings("ignore")


def _small_primes(limit):
    sieve = np.ones(limit + 1, dtype=bool)
    sieve[:2] = False
    for i in range(2, int(limit ** 0.5) + 1):
        if sieve[i]:
            sieve[i * i::i] = False
    return np.nonzero(sieve)[0]


_SP = _small_primes(1 << 16)


def trial_division_prime(n: int) -> bool:
    """Primality by trial division (independent of the Miller-Rabin test)."""
    if n < 2:
        return False
    r = math.isqrt(n)
    ps = _SP[_SP <= r]
    return not np.any(n % ps == 0) or n in set(ps.tolist())


@pytest.mark.parametrize("bits,log_n,count", [(30, 4, 6), (31, 5, 4), (20, 3, 8)])
def test_primes_are_the_largest_by_brute_force(bits, log_n, count):
    two_n = 2 << log_n
    got = params.primes_below(bits, two_n, count)
    want = []
    x = (1 << bits) - 1
    while len(want) < count:
        if x % two_n == 1 and trial_division_prime(x):
            want.append(x)
        x -= 1
    assert got == want


@pytest.mark.parametrize("log_n", [13, 16])
def test_preset_primes(log_n):
    prm = params.preset(log_n)
    n2 = 2 * prm.N
    for plist, bits in ((prm.q, 30), (prm.p, 31)):
        assert plist == sorted(plist, reverse=True)
        assert plist[0] < (1 << bits)
        for a, b in zip([(1 << bits) - 1] + plist[:-1], plist):
            assert b % n2 == 1 and trial_division_prime(b)
            # nothing prime and NTT-friendly strictly between consecutive picks
            x = b + n2
            while x < a:
                assert not trial_division_prime(x)
                x += n2
    assert set(prm.q).isdisjoint(prm.p)


@pytest.mark.parametrize("log_n", [3, 4, 13])
def test_psi_is_smallest_primitive_root(log_n):
    n = 1 << log_n
    qs = params.primes_below(30, 2 * n, 2) if log_n > 4 else params.primes_below(12, 2 * n, 2)
    for q in qs:
        psi = params.min_psi(q, n)
        assert pow(psi, n, q) == q - 1 and pow(psi, 2 * n, q) == 1
        # order exactly 2n: psi^(2n/r) != 1 for the only prime factor r = 2
        assert pow(psi, n, q) != 1
        for x in range(2, psi):
            assert pow(x, n, q) != q - 1


def test_preset_psi_orders():
    for ln in (13, 14, 15, 16):
        prm = params.preset(ln)
        for q, psi in zip(prm.q + prm.p, prm.psi_q + prm.psi_p):
            assert pow(psi, prm.N, q) == q - 1


def test_digits():
    prm = params.preset(16)
    assert prm.alpha == 8
    assert prm.digits(32) == [list(range(0, 8)), list(range(8, 16)), list(range(16, 24)), list(range(24, 32))]
    assert prm.digits(20) == [list(range(0, 8)), list(range(8, 16)), list(range(16, 20))]
    c1 = params.preset(13)
    assert c1.alpha == 1 and c1.digits(3) == [[0], [1], [2]]
    assert len(c1.digits(2)) == 2


def test_splitmix64_known_answers():
    # The first outputs of SplitMix64 started from state 0 (published sequence).
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [prng.draw(0, n) for n in range(3)] == want
    assert [int(v) for v in prng.draws(0, 3)] == want


# Known-answer vectors for the sampler conventions written in the library
# header (stream keys, ternary selection, slot values), worked by hand from
# that text and the published SplitMix64 outputs of state 0:
#   s_1..s_8 = e220a8397b1dcdaf 6e789e6aa1b965f4 06c45d188009454f
#              f88bb8a8724c81ec 1b39896a51a8749b 53cb9f0c747ea2ea
#              2c829abe1f4532e1 c584133ac916ab3c
# (s_n = mix64(n G), G = 0x9E3779B97F4A7C15), so that a misreading shared by
# the oracle and the library's host samplers fails here.
PUB = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC,
       0x1B39896A51A8749B, 0x53CB9F0C747EA2EA, 0x2C829ABE1F4532E1, 0xC584133AC916AB3C]


def test_splitmix64_published_sequence():
    assert [prng.draw(0, n) for n in range(8)] == PUB


def test_stream_key_chain_known_answer():
    """h = mix64(seed + G), then h = mix64((h ^ w) + G) for w = tag, a, b, c.
    With seed = -G the first step is mix64(0) = 0; the empty tag packs to 0,
    so the second step is mix64(G) = s_1; a = s_1 ^ G makes the third
    mix64(2G) = s_2, b = s_2 ^ 2G the fourth s_3, c = s_3 ^ 3G the last s_4.
    Any other order of the words, an add in place of the xor, or a missing
    seed offset breaks the chain."""
    G, M = prng.GAMMA, (1 << 64) - 1
    a = PUB[0] ^ G
    b = PUB[1] ^ ((2 * G) & M)
    c = PUB[2] ^ ((3 * G) & M)
    assert (a, b, c) == (0x7C17D1800457B1BA, 0x52166D185F2D9DDE, 0xDC623034FDD63170)
    assert prng.stream_key((-G) & M, "", a, b, c) == PUB[3]
    # the tag's ASCII bytes little-endian: "SK" = 0x53 'S', 0x4B 'K'
    assert prng.tag("SK") == 0x4B53 and prng.tag("EVK_A") == 0x415F4B5645
    # a non-empty tag: h after the tag step is mix64(0x4B53 + G); a = h ^ G
    # steers the next step onto 2G, and the chain again ends on s_4
    h_tag = prng.mix64(0x4B53 + G)
    assert prng.stream_key((-G) & M, "SK", h_tag ^ G, b, c) == PUB[3]


def test_ternary_selection_known_answer():
    """Partial Fisher-Yates of the header: step i takes j = i + draw(2i) mod
    (N - i), swaps positions i and j, sign + iff draw(2i + 1) is even.
    Key 0 (draw n = s_{n+1}), N = 4, h = 2:
      i = 0: s_1 = ..af, 0xaf mod 4 = 3, j = 3, order [3,1,2,0]; s_2 = ..f4
             even: position 3 gets +1;
      i = 1: s_3 mod 3 = (hex digit sum 94) mod 3 = 1, j = 2, order
             [3,2,1,0]; s_4 = ..ec even: position 2 gets +1.
    h = 3 adds i = 2: s_5 = ..9b odd, mod 2 = 1, j = 3, order [3,2,0,1];
      s_6 = ..ea even: position 0 gets +1.
    Key G (draw n = s_{n+2}), N = 4, h = 2:
      i = 0: s_2 = ..f4, mod 4 = 0, j = 0; s_3 = ..4f odd: position 0 gets -1;
      i = 1: s_4 mod 3 = (hex digit sum 139) mod 3 = 1, j = 2, order
             [0,2,1,3]; s_5 = ..9b odd: position 2 gets -1."""
    assert prng.ternary_hw(0, 4, 2).tolist() == [0, 0, 1, 1]
    assert prng.ternary_hw(0, 4, 3).tolist() == [1, 0, 1, 1]
    assert prng.ternary_hw(prng.GAMMA, 4, 2).tolist() == [-1, 0, -1, 0]


def test_slot_values_known_answer():
    """re_j from draw 2j, im_j from draw 2j + 1, each 2 (u >> 11) 2^-53 - 1.
    Key 0: s_1 >> 11 = 0x1c4415072f63b9, doubled 0x38882a0e5ec772, minus 2^53
    = 0x18882a0e5ec772, i.e. re_0 = 0x1.8882a0e5ec772p-1;
    s_2 >> 11 = 0xdcf13cd54372c, doubled 0x1b9e279aa86e58, minus 2^53 =
    -0x461d8655791a8, i.e. im_0 = -0x1.18761955e46a0p-3."""
    re, im = prng.slots(0, 2)
    assert re[0] == float.fromhex("0x1.8882a0e5ec772p-1")
    assert im[0] == float.fromhex("-0x1.18761955e46a0p-3")
    assert (PUB[2] >> 11) * 2 - (1 << 53) == int(re[1] * 2.0 ** 53)
    assert (PUB[3] >> 11) * 2 - (1 << 53) == int(im[1] * 2.0 ** 53)


def test_stream_keys_distinct_and_deterministic():
    ks = {prng.stream_key(1, "EVK_A", t, b, i) for t in range(2, 5) for b in range(4) for i in range(8)}
    assert len(ks) == 3 * 4 * 8
    assert prng.stream_key(7, "SK") == prng.stream_key(7, "SK")
    assert prng.stream_key(7, "SK") != prng.stream_key(8, "SK")


def test_ternary_weight():
    s = prng.ternary_hw(prng.stream_key(3, "SK"), 1 << 13, 64)
    assert np.count_nonzero(s) == 64 and set(np.unique(s)) <= {-1, 0, 1}
    v = prng.ternary_hw(prng.stream_key(3, "ENC_V", 5), 1 << 10, 512)
    assert np.count_nonzero(v) == 512
    assert abs(int(v.sum())) < 120


def test_gaussian_moments_and_range():
    sigma = 3.2
    x = prng.gaussian(prng.stream_key(11, "PK_E"), 1 << 18, sigma)
    assert x.min() >= -19 and x.max() <= 19
    n = x.size
    assert abs(x.mean()) < 5 * sigma / math.sqrt(n)
    assert abs(x.var() / sigma ** 2 - 1.0) < 0.03
    # the tail mass beyond 3 sigma matches the discrete Gaussian within noise
    B, T = prng.cdt_table(sigma)
    assert B == 19 and all(a < b for a, b in zip(T, T[1:]))
    # symmetry of the table: T[x] + T[-x-1] = 2^64 up to FP64 rounding
    for x in range(0, B):
        lo = T[B - x - 1]
        hi = T[B + x] if x < B else 1 << 64
        assert abs(lo + hi - (1 << 64)) < (1 << 13)


def test_slots_range():
    re, im = prng.slots(prng.stream_key(1, "MSG", 0), 4096)
    assert re.min() >= -1 and re.max() < 1 and im.min() >= -1 and im.max() < 1
    assert abs(re.mean()) < 0.05 and abs(im.mean()) < 0.05


def test_uniform_range():
    q = params.preset(13).q[0]
    u = prng.uniform_mod(prng.stream_key(1, "PK_A", 0), q, 1 << 15)
    assert u.max() < q and abs(float(u.mean()) / q - 0.5) < 0.01
