"""Pins for the oracle's keys, encryption, tensor product, basis conversion,
relinearisation and rescaling (CPU only).

Each check is against something other than the oracle itself: big-integer
arithmetic in Z[x]/(x^N + 1) written out here, the Chinese remainder theorem,
closed forms (the rescale of an integer is a floor division), stated noise
bounds derived from the scheme, and the operation counts the paper tabulates.
"""
import math

import numpy as np
import pytest

from oracle import ckks, counts, keys, mult, ntt, params, prng


# ------------------------------------------------------------------ helpers

def polymul_neg(a, b):
    """Negacyclic product of integer polynomials (Python ints, schoolbook)."""
    n = len(a)
    c = [0] * n
    for i, ai in enumerate(a):
        if ai == 0:
            continue
        for j, bj in enumerate(b):
            if i + j < n:
                c[i + j] += ai * bj
            else:
                c[i + j - n] -= ai * bj
    return c


def centered_crt(res_rows, moduli):
    """Centred integers from residue rows, by solving the CRT incrementally."""
    n = len(res_rows[0])
    out = []
    for i in range(n):
        x, M = 0, 1
        for r, m in zip(res_rows, moduli):
            # find x' = x (mod M), x' = r (mod m)
            t = ((int(r[i]) - x) * pow(M, -1, m)) % m
            x += M * t
            M *= m
        out.append(x - M if x > M // 2 else x)
    return out


def coeff_residues(prm, A, moduli, psis):
    return ntt.intt(np.asarray(A, dtype=np.uint64), moduli, psis)


def mk(log_n, L, K, dnum):
    """Small parameter sets; the secret weight is capped at N/4 so that it fits."""
    return params.make_params(log_n, L, K, dnum, h=min(64, (1 << log_n) // 4))


def tiny(log_n=5, L=6, K=2, dnum=3):
    return mk(log_n, L, K, dnum)


# ------------------------------------------------------------------ keys

def test_public_key_relation():
    prm = tiny()
    ks = keys.keygen(prm, 11, 3)
    b = centered_crt(coeff_residues(prm, ks.pk_b, prm.q, prm.psi_q), prm.q)
    a = centered_crt(coeff_residues(prm, ks.pk_a, prm.q, prm.psi_q), prm.q)
    s = [int(x) for x in ks.s]
    Q = prm.Q(prm.L)
    lhs = [(x + y) % Q for x, y in zip(b, polymul_neg(a, s))]
    assert lhs == [int(e) % Q for e in ks.pk_e]


@pytest.mark.parametrize("dnum", [1, 3])
def test_evaluation_key_relation(dnum):
    """ek_{t,b,0} + ek_{t,b,1} s = e_{t,b} + P G_b s^t, where G_b is the CRT
    idempotent of digit b (1 mod its primes, 0 mod the other q and the p)."""
    prm = tiny(L=6, K=6 if dnum == 1 else 2, dnum=dnum)
    ks = keys.keygen(prm, 12, 4)
    s = [int(x) for x in ks.s]
    moduli = prm.q + prm.p
    psis = prm.psi_q + prm.psi_p
    st = {1: s}
    for t in range(2, 5):
        st[t] = polymul_neg(st[t - 1], s)
    for t in range(2, 5):
        for b in range(prm.dnum):
            k0, k1 = ks.evk[(t, b)]
            c0 = coeff_residues(prm, k0, moduli, psis)
            c1 = coeff_residues(prm, k1, moduli, psis)
            e = [int(x) for x in ks.evk_e[(t, b)]]
            digit = set(prm.digits(prm.L)[b])
            for row, m in enumerate(moduli):
                k1s = polymul_neg([int(x) for x in c1[row]], s)
                got = [(int(x) + y) % m for x, y in zip(c0[row], k1s)]
                in_digit = row < prm.L and row in digit
                want = [(ei + (prm.P * sti if in_digit else 0)) % m for ei, sti in zip(e, st[t])]
                assert got == want, (t, b, row)


def test_secret_and_noise_shapes():
    prm = params.preset(13)
    ks = keys.keygen(prm, 1, 3)
    assert np.count_nonzero(ks.s) == 64
    assert np.abs(ks.pk_e).max() <= 19
    for e in ks.evk_e.values():
        assert np.abs(e).max() <= 19
    # every key residue is canonical
    for k0, k1 in ks.evk.values():
        mc = np.array(prm.q + prm.p, dtype=np.uint32).reshape(-1, 1)
        assert np.all(k0 < mc) and np.all(k1 < mc)


# ------------------------------------------------------------------ encryption

def test_fresh_ciphertext_decrypts_exactly():
    prm = tiny()
    ks = keys.keygen(prm, 5, 2)
    rng = np.random.default_rng(0)
    m = rng.integers(-1000, 1000, prm.N).astype(np.int64)
    for level in (prm.L, 3):
        ct = ckks.encrypt(prm, ks, m, level, 5, 7)
        v, e0, e1 = ckks.encrypt_noise(prm, 5, 7)
        s = [int(x) for x in ks.s]
        ve = polymul_neg([int(x) for x in v], [int(x) for x in ks.pk_e])
        e1s = polymul_neg([int(x) for x in e1], s)
        want = [int(a) + b + int(c) + d for a, b, c, d in zip(m, ve, e0, e1s)]
        assert ckks.decrypt(prm, ks, ct, level) == want


def test_encode_fft_matches_direct_sum_and_decodes():
    n = 64
    re, im = prng.slots(prng.stream_key(1, "MSG", 0), n // 2)
    scale = 2.0 ** 30
    m = ckks.encode(re, im, n, scale)
    assert np.array_equal(m, ckks.encode_direct(re, im, n, scale))
    r2, i2 = ckks.decode(m, n, scale)
    assert np.abs(r2 - re).max() < 1e-7 and np.abs(i2 - im).max() < 1e-7


def test_encode_is_the_canonical_embedding():
    # a real message constant across slots encodes to a constant polynomial
    n = 32
    m = ckks.encode(np.full(n // 2, 0.25), np.zeros(n // 2), n, 2.0 ** 20)
    assert m[0] == 2 ** 18 and not np.any(m[1:])
    # the monomial x decodes to the roots zeta_j = exp(i pi 5^j / N)
    x = [0, 1] + [0] * (n - 2)
    re, im = ckks.decode(x, n, 1.0)
    r = ckks.slot_exponents(n)
    z = np.exp(1j * np.pi * r / n)
    assert np.allclose(re, z.real) and np.allclose(im, z.imag)


# ------------------------------------------------------------------ tensor

@pytest.mark.parametrize("k", [2, 3, 4])
def test_tensor_against_bigint_product(k):
    prm = tiny(log_n=4, L=4, K=2, dnum=2)
    level = 3
    qs, psis = prm.q[:level], prm.psi_q[:level]
    rng = np.random.default_rng(k)
    cts = [np.stack([np.stack([rng.integers(0, q, prm.N).astype(np.uint64) for q in qs]) for _ in range(2)])
           for _ in range(k)]
    D = mult.tensor(cts, qs)
    # coefficient-domain polynomials of each input, as centred big ints
    polys = [[centered_crt(coeff_residues(prm, c[l], qs, psis), qs) for l in (0, 1)] for c in cts]
    # prod_u (c0_u + c1_u Y) as a polynomial in Y with ring coefficients
    acc = [[1] + [0] * (prm.N - 1)]
    for c0, c1 in polys:
        nxt = [[0] * prm.N for _ in range(len(acc) + 1)]
        for t, a in enumerate(acc):
            p0, p1 = polymul_neg(a, c0), polymul_neg(a, c1)
            nxt[t] = [x + y for x, y in zip(nxt[t], p0)]
            nxt[t + 1] = [x + y for x, y in zip(nxt[t + 1], p1)]
        acc = nxt
    Q = prm.Q(level)
    for t in range(k + 1):
        got = centered_crt(coeff_residues(prm, D[t], qs, psis), qs)
        want = [((x + Q // 2) % Q) - Q // 2 for x in acc[t]]
        assert [g % Q for g in got] == [w % Q for w in want]


def test_tensor_evaluation_identity_large():
    """sum_t D_t S^t = prod_u (C0_u + C1_u S) pointwise, at an N = 2^13 shape."""
    prm = params.preset(13)
    level = 3
    qs = prm.q[:level]
    qc = np.array(qs, dtype=np.uint64).reshape(-1, 1)
    rng = np.random.default_rng(9)
    k = 5
    cts = [np.stack([np.stack([rng.integers(0, q, prm.N).astype(np.uint64) for q in qs]) for _ in range(2)])
           for _ in range(k)]
    S = np.stack([rng.integers(0, q, prm.N).astype(np.uint64) for q in qs])
    D = mult.tensor(cts, qs)
    lhs = np.zeros_like(S)
    Sp = np.ones_like(S)
    for t in range(k + 1):
        lhs = (lhs + (D[t] * Sp) % qc) % qc
        Sp = (Sp * S) % qc
    rhs = np.ones_like(S)
    for c in cts:
        rhs = (rhs * ((c[0] + (c[1] * S) % qc) % qc)) % qc
    assert np.array_equal(lhs, rhs)


# ------------------------------------------------------------------ basis conversion

def test_fast_bconv_crt_invariant():
    prm = params.preset(15)
    src = prm.q[4:8]
    dst = prm.q[:4] + prm.p
    rng = np.random.default_rng(3)
    n = 64
    x = np.stack([rng.integers(0, q, n).astype(np.uint64) for q in src])
    out = mult.bconv(x, src, dst)
    Qs = math.prod(src)
    for i in range(n):
        X = centered_crt([x[:, i:i + 1][j] for j in range(len(src))], src) [0] % Qs
        # out = X + u Qs (mod m) for one u in [0, len(src)), the same for every target
        us = set()
        for row, m in enumerate(dst):
            cand = [u for u in range(len(src)) if (X + u * Qs) % m == int(out[row, i])]
            assert len(cand) == 1
            us.add(cand[0])
        assert len(us) == 1


def test_scbconv_is_p_inverse_times_bconv():
    prm = params.preset(15)
    level = 5
    rng = np.random.default_rng(4)
    n = 256
    cp = np.stack([rng.integers(0, p, n).astype(np.uint64) for p in prm.p])
    a = mult.scbconv(prm, cp, level)
    b = mult.bconv(cp, prm.p, prm.q[:level])
    for j, q in enumerate(prm.q[:level]):
        pinv = pow(prm.P % q, -1, q)
        assert np.array_equal(a[j], (b[j] * np.uint64(pinv)) % np.uint64(q))


# ------------------------------------------------------------------ rescaling

@pytest.mark.parametrize("level,mu", [(6, 1), (6, 2), (6, 5), (4, 3)])
def test_multi_rescale_is_floor_division(level, mu):
    """rs^mu(x) = floor(x / (q_{l-1} ... q_{l-mu})) for x in [0, Q_l)."""
    prm = tiny(log_n=3, L=6, K=2, dnum=3)
    rng = np.random.default_rng(level * 10 + mu)
    n = prm.N
    a = np.stack([rng.integers(0, q, n).astype(np.uint64) for q in prm.q[:level]])
    D = math.prod(prm.q[level - mu:level])
    Q = prm.Q(level)
    xs = [c % Q for c in centered_crt(a, prm.q[:level])]
    want = [[(x // D) % q for x in xs] for q in prm.q[:level - mu]]
    got = mult.multi_rs_coeff(prm, a, level, mu)
    assert [[int(v) for v in row] for row in got] == want
    # the chained single rescale of eq. (1-rs) agrees
    b = a
    for i in range(mu):
        b = mult.rs_coeff(prm, b, level - i)
    assert np.array_equal(b, got)


@pytest.mark.parametrize("mu", [1, 2, 4])
def test_alg1_and_textbook_and_baseline_rescale_agree(mu):
    prm = params.preset(13)
    prm2 = mk(10, 6, 2, 3)
    level = 6
    rng = np.random.default_rng(mu)
    A = np.stack([rng.integers(0, q, prm2.N).astype(np.uint64) for q in prm2.q[:level]])
    r1 = mult.multi_rs_alg1(prm2, A, level, mu)
    r2 = mult.rescale_textbook(prm2, A, level, mu)
    r3 = mult.rescale_baseline(prm2, A, level, mu)
    assert np.array_equal(r1, r2) and np.array_equal(r1, r3)
    assert prm.N == 8192


@pytest.mark.parametrize("L,mu", [(8, 2), (8, 5), (24, 2), (24, 7)])
def test_alg1_counts_match_table_iv(L, mu):
    """Table IV: mu-RS by Algorithm 1 takes mu INTT, L - mu NTT and
    (mu + 1) L - mu (mu + 3) / 2 constant multiplications."""
    prm = mk(3, L, 1, 1)
    rng = np.random.default_rng(1)
    A = np.stack([rng.integers(0, q, prm.N).astype(np.uint64) for q in prm.q])
    with counts.counting() as c:
        mult.multi_rs_alg1(prm, A, L, mu)
    assert c.get("intt", 0) == mu
    assert c.get("ntt", 0) == L - mu
    assert c["rs_const"] == (mu + 1) * L - mu * (mu + 3) // 2


# ------------------------------------------------------------------ relinearisation

def _bound_relin(prm, k, level):
    alpha = prm.alpha
    digits = prm.digits(level)
    qb = max(math.prod(prm.q[j] for j in d) for d in digits)
    return (k - 1) * len(digits) * prm.N * alpha * 19 * qb / prm.P + prm.K * (1 + prm.h)


@pytest.mark.parametrize("k,level", [(2, 6), (3, 6), (4, 5), (3, 3)])
def test_relinearisation_identity(k, level):
    """Decrypting the relinearised pair gives sum_t d_t s^t up to the key
    switching noise bound (k-1) B N alpha B_e max Q_b / P + K (1 + h)."""
    prm = mk(6, 6, 3, 3)
    ks = keys.keygen(prm, 21, 4)
    qs, psis = prm.q[:level], prm.psi_q[:level]
    qc = np.array(qs, dtype=np.uint64).reshape(-1, 1)
    rng = np.random.default_rng(k * 7 + level)
    D = np.stack([np.stack([rng.integers(0, q, prm.N).astype(np.uint64) for q in qs]) for _ in range(k + 1)])
    c0, c1 = mult.relin_textbook(prm, ks, D, level)
    S = ks.S[:level]
    diff = (c0 + (c1 * S) % qc) % qc
    Sp = np.ones_like(S)
    for t in range(k + 1):
        diff = (diff + qc - (D[t] * Sp) % qc) % qc
        Sp = (Sp * S) % qc
    err = centered_crt(coeff_residues(prm, diff, qs, psis), qs)
    assert max(abs(e) for e in err) <= _bound_relin(prm, k, level)
    # the relocated form (Sec. IV) gives the same ring elements, coefficient domain
    y0, y1 = mult.relin_relocated(prm, ks, D, level)
    assert np.array_equal(ntt.ntt(y0, qs, psis), c0)
    assert np.array_equal(ntt.ntt(y1, qs, psis), c1)


@pytest.mark.parametrize("path", ["textbook", "relocated"])
def test_transform_counts_match_table_v(path):
    """Table V, three inputs, single-digit keys (K >= L): the prior design takes
    6L + 2K - 6 NTT and 4L + 2K + 4 INTT, the improved one 2L + 2K - 4 NTT and
    4L + 2K INTT."""
    L, K = 5, 5
    prm = mk(3, L, K, 1)
    ks = keys.keygen(prm, 3, 3)
    rng = np.random.default_rng(2)
    cts = [np.stack([np.stack([rng.integers(0, q, prm.N).astype(np.uint64) for q in prm.q]) for _ in range(2)])
           for _ in range(3)]
    with counts.counting() as c:
        mult.mul_relin_rescale(prm, ks, cts, L, path=path)
    if path == "textbook":
        assert (c["ntt"], c["intt"]) == (6 * L + 2 * K - 6, 4 * L + 2 * K + 4)
    else:
        assert (c["ntt"], c["intt"]) == (2 * L + 2 * K - 4, 4 * L + 2 * K)
        assert c["ntt"] + c["intt"] == mult.transform_count(3, L, K, prm.alpha)


@pytest.mark.parametrize("k,level", [(3, 6), (5, 6), (2, 3)])
def test_transform_count_formula_hybrid(k, level):
    prm = mk(3, 6, 2, 3)
    ks = keys.keygen(prm, 3, 5)
    rng = np.random.default_rng(2)
    cts = [np.stack([np.stack([rng.integers(0, q, prm.N).astype(np.uint64) for q in prm.q[:level]])
                     for _ in range(2)]) for _ in range(k)]
    with counts.counting() as c:
        mult.mul_relin_rescale(prm, ks, cts, level)
    assert c["ntt"] + c["intt"] == mult.transform_count(k, level, prm.K, prm.alpha)


# ------------------------------------------------------------------ end to end

@pytest.mark.parametrize("k,level", [(2, 6), (3, 6), (4, 6), (3, 4)])
def test_end_to_end_integer_bound(k, level):
    """After mu = k - 1 rescales the decryption is within h + 2 + ceil(B/D) of
    round(prod_u Dec(ct_u) / D), D = product of the dropped primes."""
    prm = mk(5, 6, 3, 3)
    ks = keys.keygen(prm, 31, 4)
    rng = np.random.default_rng(k + level)
    ms, cts = [], []
    for u in range(k):
        m = rng.integers(-(1 << 28), 1 << 28, prm.N).astype(np.int64)
        ct = ckks.encrypt(prm, ks, m, level, 31, u)
        cts.append(ct)
        ms.append(ckks.decrypt(prm, ks, ct, level))
    prod = ms[0]
    for x in ms[1:]:
        prod = polymul_neg(prod, x)
    Q = prm.Q(level)
    prod = [((x + Q // 2) % Q) - Q // 2 for x in prod]
    D = math.prod(prm.q[level - k + 1:level])
    out_level = level - k + 1
    Qo = prm.Q(out_level)
    for path in ("relocated", "textbook"):
        out = mult.mul_relin_rescale(prm, ks, cts, level, path=path)
        dec = ckks.decrypt(prm, ks, out, out_level)
        bound = prm.h + 2 + math.ceil(_bound_relin(prm, k, level) / D)
        for x, y in zip(dec, prod):
            r = (2 * y + D) // (2 * D)          # round(y / D), half up
            d = (x - r) % Qo
            d = d - Qo if d > Qo // 2 else d
            assert abs(d) <= bound


def test_relocated_equals_textbook_bit_for_bit_c1():
    prm = params.preset(13)
    ks = keys.keygen(prm, 1, 3)
    cts = []
    for u in range(3):
        _, _, m = ckks.message(prm, 1, u, 2.0 ** 30)
        cts.append(ckks.encrypt(prm, ks, m, 3, 1, u))
    a = mult.mul_relin_rescale(prm, ks, cts, 3, path="relocated")
    b = mult.mul_relin_rescale(prm, ks, cts, 3, path="textbook")
    assert a.shape == (2, 1, prm.N) and np.array_equal(a, b)


def test_decoded_three_way_product_c1():
    """Decoding the C1 product recovers prod_u z_u slot-wise within the stated
    numeric bound (fresh noise + encoding rounding, 6-sigma)."""
    prm = params.preset(13)
    ks = keys.keygen(prm, 1, 3)
    scale = 2.0 ** 30
    zs, cts = [], []
    for u in range(3):
        re, im, m = ckks.message(prm, 1, u, scale)
        zs.append(re + 1j * im)
        cts.append(ckks.encrypt(prm, ks, m, 3, 1, u))
    out = mult.mul_relin_rescale(prm, ks, cts, 3)
    dec = ckks.decrypt(prm, ks, out, 1)
    scale_out = scale ** 3 / (prm.q[2] * prm.q[1])
    re, im = ckks.decode(dec, prm.N, scale_out)
    got = re + 1j * im
    want = zs[0] * zs[1] * zs[2]
    n, sigma, h = prm.N, prm.sigma, prm.h
    eps = 6 * math.sqrt(n) * sigma * math.sqrt(n / 2 + 1 + h + 1 / (12 * sigma ** 2)) / scale
    eps_out = 6 * math.sqrt(n) * math.sqrt((1 + h) / 12) / scale_out
    bound = 0.0
    for u in range(3):
        term = eps
        for w in range(3):
            if w != u:
                term *= (np.abs(zs[w]) + eps)
        bound = bound + term
    bound = bound + eps_out
    assert np.all(np.abs(got - want) <= bound)
    assert np.abs(got - want).max() < 1e-3


def _golden_table_v():
    rows = []
    path = __file__.rsplit("/", 1)[0] + "/golden/table_v_three_input_counts.txt"
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            d, st, L, K, a, b = line.split()
            rows.append((d, st, int(L), int(K), int(a), int(b)))
    return rows


def test_stage_counts_match_table_v_at_paper_parameters():
    """Per-stage transform counts at L = K = 24 against the printed Table V."""
    rows = _golden_table_v()
    L, K = rows[0][2], rows[0][3]
    prm = mk(3, L, K, 1)
    ks = keys.keygen(prm, 4, 3)
    rng = np.random.default_rng(8)
    cts = [np.stack([np.stack([rng.integers(0, q, prm.N).astype(np.uint64) for q in prm.q]) for _ in range(2)])
           for _ in range(3)]
    D = mult.tensor(cts, prm.q)
    got = {}
    with counts.counting() as c:
        c0, c1 = mult.relin_textbook(prm, ks, D, L)
    got[("prior", "relin")] = (c.get("ntt", 0), c.get("intt", 0))
    with counts.counting() as c:
        mult.rescale_textbook(prm, c0, L, 2)
        mult.rescale_textbook(prm, c1, L, 2)
    got[("prior", "rescale")] = (c.get("ntt", 0), c.get("intt", 0))
    with counts.counting() as c:
        y0, y1 = mult.relin_relocated(prm, ks, D, L)
    got[("improved", "relin")] = (c.get("ntt", 0), c.get("intt", 0))
    with counts.counting() as c:
        for y in (y0, y1):
            ntt.ntt(mult.multi_rs_coeff(prm, y, L, 2), prm.q[:L - 2], prm.psi_q[:L - 2])
    got[("improved", "rescale")] = (c.get("ntt", 0), c.get("intt", 0))
    for d, st, _, _, n_ntt, n_intt in rows:
        assert got[(d, st)] == (n_ntt, n_intt), (d, st)
    assert sum(sum(v) for k, v in got.items() if k[0] == "prior") == 334
    assert sum(sum(v) for k, v in got.items() if k[0] == "improved") == 236
