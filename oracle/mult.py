"""k-input multiply: tensor product, relinearisation, rescaling (oracle side).

Test infrastructure only (see ``oracle/__init__``).

Each function follows one passage of the paper, in its order and notation:

tensor           eq. (d_u formula for n-ct mult), Sec. V-A: d_t is the sum over
                 l in {0,1}^k with |l| = t of prod_u c^u_{l_u}.
bconv            eq. (basis conversion), Sec. II (fast BConv).
modup            Sec. II: INTT, BConv from each digit, NTT of the new limbs.
kip              Sec. III eq. (product3) and Sec. V-A eq. (extended relin): the
                 products d_t ek_t for all t are summed before one ModDown
                 per output polynomial (the combination of Sec. III).
moddown          eq. (moddown operation), Sec. II.
relin_textbook   ModUp, key products, ModDown, then (d0, d1) + result.
rs_ntt           eq. (1 rs NTT), Sec. II: one rescale in the NTT domain.
rs_coeff         eq. (1-rs), Sec. II: one rescale in the coefficient domain.
relin_relocated  Sec. IV: INTT of D_l + P^-1 C~^(q) (eq. (moddown improved 2)),
                 minus the scaled BConv of eq. (scBconv); result stays in the
                 coefficient domain.
multi_rs_coeff   eq. (multi rs), Sec. V-B, on coefficient-domain input.
multi_rs_alg1    Algorithm 1 (multi-RS), Sec. V-B, on NTT-domain input.
mul_relin_rescale  the whole k-input multiply, textbook or relocated.

Readings where the paper is silent: the rescaled limb enters eq. (1-rs) as its
representative in [0, q_{L-1}) (floor, not rounding); the dropped primes are
the highest remaining indices; the ModDown is combined over t (one per output
polynomial), as the paper's architecture does.
"""
from __future__ import annotations

import numpy as np

from . import counts
from . import ntt as _ntt
from .keys import Keys, evk_at_level
from .params import Params


def _col(moduli) -> np.ndarray:
    return np.array(moduli, dtype=np.uint64).reshape(-1, 1)


# ---------------------------------------------------------------- tensor

def tensor(cts, qs) -> np.ndarray:
    """D_t, t = 0..k, from k NTT-domain ciphertexts ([2, l, N] each).

    Sum over every selection l in {0,1}^k; products that share a prefix
    (l_1..l_u) are formed once and reused by all their extensions."""
    k = len(cts)
    qc = _col(qs)
    level, n = cts[0].shape[1], cts[0].shape[2]
    D = np.zeros((k + 1, level, n), dtype=np.uint64)

    def walk(u, weight, prod):
        if u == k:
            D[weight] = (D[weight] + prod) % qc
            return
        for bit in (0, 1):
            c = np.asarray(cts[u][bit], dtype=np.uint64)
            nxt = c.copy() if prod is None else (prod * c) % qc
            walk(u + 1, weight + bit, nxt)

    walk(0, 0, None)
    return D


# ---------------------------------------------------------------- BConv

def bconv(x: np.ndarray, src, dst) -> np.ndarray:
    """Fast basis conversion: [sum_j [x_j qhat_j^-1]_{q_j} qhat_j]_{m} for m in dst."""
    Qs = 1
    for q in src:
        Qs *= q
    out = np.zeros((len(dst), x.shape[1]), dtype=np.uint64)
    for j, q in enumerate(src):
        qhat = Qs // q
        y = (np.asarray(x[j], dtype=np.uint64) * np.uint64(pow(qhat % q, -1, q))) % np.uint64(q)
        for i, m in enumerate(dst):
            out[i] = (out[i] + (y * np.uint64(qhat % m)) % np.uint64(m)) % np.uint64(m)
    return out


# ---------------------------------------------------------------- ModUp

def modup(prm: Params, Dt: np.ndarray, level: int):
    """ModUp of one NTT-domain polynomial over q_0..q_{level-1}.

    Returns one NTT-domain array per digit, rows ordered as the extended basis
    (q_0..q_{level-1}, p_0..p_{K-1}).  Rows of the digit's own primes are the
    input itself; the others are NTT(BConv(INTT(input restricted to the digit)))."""
    qs, psis = prm.q[:level], prm.psi_q[:level]
    ext, epsi = prm.ext_moduli(level), prm.ext_psi(level)
    dt = _ntt.intt(Dt, qs, psis)
    out = []
    for digit in prm.digits(level):
        tgt = [i for i in range(len(ext)) if i not in digit]
        y = bconv(dt[digit], [qs[j] for j in digit], [ext[i] for i in tgt])
        Y = _ntt.ntt(y, [ext[i] for i in tgt], [epsi[i] for i in tgt])
        X = np.zeros((len(ext), Dt.shape[1]), dtype=np.uint64)
        X[digit] = Dt[digit]
        X[tgt] = Y
        out.append(X)
    return out


# ---------------------------------------------------------------- key inner product

def kip(prm: Params, keys: Keys, D: np.ndarray, level: int, scaled: bool):
    """(Acc_0, Acc_1) = sum_t sum_b ModUp_b(D_t) * ek_{t,b} over Q_level * P."""
    k = D.shape[0] - 1
    ext = prm.ext_moduli(level)
    mc = _col(ext)
    acc0 = np.zeros((len(ext), D.shape[2]), dtype=np.uint64)
    acc1 = np.zeros_like(acc0)
    for t in range(2, k + 1):
        for b, X in enumerate(modup(prm, D[t], level)):
            k0, k1 = evk_at_level(prm, keys, t, b, level, scaled=scaled)
            acc0 = (acc0 + (X * k0) % mc) % mc
            acc1 = (acc1 + (X * k1) % mc) % mc
    return acc0, acc1


# ---------------------------------------------------------------- ModDown

def moddown(prm: Params, acc: np.ndarray, level: int) -> np.ndarray:
    """[P^-1 (c~^(q) - BConv_{P->q}(c~^(p)))]_q from an NTT-domain accumulator;
    returns the coefficient-domain result c^ over q_0..q_{level-1}."""
    qs, psis = prm.q[:level], prm.psi_q[:level]
    cq = _ntt.intt(acc[:level], qs, psis)
    cp = _ntt.intt(acc[level:], prm.p, prm.psi_p)
    cbar = bconv(cp, prm.p, qs)
    qc = _col(qs)
    pinv = _col([pow(prm.P % q, -1, q) for q in qs])
    return (((cq + qc - cbar) % qc) * pinv) % qc


def relin_textbook(prm: Params, keys: Keys, D: np.ndarray, level: int):
    """(C0*, C1*) = (D0, D1) + NTT(ModDown(sum_t ModUp(D_t) ek_t)), NTT domain."""
    qs, psis = prm.q[:level], prm.psi_q[:level]
    qc = _col(qs)
    acc0, acc1 = kip(prm, keys, D, level, scaled=False)
    c0 = (D[0] + _ntt.ntt(moddown(prm, acc0, level), qs, psis)) % qc
    c1 = (D[1] + _ntt.ntt(moddown(prm, acc1, level), qs, psis)) % qc
    return c0, c1


def scbconv(prm: Params, cp: np.ndarray, level: int) -> np.ndarray:
    """eq. (scBconv): [sum_i [phat_i^-1 x_i]_{p_i} p_i^-1]_{q_j}."""
    qs = prm.q[:level]
    P = prm.P
    out = np.zeros((level, cp.shape[1]), dtype=np.uint64)
    for i, p in enumerate(prm.p):
        phat = P // p
        y = (cp[i] * np.uint64(pow(phat % p, -1, p))) % np.uint64(p)
        for j, q in enumerate(qs):
            out[j] = (out[j] + (y * np.uint64(pow(p % q, -1, q))) % np.uint64(q)) % np.uint64(q)
    return out


def relin_relocated(prm: Params, keys: Keys, D: np.ndarray, level: int):
    """Sec. IV: c*_l = INTT_q(D_l + P^-1 C~_l^(q)) - P^-1 BConv(INTT_p(C~_l^(p))),
    with P^-1 folded into the q rows of the keys; coefficient domain."""
    qs, psis = prm.q[:level], prm.psi_q[:level]
    qc = _col(qs)
    acc = kip(prm, keys, D, level, scaled=True)
    out = []
    for l in (0, 1):
        cp = _ntt.intt(acc[l][level:], prm.p, prm.psi_p)
        y = _ntt.intt((D[l] + acc[l][:level]) % qc, qs, psis)
        out.append((y + qc - scbconv(prm, cp, level)) % qc)
    return out[0], out[1]


# ---------------------------------------------------------------- rescaling

def rs_coeff(prm: Params, a: np.ndarray, level: int) -> np.ndarray:
    """eq. (1-rs): [q_{l-1}^-1 (a^(j) - a^(l-1))]_{q_j}, j < l - 1, coefficient domain."""
    top = prm.q[level - 1]
    qs = prm.q[:level - 1]
    qc = _col(qs)
    last = np.asarray(a[level - 1], dtype=np.uint64)
    counts.add("rs_const", level - 1)
    inv = _col([pow(top, -1, q) for q in qs])
    lifted = last.reshape(1, -1) % qc
    return (((a[:level - 1] + qc - lifted) % qc) * inv) % qc


def rs_ntt(prm: Params, A: np.ndarray, level: int) -> np.ndarray:
    """eq. (1 rs NTT): q_{l-1}^-1 (C^(j) - NTT_{q_j}(INTT_{q_{l-1}}(C^(l-1))))."""
    top, ptop = prm.q[level - 1], prm.psi_q[level - 1]
    qs, psis = prm.q[:level - 1], prm.psi_q[:level - 1]
    qc = _col(qs)
    last = _ntt.intt(A[level - 1:level], [top], [ptop])[0]
    lifted = _ntt.ntt(np.broadcast_to(last, (level - 1, A.shape[1])) % qc, qs, psis)
    counts.add("rs_const", level - 1)
    inv = _col([pow(top, -1, q) for q in qs])
    return (((A[:level - 1] + qc - lifted) % qc) * inv) % qc


def rescale_textbook(prm: Params, A: np.ndarray, level: int, mu: int) -> np.ndarray:
    """mu rescales one after another with eq. (1 rs NTT)."""
    for i in range(mu):
        A = rs_ntt(prm, A, level - i)
    return A


def rescale_baseline(prm: Params, A: np.ndarray, level: int, mu: int) -> np.ndarray:
    """The 2L - mu transform baseline of Sec. V-B: INTT every limb, mu times
    eq. (1-rs), NTT the rest."""
    a = _ntt.intt(A, prm.q[:level], prm.psi_q[:level])
    for i in range(mu):
        a = rs_coeff(prm, a, level - i)
    return _ntt.ntt(a, prm.q[:level - mu], prm.psi_q[:level - mu])


def g_const(prm: Params, level: int, u: int, t: int, eta: int) -> int:
    """eq. (g(u,t,eta)): q_{l-u}^-1 q_{l-u+1}^-1 ... q_t^-1 mod q_eta (L read as l)."""
    q = prm.q[eta]
    out = 1
    for x in range(level - u, t + 1):
        out = out * pow(prm.q[x], -1, q) % q
    return out


def _rs_chain(prm: Params, a_dropped: dict, level: int, mu: int) -> dict:
    """Step 2 of Algorithm 1: a^(t),{u} = rs(a^(t),{u-1}) for the dropped limbs,
    returning a^(t),{l-1-t} for t in [l - mu, l - 1]."""
    cur = {t: np.asarray(a_dropped[t], dtype=np.uint64) for t in range(level - mu, level)}
    final = {level - 1: cur[level - 1]}
    for u in range(1, mu):
        drop = level - u                      # limb removed by the u-th rescale
        qd = prm.q[drop]
        nxt = {}
        for t in range(level - mu, level - u):
            qt = np.uint64(prm.q[t])
            inv = np.uint64(pow(qd, -1, prm.q[t]))
            lifted = cur[drop] % qt
            nxt[t] = (((cur[t] + qt - lifted) % qt) * inv) % qt
            counts.add("rs_const", 1)
        cur = nxt
        final[level - 1 - u] = cur[level - 1 - u]
    return final


def multi_rs_coeff(prm: Params, a: np.ndarray, level: int, mu: int) -> np.ndarray:
    """eq. (multi rs) on coefficient-domain input: for eta < l - mu,
    a^(eta),{mu} = g^{mu,l-1}_eta a^(eta) - sum_t g^{mu,t}_eta a^(t),{l-1-t}."""
    fin = _rs_chain(prm, {t: a[t] for t in range(level - mu, level)}, level, mu)
    out = np.zeros((level - mu, a.shape[1]), dtype=np.uint64)
    for eta in range(level - mu):
        q = np.uint64(prm.q[eta])
        acc = (np.asarray(a[eta], dtype=np.uint64) * np.uint64(g_const(prm, level, mu, level - 1, eta))) % q
        for t in range(level - mu, level):
            term = ((fin[t] % q) * np.uint64(g_const(prm, level, mu, t, eta))) % q
            acc = (acc + q - term) % q
        counts.add("rs_const", mu + 1)
        out[eta] = acc
    return out


def multi_rs_alg1(prm: Params, A: np.ndarray, level: int, mu: int) -> np.ndarray:
    """Algorithm 1 (multi-RS) on NTT-domain input A^(j), j < l."""
    a = {}
    for u in range(level - mu, level):                       # step 1
        a[u] = _ntt.intt(A[u:u + 1], [prm.q[u]], [prm.psi_q[u]])[0]
    fin = _rs_chain(prm, a, level, mu)                       # step 2
    out = np.zeros((level - mu, A.shape[1]), dtype=np.uint64)
    for eta in range(level - mu):                            # step 3
        q = np.uint64(prm.q[eta])
        b = np.zeros(A.shape[1], dtype=np.uint64)
        for t in range(level - mu, level):
            b = (b + ((fin[t] % q) * np.uint64(g_const(prm, level, mu, t, eta))) % q) % q
        B = _ntt.ntt(b.reshape(1, -1), [prm.q[eta]], [prm.psi_q[eta]])[0]
        gA = (np.asarray(A[eta], dtype=np.uint64) * np.uint64(g_const(prm, level, mu, level - 1, eta))) % q
        out[eta] = (gA + q - B) % q
        counts.add("rs_const", mu + 1)
    return out


# ---------------------------------------------------------------- whole multiply

def mul_relin_rescale(prm: Params, keys: Keys, cts, level: int, path: str = "relocated") -> np.ndarray:
    """k-input multiply at `level` with mu = k - 1 rescales; NTT-domain
    output uint64 [2, level - k + 1, N]."""
    k = len(cts)
    if k < 2 or level < k or level > prm.L or k > keys.k_max:
        raise ValueError("invalid k / level")
    qs = prm.q[:level]
    D = tensor(cts, qs)
    mu = k - 1
    if path == "textbook":
        c0, c1 = relin_textbook(prm, keys, D, level)
        return np.stack([rescale_textbook(prm, c0, level, mu), rescale_textbook(prm, c1, level, mu)])
    if path == "relocated":
        y0, y1 = relin_relocated(prm, keys, D, level)
        lo, plo = prm.q[:level - mu], prm.psi_q[:level - mu]
        r0 = _ntt.ntt(multi_rs_coeff(prm, y0, level, mu), lo, plo)
        r1 = _ntt.ntt(multi_rs_coeff(prm, y1, level, mu), lo, plo)
        return np.stack([r0, r1])
    raise ValueError(path)


def transform_count(k: int, level: int, K: int, alpha: int) -> int:
    """(I)NTT limb transforms of the relocated path:
    (k-1) B (l+K) ModUp + 2K + 2l ModDown + 2(l-k+1) final NTT, B = ceil(l/alpha)."""
    B = -(-level // alpha)
    return (k - 1) * B * (level + K) + 2 * K + 4 * level - 2 * k + 2
