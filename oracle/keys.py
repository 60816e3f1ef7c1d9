"""Secret, public and evaluation keys (oracle side).

Test infrastructure only (see ``oracle/__init__``).

* s: ternary, Hamming weight h (Sec. II).
* pk = (b, a) per limb q_j with b = -a s + e (Sec. II).
* ek_t for t = 2..k_max, the key that relinearises d_t (eq. (evks-s^t) in
  Sec. V-A, generalising eq. (evks-s^2) and eq. (evks-s^3)): over the p_i the
  pair (-a s + e_t, a); over the q_j the pair (P s^t - a s + e_t, a).
  With hybrid key switching (dnum digits) there is one such key per digit b,
  and P s^t becomes P G_b s^t with G_b = Qhat_b [Qhat_b^-1]_{Q_b},
  Q_b = prod of the digit's primes at full level, Qhat_b = Q_L / Q_b.  With
  dnum = 1 this is exactly the paper's key (G = 1).  The same e_t is used on
  every limb of one key, as in the paper's equations.

Polynomials a are drawn directly in the NTT domain (uniform either way); s,
e are small integer polynomials transformed per limb.  Everything is kept in
the canonical form: residues in [0, q), NTT domain, unscaled.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Tuple

import numpy as np

from . import ntt as _ntt
from . import prng
from .params import Params


def _residues(poly_int64: np.ndarray, moduli) -> np.ndarray:
    """Integer polynomial -> [len(moduli), N] canonical residues (uint64)."""
    return np.stack([np.mod(poly_int64, np.int64(m)).astype(np.uint64) for m in moduli])


@dataclass
class Keys:
    seed: int
    k_max: int
    s: np.ndarray                      # int64 [N]
    S: np.ndarray                      # NTT(s) over q_0..q_{L-1}, p_0..p_{K-1}: uint64 [L+K, N]
    pk_b: np.ndarray                   # uint64 [L, N]
    pk_a: np.ndarray                   # uint64 [L, N]
    pk_e: np.ndarray                   # int64 [N]
    evk: Dict[Tuple[int, int], Tuple[np.ndarray, np.ndarray]] = field(default_factory=dict)
    evk_e: Dict[Tuple[int, int], np.ndarray] = field(default_factory=dict)


def gadget_residues(prm: Params, b: int):
    """[P * G_b]_m for every modulus m of the full basis (q_0..q_{L-1}, p_*)."""
    a = prm.alpha
    digit = prm.q[b * a: min((b + 1) * a, prm.L)]
    Qb = 1
    for x in digit:
        Qb *= x
    QL = prm.Q(prm.L)
    Qhat = QL // Qb
    G = Qhat * pow(Qhat % Qb, -1, Qb)
    PG = prm.P * G
    return [PG % m for m in prm.q + prm.p]


def keygen(prm: Params, seed: int, k_max: int) -> Keys:
    N, L, K = prm.N, prm.L, prm.K
    moduli = prm.q + prm.p
    psis = prm.psi_q + prm.psi_p
    s = prng.ternary_hw(prng.stream_key(seed, "SK"), N, prm.h)
    S = _ntt.ntt(_residues(s, moduli), moduli, psis)

    qcol = np.array(prm.q, dtype=np.uint64).reshape(L, 1)
    pk_a = np.stack([prng.uniform_mod(prng.stream_key(seed, "PK_A", j), prm.q[j], N) for j in range(L)])
    pk_e = prng.gaussian(prng.stream_key(seed, "PK_E"), N, prm.sigma)
    E = _ntt.ntt(_residues(pk_e, prm.q), prm.q, prm.psi_q)
    pk_b = (E + qcol - (pk_a * S[:L]) % qcol) % qcol

    keys = Keys(seed=seed, k_max=k_max, s=s, S=S, pk_b=pk_b, pk_a=pk_a, pk_e=pk_e)
    mcol = np.array(moduli, dtype=np.uint64).reshape(L + K, 1)
    # S^t in the NTT domain, t = 2..k_max (NTT is a ring homomorphism)
    St = S.copy()
    for t in range(2, k_max + 1):
        St = (St * S) % mcol
        for b in range(prm.dnum):
            a = np.stack([prng.uniform_mod(prng.stream_key(seed, "EVK_A", t, b, i), moduli[i], N)
                          for i in range(L + K)])
            e = prng.gaussian(prng.stream_key(seed, "EVK_E", t, b), N, prm.sigma)
            Ee = _ntt.ntt(_residues(e, moduli), moduli, psis)
            g = np.array(gadget_residues(prm, b), dtype=np.uint64).reshape(L + K, 1)
            k0 = (Ee + mcol - (a * S) % mcol) % mcol
            k0 = (k0 + (St * g) % mcol) % mcol
            keys.evk[(t, b)] = (k0.astype(np.uint32), a.astype(np.uint32))
            keys.evk_e[(t, b)] = e
    return keys


def evk_at_level(prm: Params, keys: Keys, t: int, b: int, level: int, scaled: bool = False):
    """Key (t, b) restricted to the extended basis of `level`: rows
    q_0..q_{level-1}, p_0..p_{K-1}.  With `scaled`, the q rows are multiplied
    by [P^-1]_{q_j} (the pre-multiplication of Sec. IV)."""
    L = prm.L
    k0, k1 = keys.evk[(t, b)]
    rows = list(range(level)) + list(range(L, L + prm.K))
    k0 = k0[rows].astype(np.uint64)
    k1 = k1[rows].astype(np.uint64)
    if scaled:
        P = prm.P
        f = np.array([pow(P % q, -1, q) for q in prm.q[:level]] + [1] * prm.K, dtype=np.uint64).reshape(-1, 1)
        mcol = np.array(prm.ext_moduli(level), dtype=np.uint64).reshape(-1, 1)
        k0 = (k0 * f) % mcol
        k1 = (k1 * f) % mcol
    return k0, k1
