"""Encode, encrypt, decrypt, decode (oracle side).

Test infrastructure only (see ``oracle/__init__``).

* Encryption (Sec. II): with v ternary of weight N/2 and e0, e1 Gaussian,
  (c0, c1) = (m + v b + e0, v a + e1) per limb, where m already carries the
  scale Delta.  Ciphertexts are kept in the NTT domain, limbs q_0..q_{l-1}.
* Decryption (Sec. II): c0 + c1 s.  The paper reads limb 0 only; this oracle
  reconstructs the residues over every active limb by CRT and centres the
  result, which agrees with limb 0 whenever |m| < q_0 / 2.
* Encoding (the paper does not describe it): CKKS canonical embedding with
  N/2 slots, slot j at zeta_j = exp(i pi (5^j mod 2N) / N), and
  m_i = round((2/N) Re sum_j Delta z_j zeta_j^-i), rounding half away from
  zero, in FP64.  Decoding evaluates m(zeta_j) / Delta.
"""
from __future__ import annotations

import numpy as np

from . import ntt as _ntt
from . import prng
from .keys import Keys, _residues
from .params import Params


def slot_exponents(n: int) -> np.ndarray:
    """r_j = 5^j mod 2N for j < N/2."""
    out = np.empty(n // 2, dtype=np.int64)
    v = 1
    for j in range(n // 2):
        out[j] = v
        v = v * 5 % (2 * n)
    return out


def _round_half_away(x: np.ndarray) -> np.ndarray:
    return (np.sign(x) * np.floor(np.abs(x) + 0.5)).astype(np.int64)


def encode(re: np.ndarray, im: np.ndarray, n: int, scale: float) -> np.ndarray:
    """m_i = round((2/N) Re sum_j scale z_j zeta_j^-i), via a length-2N FFT."""
    r = slot_exponents(n)
    W = np.zeros(2 * n, dtype=np.complex128)
    W[r] = scale * (np.asarray(re) + 1j * np.asarray(im))
    F = np.fft.fft(W)          # F[i] = sum_r W[r] exp(-2 pi i r i / 2N)
    return _round_half_away((2.0 / n) * F[:n].real)


def encode_direct(re, im, n: int, scale: float) -> np.ndarray:
    """The same sum evaluated term by term (small N only)."""
    r = slot_exponents(n)
    z = scale * (np.asarray(re) + 1j * np.asarray(im))
    i = np.arange(n)
    zeta_inv = np.exp(-1j * np.pi * np.outer(i, r) / n)
    return _round_half_away((2.0 / n) * (zeta_inv @ z).real)


def decode(m, n: int, scale: float):
    """z_j = m(zeta_j) / scale for j < N/2; m may hold Python ints."""
    r = slot_exponents(n)
    mf = np.array([float(x) for x in m], dtype=np.float64)
    pad = np.zeros(2 * n, dtype=np.complex128)
    pad[:n] = mf
    F = np.fft.ifft(pad) * (2 * n)    # F[r] = sum_i m_i exp(2 pi i r i / 2N)
    z = F[r] / scale
    return z.real.copy(), z.imag.copy()


def message(prm: Params, seed: int, ct_id: int, scale: float):
    """Slot values of message `ct_id` and their encoding."""
    re, im = prng.slots(prng.stream_key(seed, "MSG", ct_id), prm.N // 2)
    return re, im, encode(re, im, prm.N, scale)


def encrypt(prm: Params, keys: Keys, m: np.ndarray, level: int, seed: int, ct_id: int) -> np.ndarray:
    """NTT-domain ciphertext uint64 [2, level, N]."""
    N = prm.N
    qs, psis = prm.q[:level], prm.psi_q[:level]
    qcol = np.array(qs, dtype=np.uint64).reshape(level, 1)
    v = prng.ternary_hw(prng.stream_key(seed, "ENC_V", ct_id), N, N // 2)
    e0 = prng.gaussian(prng.stream_key(seed, "ENC_E0", ct_id), N, prm.sigma)
    e1 = prng.gaussian(prng.stream_key(seed, "ENC_E1", ct_id), N, prm.sigma)
    V = _ntt.ntt(_residues(v, qs), qs, psis)
    M0 = _ntt.ntt((_residues(e0, qs) + _residues(m, qs)) % qcol, qs, psis)
    E1 = _ntt.ntt(_residues(e1, qs), qs, psis)
    c0 = ((V * keys.pk_b[:level]) % qcol + M0) % qcol
    c1 = ((V * keys.pk_a[:level]) % qcol + E1) % qcol
    return np.stack([c0, c1])


def encrypt_noise(prm: Params, seed: int, ct_id: int):
    """(v, e0, e1) of ciphertext `ct_id`, for exact decryption checks."""
    N = prm.N
    v = prng.ternary_hw(prng.stream_key(seed, "ENC_V", ct_id), N, N // 2)
    e0 = prng.gaussian(prng.stream_key(seed, "ENC_E0", ct_id), N, prm.sigma)
    e1 = prng.gaussian(prng.stream_key(seed, "ENC_E1", ct_id), N, prm.sigma)
    return v, e0, e1


def crt(residues: np.ndarray, moduli) -> list:
    """Per coefficient, the integer in [0, prod moduli) with those residues."""
    Q = 1
    for q in moduli:
        Q *= q
    acc = np.zeros(residues.shape[1], dtype=object)
    for j, q in enumerate(moduli):
        qh = Q // q
        f = qh * pow(qh % q, -1, q)
        acc = acc + residues[j].astype(object) * f
    return [int(x) % Q for x in acc]


def center(xs, Q: int) -> list:
    h = Q // 2
    return [x - Q if x > h else x for x in xs]


def decrypt_residues(prm: Params, keys: Keys, ct: np.ndarray, level: int) -> np.ndarray:
    """Coefficient-domain residues of c0 + c1 s over q_0..q_{level-1}."""
    qs, psis = prm.q[:level], prm.psi_q[:level]
    qcol = np.array(qs, dtype=np.uint64).reshape(level, 1)
    c0 = np.asarray(ct[0], dtype=np.uint64)
    c1 = np.asarray(ct[1], dtype=np.uint64)
    X = (c0 + (c1 * keys.S[:level]) % qcol) % qcol
    return _ntt.intt(X, qs, psis)


def decrypt(prm: Params, keys: Keys, ct: np.ndarray, level: int) -> list:
    """Centred integer polynomial (list of Python ints)."""
    r = decrypt_residues(prm, keys, ct, level)
    return center(crt(r, prm.q[:level]), prm.Q(level))
