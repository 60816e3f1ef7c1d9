"""Seeded synthetic inputs shared by the oracle-side digest scripts and the GPU
tests.  Nothing here computes any step of the method: it only draws uniform
residues per limb from numpy's seeded generator and hashes arrays.
"""
from __future__ import annotations

import hashlib

import numpy as np


def uniform_ct(rng: np.random.Generator, qs, n: int) -> np.ndarray:
    """One NTT-domain ciphertext [2][len(qs)][n] of uniform residues, uint64."""
    return np.stack([np.stack([rng.integers(0, q, n, dtype=np.int64).astype(np.uint64) for q in qs])
                     for _ in range(2)])


def uniform_cts(seed: int, qs, n: int, k: int):
    """k ciphertexts from one seed, in the order both sides draw them."""
    rng = np.random.default_rng(seed)
    return [uniform_ct(rng, qs, n) for _ in range(k)]


def limb_digests(arr: np.ndarray):
    """SHA-256 (first 16 hex digits) of every limb of a [polys][limbs][N] array,
    taken over the residues as little-endian uint32."""
    a = np.ascontiguousarray(np.asarray(arr, dtype=np.uint64).astype("<u4"))
    return [hashlib.sha256(a[p, j].tobytes()).hexdigest()[:16]
            for p in range(a.shape[0]) for j in range(a.shape[1])]
