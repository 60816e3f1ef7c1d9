"""Tree-structured n-input multiply with rescaling inside the tree (oracle side).

Test infrastructure only (see ``oracle/__init__``).

Sec. V-C partitions the n inputs into groups, recursively; a node multiplies
the results of its children (the unrelinearised polynomials in s) and, unless
it is the root, rescales every polynomial of the product by (fan-in - 1)
levels with Algorithm 1 (Sec. V-B) in the NTT domain, so that the
multiplicative depth of the whole multiply is ceil(log2 n) instead of n - 1.
The root relinearises its product with the keys for s^2..s^n (Sec. V-A,
eq. (extended relin)) and then rescales the two output polynomials by
(fan-in - 1) levels (Sec. IV relocated ModDown, eq. (multi rs)).

A tree is an int g >= 1 (a group of g consecutive inputs multiplied
together, eq. (d_u formula for n-ct mult)) or a tuple of at least two
subtrees (an internal node).  The flat k-input multiply is the tree k.

Reading (the paper fixes it only through the (I)NTT counts of Table II):
every subtree is evaluated at the level at which its result enters its
parent, so a subtree whose depth is below that of its siblings first drops
the top limbs of its inputs.  With it, the (I)NTT counts of Table II follow
for every row except the four entries listed in tests/test_oracle_tree.py.

n_inputs, degree, fan, depth   shape of a tree (Sec. V-C)
rs_units, ntt_counts           the rescale and transform counts of Table II
plan                           the partition minimising rescale units at depth
                               ceil(log2 n) (Sec. V-C guidelines, Table II)
binary_plan                    the binary-tree partition of Table II's left column
poly_product                   product of polynomials in s (Sec. V-A)
mul_tree                       the whole multiply
"""
from __future__ import annotations

import functools
import math
from typing import List, Tuple, Union

import numpy as np

from . import ntt as _ntt
from .keys import Keys
from .mult import multi_rs_alg1, multi_rs_coeff, relin_relocated, tensor
from .params import Params

Tree = Union[int, tuple]


# ---------------------------------------------------------------- shape

def n_inputs(t: Tree) -> int:
    return t if isinstance(t, int) else sum(n_inputs(c) for c in t)


def degree(t: Tree) -> int:
    """Degree in s of a node's product: every input contributes degree 1."""
    return n_inputs(t)


def fan(t: Tree) -> int:
    """Factors of the node's product, hence its scale Delta^fan and the
    fan - 1 rescales that bring it back to Delta."""
    return t if isinstance(t, int) else len(t)


def depth(t: Tree) -> int:
    """Levels consumed on the longest path (the root's final rescale included)."""
    if isinstance(t, int):
        return t - 1
    return max(depth(c) for c in t) + len(t) - 1


def check(t: Tree) -> None:
    if isinstance(t, int):
        if t < 1:
            raise ValueError("a group holds at least one input")
        return
    if not isinstance(t, tuple) or len(t) < 2:
        raise ValueError("an internal node has at least two children")
    for c in t:
        check(c)


# ---------------------------------------------------------------- Table II counts

def _walk_levels(t: Tree, end: int, root: bool, out: list) -> None:
    """Post-order (node, product level, rescale depth mu, polynomials) with
    levels relative to L (a level L - x is recorded as -x)."""
    mu = fan(t) - 1
    prod = end + mu
    if not isinstance(t, int):
        for c in t:
            _walk_levels(c, prod, False, out)
    out.append((t, prod, mu, degree(t) + 1, root))


def rs_units(t: Tree) -> Tuple[int, int]:
    """(rescale units before relinearisation, units after it).  One unit is
    a mu-level rescale of one polynomial (Algorithm 1 costs about one single
    rescale whatever mu is); Table II prints them as a + b."""
    nodes: list = []
    _walk_levels(t, -depth(t), True, nodes)
    pre = sum(npoly for _, _, mu, npoly, root in nodes if mu > 0 and not root)
    fin = 2 if fan(t) > 1 else 0
    return pre, fin


def ntt_counts(t: Tree) -> Tuple[Tuple[int, int], Tuple[int, int]]:
    """((a, b), (c, d)): (I)NTTs before relinearisation a L - b and after it
    c (L - d).  A mu-level rescale of one polynomial at level l takes mu
    INTTs and l - mu NTTs (Algorithm 1), l in total."""
    nodes: list = []
    _walk_levels(t, -depth(t), True, nodes)
    a = b = 0
    c = d = 0
    for _, prod, mu, npoly, root in nodes:
        if mu == 0:
            continue
        if root:
            c, d = 2, -prod
        else:
            a += npoly
            b += -prod * npoly
    return (a, b), (c, d)


# ---------------------------------------------------------------- partitions

def _int_partitions(n: int, largest: int):
    if n == 0:
        yield ()
        return
    for p in range(min(n, largest), 0, -1):
        for rest in _int_partitions(n - p, p):
            yield (p,) + rest


@functools.lru_cache(maxsize=None)
def _best(n: int, max_depth: int, root: bool):
    """(units, tree) minimising rescale units over trees of n inputs whose
    depth is at most max_depth; None if there is none.  Ties keep the first
    candidate: a single group before any split, splits with larger first
    parts first."""
    best = None
    if n - 1 <= max_depth:
        best = (0 if (root or n == 1) else n + 1, n)
    for parts in _int_partitions(n, n):
        m = len(parts)
        if m < 2 or m - 1 > max_depth:
            continue
        subs = [_best(p, max_depth - (m - 1), False) for p in parts]
        if any(s is None for s in subs):
            continue
        units = sum(s[0] for s in subs) + (0 if root else n + 1)
        if best is None or units < best[0]:
            best = (units, tuple(s[1] for s in subs))
    return best


def plan(n: int) -> Tree:
    """A partition of n inputs with the fewest rescale units among those of
    depth ceil(log2 n) (Sec. V-C: depth of each group at most
    ceil(log2 n) - (m - 1))."""
    if n < 2:
        raise ValueError("n >= 2")
    return _best(n, math.ceil(math.log2(n)), True)[1]


def binary_plan(n: int) -> Tree:
    """Table II's binary partitions: the largest power of two below n, then
    the rest, recursively, down to groups of two or one inputs."""
    if n <= 2:
        return n
    p = 1 << (math.ceil(math.log2(n)) - 1)
    return (binary_plan(p), binary_plan(n - p))


# ---------------------------------------------------------------- arithmetic

def poly_product(polys: List[np.ndarray], qs) -> np.ndarray:
    """Product of polynomials in s whose coefficients are NTT-domain
    residues ([deg + 1, l, N] each): coefficient t of the product is the sum
    over t_1 + ... + t_m = t of the pointwise products (Sec. V-A)."""
    qc = np.array(qs, dtype=np.uint64).reshape(-1, 1)
    out = np.asarray(polys[0], dtype=np.uint64)
    for f in polys[1:]:
        f = np.asarray(f, dtype=np.uint64)
        nxt = np.zeros((out.shape[0] + f.shape[0] - 1,) + out.shape[1:], dtype=np.uint64)
        for i in range(out.shape[0]):
            for j in range(f.shape[0]):
                nxt[i + j] = (nxt[i + j] + (out[i] * f[j]) % qc) % qc
        out = nxt
    return out


def _eval(prm: Params, t: Tree, cts, pos: int, end: int, dropped: list):
    """Evaluates a non-root subtree so that it ends at level `end`; returns
    (polynomials [deg+1, end, N], next input position)."""
    mu = fan(t) - 1
    prod_level = end + mu
    qs = prm.q[:prod_level]
    if isinstance(t, int):
        group = [np.asarray(c, dtype=np.uint64)[:, :prod_level] for c in cts[pos:pos + t]]
        P = tensor(group, qs) if t > 1 else group[0]
        pos += t
    else:
        parts = []
        for c in t:
            sub, pos = _eval(prm, c, cts, pos, prod_level, dropped)
            parts.append(sub)
        P = poly_product(parts, qs)
    if mu == 0:
        return P, pos
    dropped.extend(prm.q[end:prod_level])
    return np.stack([multi_rs_alg1(prm, P[i], prod_level, mu) for i in range(P.shape[0])]), pos


def mul_tree(prm: Params, keys: Keys, cts, level: int, t: Tree):
    """The n-input multiply of the tree t on NTT-domain ciphertexts at
    `level`.  Returns (ciphertext [2, out_level, N], out_level, primes
    dropped by every rescale of the tree, so that the output scale is
    Delta^n over their product)."""
    check(t)
    n = n_inputs(t)
    if len(cts) != n or n < 2:
        raise ValueError("the tree takes %d inputs" % n)
    if n > keys.k_max:
        raise ValueError("keys up to s^%d needed" % n)
    out_level = level - depth(t)
    if out_level < 1:
        raise ValueError("the tree is deeper than the level allows")
    mu = fan(t) - 1
    prod_level = out_level + mu
    qs = prm.q[:prod_level]
    dropped: list = []
    if isinstance(t, int):
        D = tensor([np.asarray(c, dtype=np.uint64)[:, :prod_level] for c in cts], qs)
    else:
        parts, pos = [], 0
        for c in t:
            sub, pos = _eval(prm, c, cts, pos, prod_level, dropped)
            parts.append(sub)
        D = poly_product(parts, qs)
    y0, y1 = relin_relocated(prm, keys, D, prod_level)
    lo, plo = prm.q[:out_level], prm.psi_q[:out_level]
    dropped.extend(prm.q[out_level:prod_level])
    r0 = _ntt.ntt(multi_rs_coeff(prm, y0, prod_level, mu), lo, plo)
    r1 = _ntt.ntt(multi_rs_coeff(prm, y1, prod_level, mu), lo, plo)
    return np.stack([r0, r1]), out_level, dropped
