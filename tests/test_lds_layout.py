"""LDS tile layouts of the transform kernels, checked on the CPU.

A tile of 2^LOGR rows by COLS columns sits in LDS as blocks of 2^RB1 rows
(one consecutive-round item per column): element (r, c) at
(r >> RB1) BP + (r mod 2^RB1) PAD + c, with PAD = COLS + 32 >> RB1 (or a
given pitch) and BP = 2^RB1 PAD + XPAD.  This module restates that rule, checks that it is
a one-to-one map into the tile's words, and runs every round's lane map
through a bank model (32 banks of 4 bytes; a 32-bit access is served a
half-wave of 32 lanes at a time, and lanes of a half-wave on one bank
serialise unless they read the same word).  The extra block pitches
(XPAD) and the fused tensor kernel's row pitch are read from the kernel
sources so that a change there must pass the same checks."""

import os
import re

import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2601_15401_amd", "csrc")


def geo(logr, tl, xp, pd=-1):
    cols = 1 << (tl - logr)
    rb0 = 3 if logr == 6 else 4
    rb1 = logr - rb0
    pad = pd if pd >= 0 else cols + (32 >> rb1)
    xpad = xp if xp >= 0 else (0 if cols >= 32 else cols)
    bp = (pad << rb1) + xpad
    return dict(cols=cols, logc=tl - logr, rb0=rb0, rb1=rb1, pad=pad, bp=bp, words=bp << rb0)


def addr(g, r, c):
    return (r >> g["rb1"]) * g["bp"] + (r & ((1 << g["rb1"]) - 1)) * g["pad"] + c


def worst(addrs):
    """Largest number of distinct words one bank serves in one half-wave."""
    w = 1
    for h in range(0, len(addrs), 32):
        per_bank = {}
        for a in set(addrs[h:h + 32]):
            per_bank[a % 32] = per_bank.get(a % 32, 0) + 1
        w = max(w, max(per_bank.values()))
    return w


def strided(g, tl, nt, passb):
    """Rows lo + j 2^RB1 of column c; pass B walks the rows of a column with
    consecutive lanes, pass A the columns of a row."""
    items = (1 << tl) >> g["rb0"]
    res = 1
    for i in range(max(1, items // nt)):
        for j in range(1 << g["rb0"]):
            a = []
            for t in range(min(nt, items)):
                it = i * nt + t
                if passb:
                    lo, c = it & ((1 << g["rb1"]) - 1), it >> g["rb1"]
                else:
                    c, lo = it & (g["cols"] - 1), it >> g["logc"]
                a.append(addr(g, lo + (j << g["rb1"]), c))
            res = max(res, worst(a))
    return res


def consecutive(g, tl, nt):
    """Rows hi 2^RB1 + j of column c, lanes over (column, row block)."""
    items = (1 << tl) >> g["rb1"]
    res = 1
    for i in range(max(1, items // nt)):
        for j in range(1 << g["rb1"]):
            a = []
            for t in range(min(nt, items)):
                it = i * nt + t
                c, hi = it & (g["cols"] - 1), it >> g["logc"]
                a.append(addr(g, (hi << g["rb1"]) + j, c))
            res = max(res, worst(a))
    return res


def product_stores(g, logr, tl, nt):
    """The fused tensor kernel's stores: a lane writes residues 4l .. 4l + 3,
    four rows of one column."""
    res = 1
    for step in range(1 << (tl - 10)):
        for m in range(4):
            a = []
            for t in range(nt):
                e = 4 * (step * nt + t)
                a.append(addr(g, (e & ((1 << logr) - 1)) + m, e >> logr))
            res = max(res, worst(a))
    return res


def tensor_pad(logr, tl):
    """tib_pad(logr, tl) as written in tensor.hip: rows of COLS words (no
    padding) for 1024-residue tiles in blocks of 2^7 or 2^8 rows, the padded
    pitch otherwise."""
    src = " ".join(open(os.path.join(CSRC, "tensor.hip")).read().split())
    assert "constexpr int tib_pad(int logr, int tl) { return tl == 10 && logr >= 7 ? 1 << (tl - logr) : -1; }" in src
    assert "using TibGeo = Geo<LOGR, TL, tib_xpad(LOGR, TL), tib_pad(LOGR, TL)>;" in src
    return 1 << (tl - logr) if tl == 10 and logr >= 7 else -1


def tensor_geo(logr, tl):
    return geo(logr, tl, tensor_xpad_table()[(logr, tl)], tensor_pad(logr, tl))


def tensor_xpad_table():
    """tib_xpad(logr, tl) as written in tensor.hip."""
    src = open(os.path.join(CSRC, "tensor.hip")).read()
    m = re.search(r"constexpr int tib_xpad\(int logr, int tl\) \{\s*return (.*?);\s*\}", src, re.S)
    assert m, "tib_xpad not found"
    expr = " ".join(m.group(1).split())
    want = "logr == 8 ? (tl == 10 ? A : tl == 11 ? B : C) : logr == 7 ? (tl == 10 ? D : E) : F"
    pat = re.escape(want)
    for ch in "ABCDEF":
        pat = pat.replace(ch, r"(\d+)")
    mm = re.fullmatch(pat, expr)
    assert mm, "unexpected form of tib_xpad: " + expr
    a, b, c, d, e, f = (int(v) for v in mm.groups())
    table = {}
    for tl in (10, 11, 12):
        table[(8, tl)] = a if tl == 10 else (b if tl == 11 else c)
        table[(7, tl)] = d if tl == 10 else e
        table[(6, tl)] = f
    return table


def test_rule_matches_the_header():
    """The layout rule restated above is the one ntt_core.h compiles."""
    src = " ".join(open(os.path.join(CSRC, "ntt_core.h")).read().split())
    for text in ("static constexpr int PAD = PD >= 0 ? PD : COLS + (32 >> (LOGR - RB0));",
                 "static constexpr int XPAD = XP >= 0 ? XP : (COLS >= 32 ? 0 : COLS);",
                 "static constexpr int BP = (PAD << RB1) + XPAD;",
                 "static constexpr int LDS_WORDS = BP << RB0;",
                 "return (r >> RB1) * BP + (r & ((1 << RB1) - 1)) * PAD + c;",
                 "static constexpr int RB0 = (LOGR == 6) ? 3 : 4;"):
        assert text in src, text


def test_layout_is_one_to_one():
    cases = [(lr, 13, 0, -1) for lr in (5, 6, 7, 8)] + [(lr, 10, -1, -1) for lr in (6, 7, 8)]
    cases += [(lr, tl, xp, tensor_pad(lr, tl)) for (lr, tl), xp in tensor_xpad_table().items()]
    for logr, tl, xp, pd in cases:
        g = geo(logr, tl, xp, pd)
        seen = {addr(g, r, c) for r in range(1 << logr) for c in range(g["cols"])}
        assert len(seen) == (1 << logr) * g["cols"], (logr, tl, xp)
        assert max(seen) < g["words"], (logr, tl, xp)


@pytest.mark.parametrize("logr", [5, 6, 7, 8])
def test_transform_tiles_conflict_free(logr):
    """8192-element tiles (transform passes, ModUp): no extra block pitch,
    every round of both passes conflict-free."""
    g = geo(logr, 13, -1)
    assert g["bp"] == g["pad"] << g["rb1"]  # plain rows of PAD words
    assert strided(g, 13, 256, False) == 1
    assert strided(g, 13, 256, True) == 1
    assert consecutive(g, 13, 256) == 1


@pytest.mark.parametrize("logr", [6, 7, 8])
def test_key_product_tiles_conflict_free(logr):
    """1024-element tiles, one wave: pass B's two rounds conflict-free."""
    g = geo(logr, 10, -1)
    assert strided(g, 10, 64, True) == 1
    assert consecutive(g, 10, 64) == 1
    # the plain row pitch put every row block of a half-wave on the same
    # COLS banks
    plain = dict(g, bp=g["pad"] << g["rb1"])
    assert consecutive(plain, 10, 64) > 1


@pytest.mark.parametrize("logr,tl", [(lr, tl) for lr in (6, 7, 8) for tl in (10, 11, 12)])
def test_tensor_tiles_at_most_two_way(logr, tl):
    g = tensor_geo(logr, tl)
    if tensor_pad(logr, tl) >= 0:
        # unpadded rows: the tile takes 1024 + 2^RB0 XPAD words, and every
        # access pattern has at most two lanes of a half-wave on one bank
        assert g["pad"] == g["cols"] and g["words"] == 1024 + (g["bp"] - (g["pad"] << g["rb1"])) * (1 << g["rb0"])
        assert g["words"] < geo(logr, tl, 0)["words"] * 0.75
        assert strided(g, tl, 256, True) <= 2
    else:
        assert strided(g, tl, 256, True) == 1
    assert consecutive(g, tl, 256) <= 2
    assert product_stores(g, logr, tl, 256) <= 2
    # fewer conflicts than rows of the same pitch with no extra block pitch
    plain = dict(g, bp=g["pad"] << g["rb1"])
    ours = strided(g, tl, 256, True) + consecutive(g, tl, 256) + product_stores(g, logr, tl, 256)
    assert ours < strided(plain, tl, 256, True) + consecutive(plain, tl, 256) + product_stores(plain, logr, tl, 256)


def tw_pos(rb0, sl, rr):
    if sl < rb0:
        return rr
    u = sl - rb0
    return ((rr & ((1 << u) - 1)) << rb0) + (rr >> u)


def tw_rr(rb0, sl, pos):
    """The staging loop's inverse of tw_pos."""
    u = sl - rb0
    return pos if u < 0 else ((pos & ((1 << rb0) - 1)) << u) + (pos >> rb0)


@pytest.mark.parametrize("logr", [6, 7, 8])
def test_staged_twiddle_order(logr):
    """Consecutive-round twiddles: one-to-one per stage, undone by the
    staging loop, and read by the lanes of a half-wave at consecutive
    entries (an item with row block hi reads block hi 2^u + g at stage
    RB0 + u, for each g)."""
    rb0 = 3 if logr == 6 else 4
    for sl in range(logr):
        pos = [tw_pos(rb0, sl, rr) for rr in range(1 << sl)]
        assert sorted(pos) == list(range(1 << sl))
        assert all(tw_rr(rb0, sl, p) == rr for rr, p in enumerate(pos))
    for tl, nt in ((10, 64), (10, 256), (11, 256), (12, 256)):
        g = geo(logr, tl, -1)
        items = (1 << tl) >> g["rb1"]
        for u in range(logr - rb0):
            sl = rb0 + u
            for gg in range(1 << u):
                ent = []
                for t in range(min(nt, items)):
                    c, hi = t & (g["cols"] - 1), t >> g["logc"]
                    ent.append(tw_pos(rb0, sl, (hi << u) + gg) * g["cols"] + c)
                for h in range(0, len(ent), 32):
                    half = ent[h:h + 32]
                    assert half == list(range(half[0], half[0] + len(half))), (logr, tl, sl, gg)
