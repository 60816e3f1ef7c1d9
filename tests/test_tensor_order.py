"""The job-table launches' job-adjacent block orders, checked on the CPU.

The jobs of a launch (the tensor launch of a run of equal k; the
key-product launch over the whole table) are ranked by level, descending;
rank i has G_i groups of 8 units.  Blocks are ordered by unit group, then by
rank, 8 blocks (one per XCD) per rank and group.  Each rank carries G_i and
the block group where its segment starts; a block finds its rank by binary
search.  This module restates the plan's segment bases and the kernels'
decoding (internal.h seg_block, api.hip plan_jobs) and checks that the
blocks cover every (rank, unit) exactly once, each unit's blocks on one
XCD, the ranks of a unit back to back."""

import os
import random

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2601_15401_amd", "csrc")


def bases(groups):
    n = len(groups)
    base = [0] * n
    for r in range(n - 2, -1, -1):
        g_next = groups[r + 2] if r + 2 < n else 0
        base[r] = base[r + 1] + (groups[r + 1] - g_next) * (r + 2)
    return base


def block(groups, base, b):
    n = len(groups)
    xcd, seq = b & 7, b >> 3
    lo, hi = 0, n - 1
    while lo < hi:
        mid = (lo + hi) >> 1
        if base[mid] <= seq:
            hi = mid
        else:
            lo = mid + 1
    i = lo
    g_lo = groups[i + 1] if i + 1 < n else 0
    off = seq - base[i]
    return off % (i + 1), (g_lo + off // (i + 1)) * 8 + xcd


def test_source_holds_the_same_steps():
    internal = " ".join(open(os.path.join(CSRC, "internal.h")).read().split())
    for text in ("const int g_lo = r + 1 < n ? jt[r + 1].seg[ORDER].groups : 0;",
                 "const int off = seq - jt[r].seg[ORDER].base;",
                 "rank = off % (r + 1);",
                 "unit = (g_lo + off / (r + 1)) * 8 + xcd;",
                 "if (jt[mid].seg[ORDER].base <= seq) hi = mid; else lo = mid + 1;"):
        assert text in internal, text
    api = " ".join(open(os.path.join(CSRC, "api.hip")).read().split())
    for text in ("jt[r1 - 1].seg[order].base = 0;",
                 "const int g_next = r + 2 < r1 ? jt[r + 2].seg[order].groups : 0;",
                 "jt[r].seg[order].base = jt[r + 1].seg[order].base + (jt[r + 1].seg[order].groups - g_next) * (i + 2);",
                 "jobs[a].k != jobs[b].k ? jobs[a].k < jobs[b].k : jobs[a].level > jobs[b].level;",
                 "return jt[a].level > jt[b].level;"):
        assert text in api, text


def test_every_unit_once_and_jobs_adjacent():
    rng = random.Random(2601)
    for _ in range(2000):
        n = rng.randint(1, 12)
        tiles = rng.choice([1, 2, 4, 16, 64])
        levels = sorted((rng.randint(2, 32) for _ in range(n)), reverse=True)
        if rng.random() < 0.3:
            levels = [levels[0]] * n
        groups = [(tiles * lv + 7) // 8 for lv in levels]
        base = bases(groups)
        seen = {}
        for b in range(8 * sum(groups)):
            j, u = block(groups, base, b)
            assert 0 <= j < n and 0 <= u < 8 * groups[j]
            assert (j, u) not in seen
            assert b % 8 == u % 8
            seen[(j, u)] = b
        assert len(seen) == 8 * sum(groups)
        # the jobs of one unit group take consecutive block groups
        for g in range(max(groups)):
            seqs = sorted(seen[(j, 8 * g)] >> 3 for j in range(n) if groups[j] > g)
            assert seqs == list(range(seqs[0], seqs[0] + len(seqs)))
