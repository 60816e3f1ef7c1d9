"""Operation counters (oracle side).

Test infrastructure only (see ``oracle/__init__``).

Counts limb transforms ("ntt", "intt", one per limb of one polynomial) and
constant multiplications in the rescaling step ("rs_const", one per limb of
one polynomial), so tests can compare the oracle's data path with the counts
the paper tabulates (Table IV, Table V).
"""
from __future__ import annotations

from collections import Counter
from contextlib import contextmanager

_C = Counter()


def add(name: str, n: int = 1) -> None:
    _C[name] += n


def snapshot() -> dict:
    return dict(_C)


def reset() -> None:
    _C.clear()


@contextmanager
def counting():
    reset()
    box = {}
    try:
        yield box
    finally:
        box.update(snapshot())
