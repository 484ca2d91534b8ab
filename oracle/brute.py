"""Brute-force join and verification -- TEST INFRASTRUCTURE ONLY.

Pure-Python restatement of the problem (paper Sec. 3, Definition 1) with the
Jaccard similarity of Table 1: a pair is similar iff
|r & s| / |r | s| >= t, evaluated with Python sets and exact rationals.  Meant
for tiny collections only (quadratic in the number of sets).
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence, Tuple


def _sets(offsets, tokens) -> List[frozenset]:
    return [frozenset(int(x) for x in tokens[int(offsets[i]):int(offsets[i + 1])])
            for i in range(len(offsets) - 1)]


def jaccard(a: frozenset, b: frozenset) -> Fraction:
    return Fraction(len(a & b), len(a | b))


def brute_join(offsets, tokens, t_num: int, t_den: int) -> List[Tuple[int, int]]:
    """All (i, j) with i > j and J(set_i, set_j) >= t, ascending by (i, j)."""
    sets = _sets(offsets, tokens)
    t = Fraction(t_num, t_den)
    out = []
    for i in range(len(sets)):
        for j in range(i):
            if jaccard(sets[i], sets[j]) >= t:
                out.append((i, j))
    return out


def brute_verify(offsets, tokens, pairs: Sequence[Sequence[int]], t_num: int, t_den: int):
    """Per-pair decision (list of bool) and overlap (list of int)."""
    sets = _sets(offsets, tokens)
    t = Fraction(t_num, t_den)
    dec, ov = [], []
    for r, s in pairs:
        a, b = sets[int(r)], sets[int(s)]
        ov.append(len(a & b))
        dec.append(jaccard(a, b) >= t)
    return dec, ov
