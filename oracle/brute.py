"""Brute-force join and verification -- TEST INFRASTRUCTURE ONLY.

Pure-Python restatement of the problem (paper Sec. 3, Definition 1) with the
similarity functions of Table 1, evaluated with Python sets and exact
rationals: Jaccard |r & s| / |r | s|, Dice 2|r & s| / (|r| + |s|), Overlap
|r & s|, and Cosine |r & s| / sqrt(|r||s|), whose comparison with t is made
on the squares (both sides are non-negative).  Meant for tiny collections
only (quadratic in the number of sets).
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence, Tuple


def _sets(offsets, tokens) -> List[frozenset]:
    return [frozenset(int(x) for x in tokens[int(offsets[i]):int(offsets[i + 1])])
            for i in range(len(offsets) - 1)]


def jaccard(a: frozenset, b: frozenset) -> Fraction:
    return Fraction(len(a & b), len(a | b))


def similar(a: frozenset, b: frozenset, t: Fraction, sim: str = "jaccard") -> bool:
    """sim(a, b) >= t, exactly."""
    o = len(a & b)
    if sim == "jaccard":
        return jaccard(a, b) >= t
    if sim == "dice":
        return Fraction(2 * o, len(a) + len(b)) >= t
    if sim == "cosine":
        return Fraction(o * o, len(a) * len(b)) >= t * t
    if sim == "overlap":
        return o >= t
    raise ValueError(sim)


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


def brute_verify(offsets, tokens, pairs: Sequence[Sequence[int]], t_num: int, t_den: int,
                 sim: str = "jaccard"):
    """Per-pair decision (list of bool) and overlap (list of int)."""
    sets = _sets(offsets, tokens)
    t = Fraction(t_num, t_den)
    dec, ov = [], []
    for r, s in pairs:
        a, b = sets[int(r)], sets[int(s)]
        ov.append(len(a & b))
        dec.append(similar(a, b, t, sim))
    return dec, ov


def brute_verify_rs(offsets_r, tokens_r, offsets_s, tokens_s, pairs: Sequence[Sequence[int]],
                    t_num: int, t_den: int, sim: str = "jaccard"):
    """Per-pair decision of an R-S join (r a set of R, s a set of S)."""
    sets_r, sets_s = _sets(offsets_r, tokens_r), _sets(offsets_s, tokens_s)
    t = Fraction(t_num, t_den)
    return [similar(sets_r[int(r)], sets_s[int(s)], t, sim) for r, s in pairs]
