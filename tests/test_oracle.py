"""Pins of the verification oracle against what the paper and the mathematics fix.

Everything here runs on the CPU.  The oracle (full-merge overlap plus the
exact Jaccard test, paper Sec. 3 Definition 1 / Table 1) is checked against:
hand-worked examples (tests/golden/paper_examples.json), an independent
brute force with Python sets and exact rationals, closed forms and
invariants.  A plausible slip in the oracle (dropped term, wrong sign,
swapped operand, strict instead of non-strict comparison) fails at least one
of these.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
from ssj_inputs import synth
from ssj_inputs import filter as cfilter


def _expand(v):
    if isinstance(v, list):
        return v
    out = []
    for part in v.split("+"):
        part = part.strip()
        assert part.startswith("range(")
        a, b = part[len("range("):-1].split(",")
        out.extend(range(int(a), int(b)))
    return out


def _coll(*sets):
    return synth.collection_from_sets([sorted(s) for s in sets])


@pytest.fixture(scope="module")
def examples(golden_dir):
    with open(os.path.join(golden_dir, "paper_examples.json")) as f:
        return json.load(f)


def table1_alpha(t_num, t_den, nr, ns):
    """Jaccard row of Table 1 in exact rationals."""
    t = Fraction(t_num, t_den)
    return math.ceil(t / (1 + t) * (nr + ns))


def test_required_overlap_examples(examples):
    for ex in examples["required_overlap"]:
        assert table1_alpha(ex["t_num"], ex["t_den"], ex["size_r"], ex["size_s"]) == ex["alpha"], ex["cite"]


def test_float_trap_documented():
    # Table 1 evaluated in binary floating point mis-rounds alpha; the exact
    # rational value is 28 (Sec. 2.2 / Table 1).  This is why every threshold
    # is carried as t_num / t_den and tested in integers.
    assert math.ceil(0.8 / 1.8 * 63) == 29
    assert table1_alpha(4, 5, 32, 31) == 28


def test_pair_examples(examples):
    for ex in examples["pairs"]:
        r, s = _expand(ex["r"]), _expand(ex["s"])
        c = _coll(r, s)
        pairs = np.array([[0, 1], [1, 0]], dtype=np.int32)
        passed, ov = oracle.verify(c.offsets, c.tokens, pairs, ex["t_num"], ex["t_den"], with_overlap=True)
        assert list(ov) == [ex["overlap"]] * 2, ex["cite"]
        assert [bool(x) for x in passed] == [ex["similar"]] * 2, ex["cite"]
        dec, bov = brute.brute_verify(c.offsets, c.tokens, pairs, ex["t_num"], ex["t_den"])
        assert dec == [ex["similar"]] * 2 and bov == [ex["overlap"]] * 2, ex["cite"]


def test_merge_trace_examples(examples):
    for ex in examples["merge_trace"]:
        c = _coll(ex["r"], ex["s"])
        cr, cs, dec = oracle.merge_trace(c.offsets, c.tokens, np.array([[0, 1]]), ex["t_num"], ex["t_den"])
        assert (int(cr[0]), int(cs[0]), bool(dec[0])) == (ex["c_r"], ex["c_s"], ex["decided"]), ex["cite"]


def _random_pairs(rng, n_sets, n):
    return rng.integers(0, n_sets, size=(n, 2)).astype(np.int32)


@pytest.mark.parametrize("seed", range(12))
def test_oracle_equals_brute_random_pairs(seed):
    rng = np.random.default_rng(1000 + seed)
    c = synth.random_collection(rng, n_sets=60, max_size=12, universe=40, zipf_s=0.8)
    pairs = _random_pairs(rng, c.n_sets, 400)
    pairs[:20, 1] = pairs[:20, 0]  # self pairs
    pairs = np.concatenate([pairs, pairs[:30], pairs[:30, ::-1]])  # duplicates, reversed
    for (tn, td) in [(0, 1), (1, 5), (1, 2), (3, 5), (2, 3), (7, 10), (3, 4), (4, 5), (9, 10), (1, 1)]:
        passed, ov = oracle.verify(c.offsets, c.tokens, pairs, tn, td, with_overlap=True)
        dec, bov = brute.brute_verify(c.offsets, c.tokens, pairs, tn, td)
        assert list(ov) == bov
        assert [bool(x) for x in passed] == dec


@pytest.mark.parametrize("seed", range(6))
def test_filter_plus_oracle_equals_brute_join(seed):
    rng = np.random.default_rng(2000 + seed)
    c = synth.random_collection(rng, n_sets=200, max_size=10, universe=60, zipf_s=1.0, min_size=1)
    for (tn, td) in [(1, 2), (3, 5), (7, 10), (4, 5), (9, 10), (1, 1)]:
        cand = cfilter.candidates(c.offsets, c.tokens, tn, td)
        got = oracle.select(c.offsets, c.tokens, cand, tn, td)
        want = brute.brute_join(c.offsets, c.tokens, tn, td)
        assert sorted(map(tuple, got.tolist())) == want
        # filter safety: every similar pair is a candidate
        cand_set = set(map(tuple, cand.tolist()))
        assert all(p in cand_set for p in want)


def test_config1_join_equals_brute():
    w = synth.WORKLOADS[1]
    c = synth.workload_collection(1)
    (tn, td), = w.thresholds
    cand = cfilter.workload_candidates(1, tn, td)
    got = oracle.select(c.offsets, c.tokens, cand, tn, td)
    want = brute.brute_join(c.offsets, c.tokens, tn, td)
    assert sorted(map(tuple, got.tolist())) == want
    # The tiny workload has no similar pair at t = 0.8 (random Zipf sets);
    # near-duplicate collections below cover passing pairs.


@pytest.mark.parametrize("seed", range(3))
def test_near_duplicates_join_equals_brute(seed):
    rng = np.random.default_rng(4000 + seed)
    c = synth.near_duplicate_collection(rng, n_base=40, copies=4, max_size=14, universe=400,
                                        change_frac=0.15)
    for (tn, td) in [(1, 2), (7, 10), (4, 5), (9, 10)]:
        cand = cfilter.candidates(c.offsets, c.tokens, tn, td)
        got = oracle.select(c.offsets, c.tokens, cand, tn, td)
        want = brute.brute_join(c.offsets, c.tokens, tn, td)
        assert sorted(map(tuple, got.tolist())) == want
        if (tn, td) == (1, 2):
            assert len(want) > 50


@pytest.mark.parametrize("seed", range(4))
def test_invariants(seed):
    rng = np.random.default_rng(3000 + seed)
    c = synth.random_collection(rng, n_sets=80, max_size=20, universe=50, zipf_s=0.7)
    pairs = _random_pairs(rng, c.n_sets, 2000)
    sizes = c.sizes()
    ts = [(1, 5), (1, 2), (3, 5), (7, 10), (4, 5), (9, 10), (1, 1)]
    prev = None
    for (tn, td) in ts:
        p, ov = oracle.verify(c.offsets, c.tokens, pairs, tn, td, with_overlap=True)
        q = oracle.verify(c.offsets, c.tokens, pairs[:, ::-1], tn, td)
        assert np.array_equal(p, q)  # I1 symmetry
        nr, ns = sizes[pairs[:, 0]], sizes[pairs[:, 1]]
        alpha = np.array([table1_alpha(tn, td, a, b) for a, b in zip(nr, ns)])
        assert np.array_equal(p.astype(bool), ov >= alpha)  # I2 pass <=> o >= alpha
        # I6 length filter holds for every passing pair
        pb = p.astype(bool)
        assert np.all(tn * nr[pb] <= td * ns[pb]) and np.all(tn * ns[pb] <= td * nr[pb])
        if prev is not None:
            assert np.all(p <= prev)  # I3 monotone in t
        prev = p
        # the early-terminating merge reaches the same decision (Sec. 3.1)
        cr, cs, dec = oracle.merge_trace(c.offsets, c.tokens, pairs, tn, td)
        assert np.array_equal(dec, p)
        assert np.all(cr <= nr) and np.all(cs <= ns) and np.all(cr >= 0) and np.all(cs >= 0)
    # I4: t = 1 passes exactly the equal sets
    p1 = oracle.verify(c.offsets, c.tokens, pairs, 1, 1)
    eq = np.array([np.array_equal(c.set(a), c.set(b)) for a, b in pairs])
    assert np.array_equal(p1.astype(bool), eq)


def test_identical_and_disjoint():
    c = _coll([1, 5, 9], [1, 5, 9], [2, 3, 4], [100, 200])
    pairs = np.array([[0, 1], [0, 0], [0, 2], [3, 2]], dtype=np.int32)
    for (tn, td) in [(1, 100), (1, 2), (1, 1)]:
        p = oracle.verify(c.offsets, c.tokens, pairs, tn, td)
        assert list(p) == [1, 1, 0, 0]  # I5


def test_subset_closed_form():
    # r subset of s: J = |r| / |s|
    rng = np.random.default_rng(7)
    for _ in range(50):
        s = sorted(rng.choice(1000, size=int(rng.integers(2, 60)), replace=False).tolist())
        k = int(rng.integers(1, len(s) + 1))
        r = sorted(rng.choice(s, size=k, replace=False).tolist())
        c = _coll(r, s)
        for (tn, td) in [(1, 2), (3, 4), (9, 10)]:
            p = oracle.verify(c.offsets, c.tokens, np.array([[0, 1]]), tn, td)
            assert bool(p[0]) == (Fraction(len(r), len(s)) >= Fraction(tn, td))


def test_oracle_rejects_bad_input():
    c = _coll([1, 2], [2, 3])
    with pytest.raises(oracle.OracleError):
        oracle.verify(c.offsets, c.tokens, np.array([[0, 2]]), 1, 2)
    with pytest.raises(oracle.OracleError):
        oracle.verify(c.offsets, c.tokens, np.array([[-1, 0]]), 1, 2)
    for tn, td in [(3, 2), (-1, 2), (1, 0)]:
        with pytest.raises(oracle.OracleError):
            oracle.verify(c.offsets, c.tokens, np.array([[0, 1]]), tn, td)


def test_oracle_threads_agree():
    c = synth.workload_collection(2)
    cand = cfilter.workload_candidates(2, 7, 10)
    a = oracle.verify(c.offsets, c.tokens, cand, 7, 10, n_threads=1)
    b = oracle.verify(c.offsets, c.tokens, cand, 7, 10, n_threads=4)
    assert np.array_equal(a, b)


def test_select_keeps_order_and_multiplicity():
    c = _coll([1, 2, 3], [1, 2, 3], [7, 8])
    pairs = np.array([[1, 0], [2, 0], [0, 1], [1, 0]], dtype=np.int32)
    out = oracle.select(c.offsets, c.tokens, pairs, 1, 2)
    assert out.tolist() == [[1, 0], [0, 1], [1, 0]]


# ---------------------------------------------------------------------------
# The other similarity functions of Table 1 (Cosine, Dice, Overlap).

SIMS = ("jaccard", "cosine", "dice", "overlap")


def table1_equivalent_overlap(sim, t_num, t_den, nr, ns):
    """The "Equivalent Overlap" column of Table 1, in exact rationals."""
    t = Fraction(t_num, t_den)
    if sim == "jaccard":
        return math.ceil(t / (1 + t) * (nr + ns))
    if sim == "dice":
        return math.ceil(t * (nr + ns) / 2)
    if sim == "overlap":
        return math.ceil(t)
    # cosine: ceil(t sqrt(nr ns)), i.e. the least o >= 0 with o >= t sqrt(nr ns)
    x = t * t * nr * ns  # = (t sqrt(nr ns))^2
    o = math.isqrt(x.numerator // x.denominator)
    while Fraction(o * o) < x:
        o += 1
    return o


def test_sim_required_overlap_examples(examples):
    for ex in examples["sim_required_overlap"]:
        got = table1_equivalent_overlap(ex["sim"], ex["t_num"], ex["t_den"], ex["size_r"], ex["size_s"])
        assert got == ex["alpha"], ex["cite"]


def test_sim_float_traps_documented():
    # Table 1 in binary floating point rounds 55 up to 56 for t = 0.55 at these
    # sizes (Dice |r|+|s| = 200, Cosine |r| = |s| = 100); exact value 55.
    assert math.ceil(0.55 * 200 / 2) == 56
    assert math.ceil(0.55 * math.sqrt(100 * 100)) == 56
    assert table1_equivalent_overlap("dice", 11, 20, 100, 100) == 55
    assert table1_equivalent_overlap("cosine", 11, 20, 100, 100) == 55


def test_sim_pair_examples(examples):
    for ex in examples["sim_pairs"]:
        r, s = _expand(ex["r"]), _expand(ex["s"])
        c = _coll(r, s)
        pairs = np.array([[0, 1], [1, 0]], dtype=np.int32)
        passed, ov = oracle.verify(c.offsets, c.tokens, pairs, ex["t_num"], ex["t_den"],
                                   with_overlap=True, sim=ex["sim"])
        assert list(ov) == [ex["overlap"]] * 2, ex["cite"]
        assert [bool(x) for x in passed] == [ex["similar"]] * 2, ex["cite"]
        dec, bov = brute.brute_verify(c.offsets, c.tokens, pairs, ex["t_num"], ex["t_den"], sim=ex["sim"])
        assert dec == [ex["similar"]] * 2 and bov == [ex["overlap"]] * 2, ex["cite"]


SIM_THRESHOLDS = {
    "jaccard": [(0, 1), (1, 2), (3, 5), (4, 5), (11, 20), (1, 1)],
    "cosine": [(0, 1), (1, 2), (3, 5), (4, 5), (11, 20), (9, 10), (1, 1)],
    "dice": [(0, 1), (1, 2), (3, 5), (4, 5), (11, 20), (9, 10), (1, 1)],
    "overlap": [(0, 1), (1, 1), (2, 1), (5, 1), (7, 2), (12, 1)],
}


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("sim", SIMS)
def test_sim_oracle_equals_brute_and_table1(seed, sim):
    """Oracle decision = brute force (definition with Fractions) = o >= the
    Table 1 equivalent overlap, on random pairs (many near the threshold)."""
    rng = np.random.default_rng(5000 + seed)
    c = synth.near_duplicate_collection(rng, n_base=25, copies=4, max_size=14, universe=60,
                                        change_frac=0.25)
    pairs = _random_pairs(rng, c.n_sets, 400)
    sizes = np.diff(c.offsets)
    for tn, td in SIM_THRESHOLDS[sim]:
        passed, ov = oracle.verify(c.offsets, c.tokens, pairs, tn, td, with_overlap=True, sim=sim)
        dec, bov = brute.brute_verify(c.offsets, c.tokens, pairs, tn, td, sim=sim)
        assert list(ov) == bov
        assert [bool(x) for x in passed] == dec, (sim, tn, td)
        for (r, s), o, p in zip(pairs, ov, passed):
            alpha = table1_equivalent_overlap(sim, tn, td, int(sizes[r]), int(sizes[s]))
            assert bool(p) == (int(o) >= alpha), (sim, tn, td, r, s)


@pytest.mark.parametrize("seed", range(6))
def test_dice_is_jaccard_at_transformed_threshold(seed):
    """D = 2J / (1 + J), so D >= a/b  <=>  J >= a / (2b - a)."""
    rng = np.random.default_rng(6000 + seed)
    c = synth.near_duplicate_collection(rng, n_base=30, copies=4, max_size=16, universe=70,
                                        change_frac=0.3)
    pairs = _random_pairs(rng, c.n_sets, 500)
    for a, b in [(0, 1), (1, 2), (3, 5), (2, 3), (4, 5), (9, 10), (1, 1)]:
        d = oracle.verify(c.offsets, c.tokens, pairs, a, b, sim="dice")
        j = oracle.verify(c.offsets, c.tokens, pairs, a, 2 * b - a, sim="jaccard")
        assert np.array_equal(d, j), (a, b)


@pytest.mark.parametrize("seed", range(6))
def test_similarity_orderings(seed):
    """Jaccard <= Dice <= Cosine for every pair (|r|+|s|-o >= (|r|+|s|)/2 and
    the arithmetic-geometric mean inequality), with Cosine = Dice when
    |r| = |s|: so at one threshold the passing sets are nested."""
    rng = np.random.default_rng(7000 + seed)
    c = synth.near_duplicate_collection(rng, n_base=30, copies=4, max_size=16, universe=70,
                                        change_frac=0.3)
    pairs = _random_pairs(rng, c.n_sets, 500)
    sizes = np.diff(c.offsets)
    eq = sizes[pairs[:, 0]] == sizes[pairs[:, 1]]
    for tn, td in [(1, 2), (3, 5), (7, 10), (4, 5), (9, 10)]:
        j = oracle.verify(c.offsets, c.tokens, pairs, tn, td, sim="jaccard").astype(bool)
        d = oracle.verify(c.offsets, c.tokens, pairs, tn, td, sim="dice").astype(bool)
        k = oracle.verify(c.offsets, c.tokens, pairs, tn, td, sim="cosine").astype(bool)
        assert not np.any(j & ~d) and not np.any(d & ~k)
        assert np.array_equal(d[eq], k[eq])


def test_overlap_closed_forms():
    rng = np.random.default_rng(8000)
    c = synth.near_duplicate_collection(rng, n_base=20, copies=3, max_size=12, universe=40,
                                        change_frac=0.3)
    pairs = _random_pairs(rng, c.n_sets, 300)
    sizes = np.diff(c.offsets)
    _, ov = oracle.verify(c.offsets, c.tokens, pairs, 0, 1, with_overlap=True, sim="overlap")
    assert oracle.verify(c.offsets, c.tokens, pairs, 0, 1, sim="overlap").all()
    big = int(sizes.max()) + 1
    assert not oracle.verify(c.offsets, c.tokens, pairs, big, 1, sim="overlap").any()
    for k in range(0, 8):
        assert np.array_equal(oracle.verify(c.offsets, c.tokens, pairs, k, 1, sim="overlap"),
                              (ov >= k).astype(np.uint8))


def test_sim_rejects_bad_input():
    c = _coll([1, 2, 3], [2, 3, 4])
    pairs = np.array([[0, 1]], dtype=np.int32)
    for sim in ("jaccard", "cosine", "dice"):
        with pytest.raises(oracle.OracleError):
            oracle.verify(c.offsets, c.tokens, pairs, 3, 2, sim=sim)  # t > 1
    assert oracle.verify(c.offsets, c.tokens, pairs, 3, 2, sim="overlap")[0] == 1  # 2 >= 1.5
    assert oracle.verify(c.offsets, c.tokens, pairs, 5, 2, sim="overlap")[0] == 0  # 2 < 2.5
    with pytest.raises(oracle.OracleError):
        oracle.verify(c.offsets, c.tokens, pairs, 1, 0, sim="overlap")
    with pytest.raises(oracle.OracleError):
        oracle.verify(c.offsets, c.tokens, pairs, 1, 2, sim="hamming")


# --- R-S joins (Definition 1 with two collections) ---------------------------

def _two_collections(rng):
    """R and S drawn around shared base sets, so many cross pairs are similar."""
    c = synth.near_duplicate_collection(rng, n_base=20, copies=4, max_size=15, universe=60,
                                        change_frac=0.25)
    sets = [c.tokens[c.offsets[i]:c.offsets[i + 1]].tolist() for i in range(c.n_sets)]
    order = rng.permutation(len(sets))
    cut = len(sets) // 3
    r_sets = [sets[i] for i in order[:cut]]
    s_sets = [sets[i] for i in order[cut:]]
    return synth.collection_from_sets(r_sets), synth.collection_from_sets(s_sets)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("sim", ["jaccard", "cosine", "dice", "overlap"])
def test_rs_oracle_equals_brute(seed, sim):
    rng = np.random.default_rng(7000 + seed)
    R, S = _two_collections(rng)
    pairs = np.stack([rng.integers(0, R.n_sets, 500), rng.integers(0, S.n_sets, 500)],
                     axis=1).astype(np.int32)
    ts = {"overlap": [(0, 1), (3, 1), (7, 1)]}.get(sim, [(0, 1), (1, 2), (3, 5), (4, 5), (1, 1)])
    for tn, td in ts:
        got = oracle.select_rs(R.offsets, R.tokens, S.offsets, S.tokens, pairs, tn, td, sim=sim)
        dec = brute.brute_verify_rs(R.offsets, R.tokens, S.offsets, S.tokens, pairs, tn, td, sim)
        want = pairs[np.array(dec, dtype=bool)]
        assert np.array_equal(got, want), (sim, tn, td)


def test_rs_with_r_equal_s_is_the_self_join():
    rng = np.random.default_rng(7100)
    c = synth.near_duplicate_collection(rng, n_base=25, copies=4, max_size=14, universe=60,
                                        change_frac=0.25)
    pairs = _random_pairs(rng, c.n_sets, 600)
    for tn, td in [(1, 2), (3, 5), (4, 5)]:
        a = oracle.select_rs(c.offsets, c.tokens, c.offsets, c.tokens, pairs, tn, td)
        b = oracle.select(c.offsets, c.tokens, pairs, tn, td)
        assert np.array_equal(a, b)


def test_rs_is_not_symmetric_in_ids():
    """An R-S pair names a set of R and a set of S: (0, 1) and (1, 0) are
    different pairs when R and S differ."""
    R = _coll([1, 2, 3], [7, 8])
    S = _coll([9], [1, 2, 3])
    got = oracle.select_rs(R.offsets, R.tokens, S.offsets, S.tokens, [[0, 1], [1, 0], [0, 0]], 1, 1)
    assert got.tolist() == [[0, 1]]


def test_rs_rejects_ids_outside_their_collection():
    R = _coll([1, 2], [3, 4], [5, 6])
    S = _coll([1, 2])
    with pytest.raises(oracle.OracleError):
        oracle.select_rs(R.offsets, R.tokens, S.offsets, S.tokens, [[2, 1]], 1, 2)
    with pytest.raises(oracle.OracleError):
        oracle.select_rs(R.offsets, R.tokens, S.offsets, S.tokens, [[3, 0]], 1, 2)
