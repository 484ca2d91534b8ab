"""Seeded input generators and the CPU candidate filter (no GPU)."""
import numpy as np
import pytest

import oracle
from oracle import brute
from ssj_inputs import filter as cfilter
from ssj_inputs import synth


def _check_contract(c):
    off, tok = c.offsets, c.tokens
    sizes = np.diff(off)
    assert off[0] == 0 and np.all(sizes >= 1)
    assert np.all(np.diff(sizes) >= 0)  # sorted by size
    d = np.diff(tok.astype(np.int64))
    inside = np.ones(d.shape[0], dtype=bool)
    inside[off[1:-1] - 1] = False
    assert np.all(d[inside] > 0)  # strictly increasing inside a set
    assert tok.min() >= 0
    # lexicographic order among equal sizes
    for L in np.unique(sizes)[:5]:
        ids = np.nonzero(sizes == L)[0][:200]
        rows = [tuple(c.set(i)) for i in ids]
        assert rows == sorted(rows)
    # ids ascend with document frequency (rarest token first)
    df = np.bincount(tok)
    assert np.all(np.diff(df[df > 0]) >= 0)


def test_determinism():
    a = synth.make_collection(3000, ("lognormal", 12.0, 0.5, 2, 200), 1.0, 20000, seed=5, cfg=9)
    b = synth.make_collection(3000, ("lognormal", 12.0, 0.5, 2, 200), 1.0, 20000, seed=5, cfg=9)
    c = synth.make_collection(3000, ("lognormal", 12.0, 0.5, 2, 200), 1.0, 20000, seed=6, cfg=9)
    assert a.digest() == b.digest()
    assert a.digest() != c.digest()


@pytest.mark.parametrize("cfg", [1, 2])
def test_workload_contract(cfg):
    c = synth.workload_collection(cfg)
    w = synth.WORKLOADS[cfg]
    assert c.n_sets == w.n_sets
    _check_contract(c)


def test_size_laws():
    rng = np.random.default_rng(0)
    s = synth.draw_sizes(("lognormal", 12.0, 0.5, 2, 200), 200000, rng)
    assert abs(s.mean() - 12.0) < 0.1 and s.min() >= 2 and s.max() <= 200
    s = synth.draw_sizes(("uniform", 5, 15), 100000, rng)
    assert s.min() == 5 and s.max() == 15 and abs(s.mean() - 10) < 0.05
    s = synth.draw_sizes(("pareto", 1.5, 3, 5000), 400000, rng)
    assert s.min() == 3 and s.max() <= 5000
    # Pareto-I tail: P(X >= 30) = (3/30)^1.5 before flooring at integers
    assert abs((s >= 30).mean() - (3 / 30) ** 1.5) < 0.003


def test_zipf_head_frequency():
    rng = np.random.default_rng(1)
    cdf = synth.zipf_cdf(1000, 1.0)
    u = rng.random(200000)
    k = np.searchsorted(cdf, u, side="right") + 1
    h = np.sum(1.0 / np.arange(1, 1001))
    assert abs((k == 1).mean() - 1.0 / h) < 0.005
    assert abs((k == 2).mean() - 0.5 / h) < 0.004


def test_no_repeats_within_set_and_sizes_kept():
    rng = np.random.default_rng(3)
    sizes = rng.integers(1, 300, size=500)
    set_idx, rank = synth.draw_token_ranks(sizes, 400, 1.2, rng)
    assert np.array_equal(np.bincount(set_idx, minlength=500), sizes)
    key = set_idx * 1000 + rank
    assert np.unique(key).shape[0] == key.shape[0]


@pytest.mark.parametrize("seed", range(4))
def test_filter_safe_and_well_formed(seed):
    rng = np.random.default_rng(500 + seed)
    c = synth.random_collection(rng, n_sets=300, max_size=12, universe=80)
    for (tn, td) in [(1, 2), (7, 10), (9, 10)]:
        cand = cfilter.candidates(c.offsets, c.tokens, tn, td)
        assert np.all(cand[:, 0] > cand[:, 1])  # probe r after indexed s
        assert np.unique(cand, axis=0).shape[0] == cand.shape[0]  # no duplicates
        assert np.all(np.diff(cand[:, 0]) >= 0)  # grouped by probe
        sizes = c.sizes()
        nr, ns = sizes[cand[:, 0]], sizes[cand[:, 1]]
        assert np.all(td * ns >= tn * nr)  # length filter
        want = brute.brute_join(c.offsets, c.tokens, tn, td)
        cs = set(map(tuple, cand.tolist()))
        assert all(p in cs for p in want)  # I8: the filter never loses a similar pair


def test_filter_probe_batches_equal_all():
    c = synth.workload_collection(1)
    ix = cfilter.PrefixIndex(c.offsets, c.tokens, 3, 5)
    full = ix.all_candidates(n_threads=3)
    buf = np.empty((97, 2), dtype=np.int32)
    got, r = [], 0
    while r < c.n_sets:
        n, r = ix.probe(r, c.n_sets, buf)
        assert n > 0 or r == c.n_sets
        got.append(buf[:n].copy())
    assert np.array_equal(np.concatenate(got), full)
    ix.close()


def test_filter_rejects_bad_threshold():
    c = synth.workload_collection(1)
    for tn, td in [(0, 1), (3, 2), (1, 0)]:
        with pytest.raises(ValueError):
            cfilter.PrefixIndex(c.offsets, c.tokens, tn, td)


def test_stream_schedule():
    sizes, ts, _ = synth.stream_schedule(2000, seed=0)
    assert sizes.min() >= 1000 and sizes.max() <= 1_000_000
    lg = np.log10(sizes)
    assert abs(lg.mean() - 4.5) < 0.1
    assert set(ts) == {(3, 5), (4, 5), (9, 10)}


def test_serving_batches_cover_the_candidate_stream():
    """Batches cut by the serving driver are the filter's candidates, in order."""
    from paper_1812_09141_amd import serving
    rng = np.random.default_rng(77)
    c = synth.random_collection(rng, n_sets=400, max_size=12, universe=120)
    full = cfilter.candidates(c.offsets, c.tokens, 1, 2)
    sizes = [50, 120, 7, 300, 10_000]
    batches = serving.build_batches(c.offsets, c.tokens, sizes, [(1, 2)] * len(sizes), n_threads=3)
    got = np.concatenate([b[0] for b in batches])
    # the stream wraps around at the end of the collection
    k = min(got.shape[0], full.shape[0])
    assert np.array_equal(got[:k], full[:k])
    if got.shape[0] > full.shape[0]:
        assert np.array_equal(got[full.shape[0]:], full[:got.shape[0] - full.shape[0]])
    assert all(b[1:] == (1, 2) for b in batches)


# --- PPJoin's positional filter (Sec. 2.2 "Filters") -------------------------

@pytest.mark.parametrize("seed", range(6))
def test_ppjoin_safe_and_inside_allpairs(seed):
    """Every similar pair survives the positional filter (brute force), and
    its candidates are the AllPairs candidates minus some, in the same order."""
    rng = np.random.default_rng(800 + seed)
    if seed % 2:
        c = synth.near_duplicate_collection(rng, n_base=40, copies=5, max_size=18, universe=90,
                                            change_frac=0.25)
    else:
        c = synth.random_collection(rng, n_sets=300, max_size=14, universe=70)
    for (tn, td) in [(1, 3), (1, 2), (3, 5), (7, 10), (4, 5), (9, 10), (1, 1)]:
        ap = cfilter.candidates(c.offsets, c.tokens, tn, td)
        pp = cfilter.candidates(c.offsets, c.tokens, tn, td, positional=True)
        want = brute.brute_join(c.offsets, c.tokens, tn, td)
        ps = set(map(tuple, pp.tolist()))
        assert all(p in ps for p in want), (tn, td)
        # a subsequence of the AllPairs candidates
        k = 0
        for pair in ap.tolist():
            if k < pp.shape[0] and pair == pp[k].tolist():
                k += 1
        assert k == pp.shape[0], (tn, td)


def test_ppjoin_prunes_and_keeps_the_join():
    """Fewer candidates on the offline collection's thresholds, same join result."""
    c = synth.workload_collection(2)
    for (tn, td) in synth.WORKLOADS[2].thresholds:
        ap = cfilter.workload_candidates(2, tn, td)
        pp = cfilter.workload_candidates(2, tn, td, positional=True)
        assert pp.shape[0] < ap.shape[0]
        a = oracle.sort_pairs(oracle.select(c.offsets, c.tokens, ap, tn, td, n_threads=8))
        b = oracle.sort_pairs(oracle.select(c.offsets, c.tokens, pp, tn, td, n_threads=8))
        assert np.array_equal(a, b), (tn, td)


def test_ppjoin_hand_example():
    """Two 10-token sets at t = 1/2: prefixes of 10 - 5 + 1 = 6 tokens, and a
    pair needs overlap ceil(20 / 3) = 7.  x = {1..5, 50, 60..63} (set 0 by the
    lexicographic order) and y = {50..59} (set 1, the probe) share only 50,
    at position 0 of y and position 5 of x, both inside the prefixes, so
    AllPairs keeps (1, 0); the positional bound is 0 + 1 + min(9, 4) = 5 < 7,
    so PPJoin drops it.  With 50 at position 1 of x instead, the bound is
    1 + min(9, 8) = 9 and both keep the pair."""
    x = [1, 2, 3, 4, 5, 50, 60, 61, 62, 63]
    y = list(range(50, 60))
    c = synth.collection_from_sets([x, y])
    assert c.tokens[:10].tolist() == x
    assert cfilter.candidates(c.offsets, c.tokens, 1, 2).tolist() == [[1, 0]]
    assert cfilter.candidates(c.offsets, c.tokens, 1, 2, positional=True).shape[0] == 0
    x2 = [1, 50, 60, 61, 62, 63, 64, 65, 66, 67]
    c2 = synth.collection_from_sets([x2, y])
    assert c2.tokens[:10].tolist() == x2
    assert cfilter.candidates(c2.offsets, c2.tokens, 1, 2, positional=True).tolist() == [[1, 0]]


def test_ppjoin_thread_count_does_not_change_output():
    c = synth.workload_collection(1)
    a = cfilter.candidates(c.offsets, c.tokens, 3, 5, n_threads=1, positional=True)
    b = cfilter.candidates(c.offsets, c.tokens, 3, 5, n_threads=8, positional=True)
    assert np.array_equal(a, b)
