"""GPU parity: libssj (through the C ABI) against the oracle, bit-exact.

Results are integer pair multisets; the bar is identical sorted multisets
(tolerance 0).  Every lane mapping is forced on every case so that the plan
cannot hide a broken kernel.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import brute  # noqa: E402
from ssj_inputs import filter as cfilter  # noqa: E402
from ssj_inputs import synth  # noqa: E402

ALL_LANES = [1, 4, 8, 16, 32, 64, 256]


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_09141_amd.ssj as ssj
    ssj.load_library()
    return ssj


@pytest.fixture(scope="module")
def ctx(S):
    c = S.ssj_init(0)
    yield c
    S.ssj_shutdown(c)


def plans():
    """(name, plan kwargs) covering every mapping in both kernels."""
    out = [("default", None)]
    for L in [1, 4, 8, 16, 32, 64]:
        out.append((f"inline-{L}", dict(inline_lanes=L, defer_from=5)))
    for F in [8, 16]:
        out.append((f"inline-1h{F}", dict(inline_lanes=1, hard_lanes=F, defer_from=5)))
        out.append((f"inline-1h{F}-defer", dict(inline_lanes=1, hard_lanes=F, defer_from=1,
                                                 lanes=[4, 16, 32, 64, 256])))
    for L in ALL_LANES:
        out.append((f"deferred-all-{L}", dict(inline_lanes=4, defer_from=0, lanes=[L] * 5)))
    out.append(("mixed-1", dict(inline_lanes=1, defer_from=1, lanes=[4, 8, 32, 256, 256])))
    out.append(("mixed-graph", dict(inline_lanes=8, defer_from=2, lanes=[4, 16, 16, 64, 256],
                                    use_graph=1)))
    out.append(("inline-graph", dict(inline_lanes=4, defer_from=5, use_graph=1)))
    # thread-per-pair merges cut off after 1..3 window steps (nearly every
    # merge past the record tokens is verified again by the deferred kernel)
    for I, G in [(1, 16), (1, 1), (2, 4), (3, 64), (1, 256)]:
        out.append((f"spill-{I}x{G}", dict(inline_lanes=1, defer_from=5, spill_iters=I,
                                           spill_lanes=G)))
    out.append(("spill-2-defer", dict(inline_lanes=1, defer_from=2, lanes=[4, 8, 32, 64, 256],
                                      spill_iters=2, spill_lanes=32)))
    out.append(("spill-graph", dict(inline_lanes=1, defer_from=3, lanes=[4, 8, 16, 32, 256],
                                    spill_iters=1, spill_lanes=8, use_graph=1)))
    # the window ring (thread-per-pair merges with their window loads two
    # steps ahead): alone, cut off after one or two window steps (the rest
    # verified again by the deferred kernel), with deferred classes, in a
    # graph and on a one-workgroup grid
    out.append(("staged", dict(inline_lanes=1, defer_from=5, staged=1)))
    for I, G in [(1, 16), (2, 1), (1, 256)]:
        out.append((f"staged-spill-{I}x{G}", dict(inline_lanes=1, defer_from=5, staged=1, spill_iters=I,
                                                  spill_lanes=G)))
    out.append(("staged-defer", dict(inline_lanes=1, defer_from=2, lanes=[4, 8, 32, 64, 256], staged=1)))
    out.append(("staged-spill-2-defer", dict(inline_lanes=1, defer_from=3, lanes=[4, 8, 16, 64, 256],
                                             staged=1, spill_iters=2, spill_lanes=64)))
    out.append(("staged-graph", dict(inline_lanes=1, defer_from=4, lanes=[4, 8, 16, 32, 64], staged=1,
                                     use_graph=1)))
    out.append(("staged-wg1", dict(inline_lanes=1, defer_from=5, staged=1, wg_per_cu=1)))
    # in-order grids of one and of many workgroups per compute unit
    out.append(("inline-1-wg1", dict(inline_lanes=1, defer_from=5, wg_per_cu=1)))
    out.append(("inline-8-wg13", dict(inline_lanes=8, defer_from=5, wg_per_cu=13)))
    out.append(("spill-2x16-wg20", dict(inline_lanes=1, defer_from=4, lanes=[4, 8, 16, 32, 64],
                                        spill_iters=2, spill_lanes=16, wg_per_cu=20)))
    return out


def set_plan(S, ctx, plan):
    if plan is None:
        S.ssj_set_plan(ctx, S.make_plan(inline_lanes=1, hard_lanes=16, defer_from=3,
                                         lanes=[4, 16, 64, 256, 256]))
    else:
        S.ssj_set_plan(ctx, S.make_plan(**plan))


def run_host(S, ctx, h, cand, tn, td):
    return oracle.sort_pairs(S.ssj_verify(ctx, h, cand, tn, td))


def run_device(S, ctx, h, cand, tn, td):
    import torch
    dev = torch.device("cuda:0")
    d_cand = torch.from_numpy(np.ascontiguousarray(cand, dtype=np.int32)).to(dev)
    d_out = torch.empty((max(cand.shape[0], 1), 2), dtype=torch.int32, device=dev)
    d_cnt = torch.full((1,), -7, dtype=torch.int64, device=dev)
    S.ssj_verify_device(ctx, h, d_cand, tn, td, d_out, d_cnt)
    torch.cuda.synchronize()
    k = int(d_cnt.item())
    assert k >= 0
    return oracle.sort_pairs(d_out[:k].cpu().numpy())


def want_of(coll, cand, tn, td):
    return oracle.sort_pairs(oracle.select(coll.offsets, coll.tokens, cand, tn, td, n_threads=8))


def test_config1_all_plans(S, ctx, golden_dir):
    """The tiny collection at its stated threshold (no similar pairs) and at
    t = 1/2 (six), against brute force and the manifest, in every plan."""
    import json
    man = json.load(open(os.path.join(golden_dir, "manifest.json")))["1"]
    c = synth.workload_collection(1)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    (tn0, td0), = synth.WORKLOADS[1].thresholds
    for (tn, td) in [(tn0, td0), (1, 2)]:
        key = f"{tn}/{td}"
        m = man["thresholds"].get(key) or man["extra_thresholds"][key]
        cand = cfilter.workload_candidates(1, tn, td)
        assert cand.shape[0] == m["n_candidates"]
        want = want_of(c, cand, tn, td)
        assert [tuple(x) for x in want.tolist()] == sorted(brute.brute_join(c.offsets, c.tokens, tn, td))
        assert want.shape[0] == m["n_result"] and oracle.result_digest(want) == m["result_sha256"]
        for name, plan in plans():
            _log(f"config1 t={key} {name}")
            set_plan(S, ctx, plan)
            assert np.array_equal(run_host(S, ctx, h, cand, tn, td), want), (name, key)
    S.ssj_free_collection(ctx, h)


@pytest.mark.parametrize("seed", [0, 1])
def test_near_duplicates_all_plans(S, ctx, seed):
    rng = np.random.default_rng(100 + seed)
    c = synth.near_duplicate_collection(rng, n_base=150, copies=4, max_size=700, universe=6000,
                                        change_frac=0.08, min_size=1)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    rp = rng.integers(0, c.n_sets, size=(3000, 2)).astype(np.int32)
    for (tn, td) in [(1, 2), (7, 10), (9, 10)]:
        cand = np.concatenate([cfilter.candidates(c.offsets, c.tokens, tn, td), rp])
        want = want_of(c, cand, tn, td)
        assert want.shape[0] > (100 if tn * 2 <= td else 0)
        for name, plan in plans():
            _log(f"near-dup seed={seed} t={tn}/{td} {name} n={cand.shape[0]}")
            set_plan(S, ctx, plan)
            got = run_host(S, ctx, h, cand, tn, td)
            assert np.array_equal(got, want), (name, tn, td)
    S.ssj_free_collection(ctx, h)


def _adversarial():
    """Hand-built sets: equal, disjoint, subsets, tile seams, long sets."""
    rng = np.random.default_rng(5)
    sets = []
    sets.append(list(range(0, 10)))                         # 0
    sets.append(list(range(0, 10)))                         # 1 equal to 0
    sets.append(list(range(100, 110)))                      # 2 disjoint
    sets.append(list(range(0, 9)) + [50])                   # 3 overlap 9 with 0 (alpha at t=.8)
    sets.append(list(range(0, 8)) + [50, 51])               # 4 overlap 8 with 0
    sets.append([0])                                        # 5 first token only
    sets.append([9])                                        # 6 last token only
    evens = list(range(0, 4000, 2))
    sets.append(evens)                                      # 7
    sets.append(list(range(0, 4000)))                       # 8 superset of 7
    sets.append(list(range(1, 4000, 2)))                    # 9 disjoint from 7, interleaved
    big = sorted(rng.choice(200000, size=5000, replace=False).tolist())
    sets.append(big)                                        # 10
    b2 = sorted(set(big[:4500]) | set(rng.choice(np.arange(200000, 300000), size=500, replace=False).tolist()))
    sets.append(b2)                                         # 11 5000 vs 5000, overlap 4500
    for G in [4, 8, 16, 32, 64, 256]:                       # seams: matches at tile edges
        a = list(range(0, 3 * G))
        b = [x for x in a if x % G in (0, G - 1)] + list(range(10 ** 6, 10 ** 6 + 2 * G))
        sets.append(a)
        sets.append(sorted(b))
    # tile maxima equal / less / greater in every combination
    for k in range(6):
        x = sorted(rng.choice(300, size=int(rng.integers(30, 200)), replace=False).tolist())
        y = sorted(set(x[: len(x) // 2]) | set(rng.choice(300, size=40, replace=False).tolist()))
        sets.append(x)
        sets.append(y)
    return sets


def test_adversarial_all_plans(S, ctx):
    sets = _adversarial()
    c = synth.collection_from_sets(sets)
    n = c.n_sets
    pairs = [(i, j) for i in range(n) for j in range(n)]  # every orientation, self pairs
    cand = np.array(pairs + pairs[:50], dtype=np.int32)   # duplicates
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    for (tn, td) in [(0, 1), (1, 10), (1, 2), (4, 5), (9, 10), (1, 1)]:
        want = want_of(c, cand, tn, td)
        for name, plan in plans():
            _log(f"adversarial t={tn}/{td} {name}")
            set_plan(S, ctx, plan)
            assert np.array_equal(run_host(S, ctx, h, cand, tn, td), want), (name, tn, td)
            assert np.array_equal(run_device(S, ctx, h, cand, tn, td), want), (name, tn, td)
    S.ssj_free_collection(ctx, h)


def test_config2_default_plan_matches_manifest(S, ctx, golden_dir):
    import json
    man = json.load(open(os.path.join(golden_dir, "manifest.json")))["2"]
    c = synth.workload_collection(2)
    assert c.digest() == man["collection_sha256"]
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    set_plan(S, ctx, None)
    for (tn, td) in synth.WORKLOADS[2].thresholds:
        _log(f"config2 t={tn}/{td}")
        cand = cfilter.workload_candidates(2, tn, td)
        m = man["thresholds"][f"{tn}/{td}"]
        assert cand.shape[0] == m["n_candidates"]
        got = run_device(S, ctx, h, cand, tn, td)
        assert got.shape[0] == m["n_result"]
        assert oracle.result_digest(got) == m["result_sha256"]
        for L in [1, 16]:
            S.ssj_set_plan(ctx, S.make_plan(inline_lanes=L, defer_from=5))
            assert oracle.result_digest(run_host(S, ctx, h, cand, tn, td)) == m["result_sha256"]
        set_plan(S, ctx, None)
    S.ssj_free_collection(ctx, h)


def test_host_ring_batches_pieces_errors(S, golden_dir):
    """Host buffers of millions of pairs: several device batches (a budget of
    2.5M pairs) of several 1M-pair pieces each, against the manifest-checked
    result; an id error in a late piece; truncation over pieces."""
    import json
    man = json.load(open(os.path.join(golden_dir, "manifest.json")))["2"]
    c = synth.workload_collection(2)
    cand = cfilter.workload_candidates(2, 3, 5)
    m = man["thresholds"]["3/5"]
    # the collection's own device bytes (8.6 MB), then 2.5M pairs per batch
    ctx = S.ssj_init(0, hbm_budget=synth.device_bytes(c) + 40 * 2_500_000)
    try:
        h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        S.ssj_set_plan(ctx, S.make_plan(inline_lanes=1, defer_from=5))
        one = run_device(S, ctx, h, cand, 3, 5)
        assert one.shape[0] == m["n_result"] and oracle.result_digest(one) == m["result_sha256"]
        two = np.concatenate([cand, cand[::-1]])                       # 6.1M pairs
        _log(f"host ring: {two.shape[0]} pairs")
        got = oracle.sort_pairs(S.ssj_verify(ctx, h, two, 3, 5))
        assert np.array_equal(got, oracle.sort_pairs(np.concatenate([one, one])))
        bad = two.copy()
        bad[6_100_000] = [c.n_sets, 0]                                 # third batch, second piece
        with pytest.raises(S.SsjError) as e:
            S.ssj_verify(ctx, h, bad, 3, 5)
        assert e.value.code == S.SSJ_EINVAL
        k = 2 * m["n_result"]
        with pytest.raises(S.SsjError) as e:
            S.ssj_verify(ctx, h, two, 3, 5, out_cap=k // 3)
        assert e.value.code == S.SSJ_ETRUNC and e.value.n == k
        # the context keeps working
        assert oracle.sort_pairs(S.ssj_verify(ctx, h, cand, 3, 5)).shape[0] == m["n_result"]
        S.ssj_free_collection(ctx, h)
    finally:
        S.ssj_shutdown(ctx)


def test_config3_long_sets(S, ctx, golden_dir):
    import json
    man = json.load(open(os.path.join(golden_dir, "manifest.json")))["3"]
    c = synth.workload_collection(3)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    (tn, td), = synth.WORKLOADS[3].thresholds
    cand = cfilter.workload_candidates(3, tn, td)
    m = man["thresholds"][f"{tn}/{td}"]
    # the random workload has few similar pairs: its whole candidate list is
    # also verified at lower thresholds (11 pass at t = 1/10), pinned in the
    # manifest, in every plan
    for name, plan in LONG_PLANS:
        set_plan(S, ctx, plan)
        _log(f"config3 {name}")
        got = run_host(S, ctx, h, cand, tn, td)
        assert got.shape[0] == m["n_result"] and oracle.result_digest(got) == m["result_sha256"], name
        for key, v in man["verify_at"].items():
            if key == "candidates":
                continue
            vn, vd = (int(x) for x in key.split("/"))
            got = run_device(S, ctx, h, cand, vn, vd)
            assert got.shape[0] == v["n_result"] and oracle.result_digest(got) == v["result_sha256"], \
                (name, key)
    S.ssj_free_collection(ctx, h)


# Long-set plans: every mapping family plus the plans the autotuner picks on
# the long-set workload (thread per pair with a step budget and the longest
# class on 64 lanes; the window ring with a step budget).
LONG_PLANS = [("default", None), ("inline-16", dict(inline_lanes=16, defer_from=5)),
              ("inline-64", dict(inline_lanes=64, defer_from=5)),
              ("deferred-all-256", dict(inline_lanes=4, defer_from=0, lanes=[256] * 5)),
              ("deferred-long", dict(inline_lanes=1, defer_from=2, lanes=[4, 8, 16, 64, 256])),
              ("spill-8x16", dict(inline_lanes=1, defer_from=5, spill_iters=8, spill_lanes=16)),
              ("spill-4x64-defer", dict(inline_lanes=1, defer_from=4, lanes=[4, 8, 16, 32, 32],
                                        spill_iters=4, spill_lanes=64)),
              ("tuned-s32x16w4", dict(inline_lanes=1, defer_from=4, lanes=[4, 4, 8, 16, 64],
                                      spill_iters=32, spill_lanes=16, wg_per_cu=4)),
              ("staged", dict(inline_lanes=1, defer_from=5, staged=1)),
              ("staged-s24x16", dict(inline_lanes=1, defer_from=5, staged=1, spill_iters=24, spill_lanes=16)),
              ("staged-s4x64-defer", dict(inline_lanes=1, defer_from=4, lanes=[4, 8, 16, 32, 64], staged=1,
                                          spill_iters=4, spill_lanes=64)),
              ("staged-s8x16-wg2", dict(inline_lanes=1, defer_from=5, staged=1, spill_iters=8,
                                        spill_lanes=16, wg_per_cu=2))]


def test_long_near_duplicates_all_plans(S, ctx):
    """Long sets (10 to 600 tokens, Zipf(0.9) over 1,000,000 tokens as in the
    long-set workload) of which each appears three times with 8% of its tokens
    changed: thousands of passing long pairs, in every long-set plan."""
    rng = np.random.default_rng(31)
    c = synth.near_duplicate_collection(rng, n_base=1500, copies=3, max_size=600, universe=1_000_000,
                                        change_frac=0.08, min_size=10, zipf_s=0.9)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        for (tn, td) in [(7, 10), (1, 2)]:
            cand = cfilter.candidates(c.offsets, c.tokens, tn, td)
            want = want_of(c, cand, tn, td)
            assert want.shape[0] > 1000
            for name, plan in LONG_PLANS:
                _log(f"long near-dup t={tn}/{td} {name} n={cand.shape[0]}")
                set_plan(S, ctx, plan)
                assert np.array_equal(run_device(S, ctx, h, cand, tn, td), want), (name, tn, td)
    finally:
        S.ssj_free_collection(ctx, h)


def test_extreme_tokens_and_very_long_sets(S, ctx):
    """Token ids at both ends of the allowed range (0 and 2^31 - 1), and sets
    of 120,000 tokens (far past the longest length class bound) against each
    other and against one-token sets, in every mapping."""
    top = (1 << 31) - 1
    long1 = list(range(0, 120000))
    long2 = list(range(0, 119000)) + list(range(top - 999, top + 1))   # overlap 119,000 with long1
    long3 = list(range(0, 240000, 2))                                     # overlap 60,000 with long1
    sets = [[top], [top - 1, top], [0, top], list(range(top - 999, top + 1)), [0],
            long1, long2, long3, list(range(top - 99, top + 1))]
    c = synth.collection_from_sets(sets)
    n = c.n_sets
    cand = np.array([(i, j) for i in range(n) for j in range(n)], dtype=np.int32)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        for (tn, td) in [(0, 1), (1, 1000), (1, 2), (99, 100), (1, 1)]:
            want = want_of(c, cand, tn, td)
            for name, plan in plans():
                _log(f"extreme tokens t={tn}/{td} {name}")
                set_plan(S, ctx, plan)
                assert np.array_equal(run_device(S, ctx, h, cand, tn, td), want), (name, tn, td)
            assert np.array_equal(run_host(S, ctx, h, cand, tn, td), want), (tn, td)
    finally:
        S.ssj_free_collection(ctx, h)


def test_errors_and_edges(S, ctx):
    import torch
    c = synth.collection_from_sets([[1, 2, 3], [2, 3, 4], [7]])
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    set_plan(S, ctx, None)
    # empty candidate list
    assert S.ssj_verify(ctx, h, np.zeros((0, 2), np.int32), 1, 2).shape == (0, 2)
    # out-of-range ids
    for bad in ([0, 3], [-1, 0], [2, 1 << 30]):
        with pytest.raises(S.SsjError) as e:
            S.ssj_verify(ctx, h, np.array([[0, 1], bad], np.int32), 1, 2)
        assert e.value.code == S.SSJ_EINVAL
    dev = torch.device("cuda:0")
    d_cand = torch.tensor([[0, 1], [0, 5]], dtype=torch.int32, device=dev)
    d_out = torch.empty((2, 2), dtype=torch.int32, device=dev)
    d_cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    S.ssj_verify_device(ctx, h, d_cand, 1, 2, d_out, d_cnt)
    torch.cuda.synchronize()
    assert int(d_cnt.item()) == -1
    # the context keeps working after an id error (counters were reset)
    got = S.ssj_verify(ctx, h, np.array([[0, 1], [1, 0], [0, 0]], np.int32), 1, 2)
    assert oracle.sort_pairs(got).tolist() == [[0, 0], [0, 1], [1, 0]]
    # bad thresholds
    for tn, td in [(3, 2), (-1, 2), (1, 0), (1, 1 << 31)]:
        with pytest.raises(S.SsjError) as e:
            S.ssj_verify(ctx, h, np.array([[0, 1]], np.int32), tn, td)
        assert e.value.code == S.SSJ_EINVAL
    # truncation: count is reported, retry with room succeeds
    cand = np.array([[0, 0], [1, 1], [0, 1]] * 5, np.int32)
    with pytest.raises(S.SsjError) as e:
        S.ssj_verify(ctx, h, cand, 1, 2, out_cap=3)
    assert e.value.code == S.SSJ_ETRUNC and e.value.n == 15
    assert S.ssj_verify(ctx, h, cand, 1, 2, out_cap=15).shape[0] == 15
    # unsupported plans are refused and leave the plan unchanged
    before = S.ssj_get_plan(ctx).as_dict()
    for bad in [dict(inline_lanes=3), dict(inline_lanes=4, hard_lanes=8), dict(defer_from=6),
                dict(lanes=[4, 16, 3, 256, 256]), dict(inline_lanes=4, spill_iters=2),
                dict(inline_lanes=1, hard_lanes=8, spill_iters=2), dict(spill_iters=-1),
                dict(spill_iters=(1 << 20) + 1), dict(spill_iters=4, spill_lanes=2),
                dict(wg_per_cu=-1), dict(wg_per_cu=65)]:
        with pytest.raises(S.SsjError) as e:
            S.ssj_set_plan(ctx, S.make_plan(**bad))
        assert e.value.code == S.SSJ_EINVAL, bad
    assert S.ssj_get_plan(ctx).as_dict() == before
    S.ssj_free_collection(ctx, h)


def test_upload_validation(S, ctx):
    bad = [
        (np.array([0, 2, 2]), np.array([1, 2], np.int32)),       # empty set
        (np.array([0, 2, 4]), np.array([1, 1, 2, 3], np.int32)),  # duplicate token
        (np.array([0, 2, 4]), np.array([2, 1, 2, 3], np.int32)),  # unsorted
        (np.array([0, 2, 4]), np.array([-1, 1, 2, 3], np.int32)),  # negative
        (np.array([1, 2, 4]), np.array([0, 1, 2, 3], np.int32)),  # offsets[0] != 0
        (np.array([0, 3, 2]), np.array([0, 1, 2], np.int32)),     # decreasing
    ]
    for off, tok in bad:
        with pytest.raises(S.SsjError) as e:
            S.ssj_upload_collection(ctx, off, tok)
        assert e.value.code == S.SSJ_EINVAL


def test_chunked_budget(S):
    # a budget of a few KiB beyond the collection's own device bytes forces
    # many chunks inside one ssj_verify call
    rng = np.random.default_rng(9)
    c = synth.near_duplicate_collection(rng, n_base=100, copies=4, max_size=30, universe=2000,
                                        change_frac=0.1)
    ctx = S.ssj_init(0, hbm_budget=synth.device_bytes(c) + 36 * 1000)
    try:
        h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        cand = np.concatenate([cfilter.candidates(c.offsets, c.tokens, 1, 2),
                               rng.integers(0, c.n_sets, size=(20000, 2)).astype(np.int32)])
        want = want_of(c, cand, 1, 2)
        assert np.array_equal(run_host(S, ctx, h, cand, 1, 2), want)
    finally:
        S.ssj_shutdown(ctx)


def test_config4_full_size(S, ctx, golden_dir):
    """Heavy-tail collection at full size (168M candidates) through the device
    entry point, as bench.py launches it; compared with the oracle's digest."""
    import json
    import torch
    man = json.load(open(os.path.join(golden_dir, "manifest.json")))["4"]
    c = synth.workload_collection(4)
    assert c.digest() == man["collection_sha256"]
    (tn, td), = synth.WORKLOADS[4].thresholds
    m = man["thresholds"][f"{tn}/{td}"]
    cand = cfilter.workload_candidates(4, tn, td)
    assert cand.shape[0] == m["n_candidates"]
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    d_cand = torch.from_numpy(cand).to("cuda:0")
    d_out = torch.empty((m["n_result"] + 1024, 2), dtype=torch.int32, device="cuda:0")
    d_cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    for name, plan in [("inline-1", dict(inline_lanes=1, defer_from=5)),
                       ("defer-3", dict(inline_lanes=1, defer_from=3, lanes=[4, 16, 64, 256, 256])),
                       ("defer-1", dict(inline_lanes=1, defer_from=1, lanes=[4, 16, 32, 64, 256])),
                       ("spill-2x32", dict(inline_lanes=1, defer_from=5, spill_iters=2, spill_lanes=32))]:
        _log(f"config4 {name}")
        set_plan(S, ctx, plan)
        S.ssj_verify_device(ctx, h, d_cand, tn, td, d_out, d_cnt)
        torch.cuda.synchronize()
        k = int(d_cnt.item())
        assert k == m["n_result"], name
        got = d_out[:k].cpu().numpy()
        assert oracle.result_digest(got) == m["result_sha256"], name
        S.ssj_verify_device(ctx, h, d_cand, tn, td, None, d_cnt)  # output-count mode
        torch.cuda.synchronize()
        assert int(d_cnt.item()) == m["n_result"], name
    del d_cand, d_out
    S.ssj_free_collection(ctx, h)


def test_config5_stream_batches(S, golden_dir):
    """Streamed batches of the 1,000,000-set collection, each against the oracle."""
    from paper_1812_09141_amd import serving
    c = synth.workload_collection(5)
    sizes, ts, _ = synth.stream_schedule(24, seed=3, thresholds=synth.WORKLOADS[5].thresholds)
    batches = serving.build_batches(c.offsets, c.tokens, sizes, ts, n_threads=8)
    ctx = S.ssj_init(0, n_slots=3, queue_depth=8)
    try:
        h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        tickets = [S.ssj_stream_submit(ctx, h, b, tn, td) for (b, tn, td) in batches]
        for t, (b, tn, td) in zip(tickets, batches):
            got = oracle.sort_pairs(S.ssj_stream_collect(ctx, t))
            want = want_of(c, b, tn, td)
            assert np.array_equal(got, want), (tn, td, b.shape[0])
    finally:
        S.ssj_shutdown(ctx)


def test_ppjoin_candidates_same_join(S, ctx, golden_dir):
    """Candidates thinned by PPJoin's positional filter give the manifest's join
    result on the GPU (offline and long-set collections, every threshold)."""
    import json
    for cfg in (2, 3):
        man = json.load(open(os.path.join(golden_dir, "manifest.json")))[str(cfg)]
        c = synth.workload_collection(cfg)
        h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        try:
            set_plan(S, ctx, None)
            for (tn, td) in synth.WORKLOADS[cfg].thresholds:
                cand = cfilter.workload_candidates(cfg, tn, td, positional=True)
                m = man["thresholds"][f"{tn}/{td}"]
                _log(f"ppjoin config{cfg} t={tn}/{td}: {cand.shape[0]} candidates")
                got = run_host(S, ctx, h, cand, tn, td)
                assert got.shape[0] == m["n_result"]
                assert oracle.result_digest(got) == m["result_sha256"]
        finally:
            S.ssj_free_collection(ctx, h)
