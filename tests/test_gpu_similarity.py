"""GPU parity for the similarity functions of Table 1 (Cosine, Dice, Overlap
next to Jaccard): libssj through the C ABI against the oracle, bit-exact.

Every lane mapping is forced on every case, candidates are all pairs of
small near-duplicate collections (many pairs sit at the threshold), and the
thresholds include the ones where Table 1 in binary floating point would
round the equivalent overlap the wrong way.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from ssj_inputs import synth  # noqa: E402

THRESHOLDS = {
    "jaccard": [(1, 2), (3, 5), (4, 5), (1, 1)],
    "cosine": [(0, 1), (1, 2), (11, 20), (4, 5), (9, 10), (1, 1)],
    "dice": [(1, 2), (11, 20), (3, 5), (4, 5), (1, 1)],
    "overlap": [(0, 1), (1, 1), (3, 1), (7, 2), (8, 1), (40, 1)],
}

PLANS = [
    ("inline-1", dict(inline_lanes=1, defer_from=5)),
    ("inline-1h8", dict(inline_lanes=1, hard_lanes=8, defer_from=5)),
    ("inline-1h16-defer", dict(inline_lanes=1, hard_lanes=16, defer_from=1,
                               lanes=[4, 16, 32, 64, 256])),
    ("inline-4", dict(inline_lanes=4, defer_from=5)),
    ("inline-16", dict(inline_lanes=16, defer_from=5)),
    ("inline-64", dict(inline_lanes=64, defer_from=5)),
    ("deferred-1", dict(inline_lanes=4, defer_from=0, lanes=[1] * 5)),
    ("deferred-8", dict(inline_lanes=4, defer_from=0, lanes=[8] * 5)),
    ("deferred-32", dict(inline_lanes=4, defer_from=0, lanes=[32] * 5)),
    ("deferred-256", dict(inline_lanes=4, defer_from=0, lanes=[256] * 5)),
    ("spill-1x16", dict(inline_lanes=1, defer_from=5, spill_iters=1, spill_lanes=16)),
    ("spill-2x1-defer", dict(inline_lanes=1, defer_from=3, lanes=[4, 8, 16, 32, 256],
                             spill_iters=2, spill_lanes=1)),
    ("ring", dict(inline_lanes=1, defer_from=5, staged=1)),
    ("ring-spill-2x16-defer", dict(inline_lanes=1, defer_from=2, lanes=[4, 8, 32, 64, 256], staged=1,
                                   spill_iters=2, spill_lanes=16)),
]


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


def _all_pairs(n):
    i, j = np.tril_indices(n, -1)
    return np.stack([i, j], axis=1).astype(np.int32)


def _case(seed, max_size):
    rng = np.random.default_rng(9100 + seed)
    c = synth.near_duplicate_collection(rng, n_base=24, copies=5, max_size=max_size,
                                        universe=4 * max_size, change_frac=0.2)
    return c, _all_pairs(c.n_sets)


@pytest.mark.parametrize("seed,max_size", [(0, 12), (1, 40), (2, 300)])
def test_similarity_all_plans(S, ctx, seed, max_size):
    c, cand = _case(seed, max_size)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        for sim, ts in THRESHOLDS.items():
            for tn, td in ts:
                want = oracle.sort_pairs(oracle.select(c.offsets, c.tokens, cand, tn, td, sim=sim))
                for name, plan in PLANS:
                    _log(f"similarity seed={seed} max={max_size} {sim} t={tn}/{td} plan={name}")
                    S.ssj_set_plan(ctx, S.make_plan(**plan))
                    got = oracle.sort_pairs(S.ssj_verify_sim(ctx, h, cand, sim, tn, td))
                    assert np.array_equal(got, want), (sim, tn, td, name)
    finally:
        S.ssj_free_collection(ctx, h)


def test_similarity_mixed_batch_and_count_mode(S, ctx):
    import torch
    c, cand = _case(3, 60)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        S.ssj_set_plan(ctx, S.make_plan(inline_lanes=1, hard_lanes=8, defer_from=3,
                                         lanes=[4, 16, 32, 64, 256]))
        dev = torch.device("cuda:0")
        reqs, want = [], []
        for sim, tn, td in [("jaccard", 3, 5), ("cosine", 11, 20), ("dice", 11, 20),
                            ("overlap", 6, 1), ("cosine", 4, 5)]:
            d_cand = torch.from_numpy(cand).to(dev)
            count_only = sim == "overlap"
            d_out = None if count_only else torch.empty_like(d_cand)
            d_count = torch.zeros(1, dtype=torch.int64, device=dev)
            reqs.append((d_cand, tn, td, d_out, d_count, sim))
            want.append(oracle.sort_pairs(oracle.select(c.offsets, c.tokens, cand, tn, td, sim=sim)))
        _log("similarity mixed batch")
        S.ssj_verify_batch_device(ctx, h, reqs)
        torch.cuda.synchronize()
        for (d_cand, tn, td, d_out, d_count, sim), w in zip(reqs, want):
            k = int(d_count.item())
            assert k == w.shape[0], (sim, tn, td)
            if d_out is not None:
                got = oracle.sort_pairs(d_out[:k].cpu().numpy())
                assert np.array_equal(got, w), (sim, tn, td)
        # the device entry point with a named function
        d_cand = torch.from_numpy(cand).to(dev)
        d_out = torch.empty_like(d_cand)
        d_count = torch.zeros(1, dtype=torch.int64, device=dev)
        S.ssj_verify_device_sim(ctx, h, d_cand, "dice", 3, 5, d_out, d_count)
        torch.cuda.synchronize()
        w = oracle.sort_pairs(oracle.select(c.offsets, c.tokens, cand, 3, 5, sim="dice"))
        k = int(d_count.item())
        assert np.array_equal(oracle.sort_pairs(d_out[:k].cpu().numpy()), w)
    finally:
        S.ssj_free_collection(ctx, h)


def test_similarity_stream(S, ctx):
    c, cand = _case(4, 40)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        jobs = [("cosine", 3, 5), ("dice", 4, 5), ("overlap", 5, 1), ("jaccard", 1, 2)]
        tickets = []
        for sim, tn, td in jobs:
            _log(f"similarity stream submit {sim} {tn}/{td}")
            tickets.append(S.ssj_stream_submit_sim(ctx, h, cand, sim, tn, td))
        for (sim, tn, td), t in zip(jobs, tickets):
            got = oracle.sort_pairs(S.ssj_stream_collect(ctx, t))
            want = oracle.sort_pairs(oracle.select(c.offsets, c.tokens, cand, tn, td, sim=sim))
            assert np.array_equal(got, want), (sim, tn, td)
    finally:
        S.ssj_free_collection(ctx, h)


def test_cosine_long_sets(S, ctx):
    """Large |r| |s| products (the Cosine rule's exact square-root search) and
    pairs placed exactly at the threshold."""
    rng = np.random.default_rng(9200)
    sets = []
    base = np.arange(0, 4000, dtype=np.int64)
    for n_r, n_s, shared in [(100, 100, 55), (2500, 2500, 1375), (3000, 1200, 1045),
                             (1800, 800, 660), (400, 3600, 660), (1000, 1000, 550)]:
        r = base[:n_r]
        s = np.concatenate([base[:shared], 10000 + rng.choice(20000, n_s - shared, replace=False)])
        sets.append(sorted(r.tolist()))
        sets.append(sorted(set(s.tolist())))
    c = synth.collection_from_sets(sets)
    cand = _all_pairs(c.n_sets)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        for sim in ("cosine", "dice"):
            for tn, td in [(11, 20), (1, 2), (3, 5), (7, 10)]:
                want = oracle.sort_pairs(oracle.select(c.offsets, c.tokens, cand, tn, td, sim=sim))
                for name, plan in PLANS:
                    _log(f"long sets {sim} t={tn}/{td} plan={name}")
                    S.ssj_set_plan(ctx, S.make_plan(**plan))
                    got = oracle.sort_pairs(S.ssj_verify_sim(ctx, h, cand, sim, tn, td))
                    assert np.array_equal(got, want), (sim, tn, td, name)
    finally:
        S.ssj_free_collection(ctx, h)


def test_required_overlap_large_terms(S, ctx):
    """Thresholds whose terms reach 2^31 - 1: the required overlap
    ceil(num (|r| + |s|) / den) with divisors up to 2^32 - 2, with dividends
    on both sides of 2^32 (the kernels divide the smaller ones by a
    per-request magic number and the larger ones exactly), and one-token up
    to 2,000-token sets, in every mapping."""
    rng = np.random.default_rng(9300)
    c = synth.near_duplicate_collection(rng, n_base=30, copies=4, max_size=2000, universe=8000,
                                        change_frac=0.05)
    sets = [c.tokens[c.offsets[i]:c.offsets[i + 1]].tolist() for i in range(c.n_sets)]
    # exact copies (similarity 1, so they pass thresholds just below 1) and tiny sets
    c = synth.collection_from_sets(sets + [sets[0], sets[7], sets[50], [5], [5, 9], [1, 2, 3], [5, 9]])
    cand = _all_pairs(c.n_sets)
    top = (1 << 31) - 1
    cases = [("jaccard", 1, top), ("jaccard", top - 1, top), ("jaccard", 1 << 30, top),
             ("jaccard", 999999937, 1000000007), ("jaccard", 65537, 131071), ("jaccard", 1, 2),
             ("dice", 1, top), ("dice", top - 1, top), ("dice", 999999937, 1000000007)]
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        for sim, tn, td in cases:
            want = oracle.sort_pairs(oracle.select(c.offsets, c.tokens, cand, tn, td, sim=sim))
            for name, plan in PLANS:
                _log(f"large terms {sim} t={tn}/{td} plan={name}")
                S.ssj_set_plan(ctx, S.make_plan(**plan))
                got = oracle.sort_pairs(S.ssj_verify_sim(ctx, h, cand, sim, tn, td))
                assert np.array_equal(got, want), (sim, tn, td, name)
    finally:
        S.ssj_free_collection(ctx, h)


def test_similarity_threshold_errors(S, ctx):
    c, cand = _case(5, 10)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        for sim in ("jaccard", "cosine", "dice"):
            with pytest.raises(S.SsjError) as e:
                S.ssj_verify_sim(ctx, h, cand, sim, 3, 2)
            assert e.value.code == S.SSJ_EINVAL
        got = oracle.sort_pairs(S.ssj_verify_sim(ctx, h, cand, "overlap", 3, 2))
        want = oracle.sort_pairs(oracle.select(c.offsets, c.tokens, cand, 3, 2, sim="overlap"))
        assert np.array_equal(got, want)
        with pytest.raises(S.SsjError):
            S.ssj_verify_sim(ctx, h, cand, 7, 1, 2)
        with pytest.raises(S.SsjError):
            S.ssj_verify_sim(ctx, h, cand, "overlap", 1, 0)
    finally:
        S.ssj_free_collection(ctx, h)
