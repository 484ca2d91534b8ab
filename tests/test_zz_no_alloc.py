"""The allocation-free entry point (ssj_verify_device_noalloc) against
ssj_verify_device, the entry point it varies, on the same inputs: identical
result multisets and counts (tolerance 0), two calls in a row with the second
smaller, under plans that use its deferral queues and the window ring."""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from ssj_inputs import filter as cfilter  # noqa: E402
from ssj_inputs import synth  # noqa: E402


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_09141_amd.ssj as ssj
    ssj.load_library()
    return ssj


def _run(S, torch, fn, ctx, h, d_cand, tn, td):
    n = d_cand.shape[0]
    d_out = torch.empty((max(n, 1), 2), dtype=torch.int32, device="cuda:0")
    d_cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda:0")
    fn(ctx, h, d_cand, tn, td, d_out, d_cnt)
    torch.cuda.synchronize()
    k = int(d_cnt.item())
    assert k >= 0
    return oracle.sort_pairs(d_out[:k].cpu().numpy())


def test_noalloc_equals_verify_device(S):
    import torch
    man = json.load(open(os.path.join(ROOT, "tests", "golden", "manifest.json")))["2"]
    c = synth.workload_collection(2)
    ctx = S.ssj_init(0)
    try:
        h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        big = cfilter.workload_candidates(2, 7, 10)        # 614,384 pairs
        small = cfilter.workload_candidates(2, 9, 10)      # 9,833 pairs
        lists = [(big, 7, 10), (small, 9, 10)]
        plans = [dict(inline_lanes=1, defer_from=5),
                 dict(inline_lanes=1, defer_from=1, lanes=[4, 8, 16, 64, 256], spill_iters=1, spill_lanes=16),
                 dict(inline_lanes=1, defer_from=3, lanes=[4, 8, 16, 64, 256], staged=1, spill_iters=1,
                      spill_lanes=8)]
        for plan in plans:
            S.ssj_set_plan(ctx, S.make_plan(**plan))
            for cand, tn, td in lists:                     # two calls in a row, the second smaller
                d_cand = torch.from_numpy(cand).to("cuda:0")
                want = _run(S, torch, S.ssj_verify_device, ctx, h, d_cand, tn, td)
                got = _run(S, torch, S.ssj_verify_device_noalloc, ctx, h, d_cand, tn, td)
                assert np.array_equal(got, want), (plan, tn, td)
                m = man["thresholds"][f"{tn}/{td}"]
                assert got.shape[0] == m["n_result"] and oracle.result_digest(got) == m["result_sha256"]
        # count-only, and an id error in one call does not leak into the next
        d_cand = torch.from_numpy(small).to("cuda:0")
        d_cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        S.ssj_verify_device_noalloc(ctx, h, d_cand, 9, 10, None, d_cnt)
        torch.cuda.synchronize()
        assert int(d_cnt.item()) == man["thresholds"]["9/10"]["n_result"]
        bad = small.copy()
        bad[7] = [c.n_sets, 0]
        assert _count(S, torch, ctx, h, bad, 9, 10) == -1
        assert _count(S, torch, ctx, h, small, 9, 10) == man["thresholds"]["9/10"]["n_result"]
        # beyond the maximum: refused before anything is enqueued
        over = np.zeros((S.SSJ_NOALLOC_MAX_PAIRS + 1, 2), np.int32)
        d_over = torch.from_numpy(over).to("cuda:0")
        d_cnt.fill_(-7)
        with pytest.raises(S.SsjError) as e:
            S.ssj_verify_device_noalloc(ctx, h, d_over, 1, 2, None, d_cnt)
        assert e.value.code == S.SSJ_EINVAL
        torch.cuda.synchronize()
        assert int(d_cnt.item()) == -7
        S.ssj_free_collection(ctx, h)
    finally:
        S.ssj_shutdown(ctx)


def _count(S, torch, ctx, h, cand, tn, td):
    d_cand = torch.from_numpy(np.ascontiguousarray(cand)).to("cuda:0")
    d_cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    S.ssj_verify_device_noalloc(ctx, h, d_cand, tn, td, None, d_cnt)
    torch.cuda.synchronize()
    return int(d_cnt.item())


def test_noalloc_shared_by_two_contexts(S):
    """Two contexts on one device share the device's scratch; calls ordered
    on one stream give each its own correct result."""
    import torch
    rng = np.random.default_rng(8)
    c = synth.near_duplicate_collection(rng, n_base=200, copies=3, max_size=80, universe=5000, change_frac=0.1)
    cand = cfilter.candidates(c.offsets, c.tokens, 1, 2)
    want = oracle.sort_pairs(oracle.select(c.offsets, c.tokens, cand, 1, 2))
    a, b = S.ssj_init(0), S.ssj_init(0)
    try:
        ha = S.ssj_upload_collection(a, c.offsets, c.tokens)
        hb = S.ssj_upload_collection(b, c.offsets, c.tokens)
        d_cand = torch.from_numpy(cand).to("cuda:0")
        for ctx, h in ((a, ha), (b, hb), (a, ha)):
            assert np.array_equal(_run(S, torch, S.ssj_verify_device_noalloc, ctx, h, d_cand, 1, 2), want)
    finally:
        S.ssj_shutdown(a)
        S.ssj_shutdown(b)
