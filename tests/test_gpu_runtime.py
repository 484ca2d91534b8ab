"""GPU runtime tests: batched launches, graph replay, autotuning, streaming.

Every result is compared with the oracle as a sorted multiset (tolerance 0).
"""
import os
import sys
import threading
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from ssj_inputs import filter as cfilter  # noqa: E402
from ssj_inputs import synth  # noqa: E402


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


@pytest.fixture(scope="module")
def data():
    rng = np.random.default_rng(21)
    c = synth.near_duplicate_collection(rng, n_base=300, copies=4, max_size=300, universe=20000,
                                        change_frac=0.1, min_size=1)
    reqs = []
    for (tn, td) in [(1, 2), (3, 5), (7, 10), (4, 5), (9, 10), (0, 1), (1, 1)]:
        cand = cfilter.candidates(c.offsets, c.tokens, max(tn, 1), td) if tn > 0 else \
            rng.integers(0, c.n_sets, size=(5000, 2)).astype(np.int32)
        cand = np.concatenate([cand, rng.integers(0, c.n_sets, size=(2000, 2)).astype(np.int32)])
        want = oracle.sort_pairs(oracle.select(c.offsets, c.tokens, cand, tn, td, n_threads=8))
        reqs.append((cand, tn, td, want))
    return c, reqs


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to("cuda:0")


def test_batched_launch_equals_oracle(S, ctx, data):
    import torch
    c, reqs = data
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    for plan in [dict(inline_lanes=4, defer_from=5), dict(inline_lanes=1, defer_from=1,
                                                         lanes=[4, 8, 32, 256, 256]),
                 dict(inline_lanes=8, defer_from=2, lanes=[4, 16, 16, 64, 256], use_graph=1)]:
        _log(f"batch plan {plan}")
        S.ssj_set_plan(ctx, S.make_plan(**plan))
        d = []
        for (cand, tn, td, want) in reqs:
            d.append((_dev(torch, cand), tn, td,
                      torch.empty((cand.shape[0], 2), dtype=torch.int32, device="cuda:0"),
                      torch.full((1,), -7, dtype=torch.int64, device="cuda:0")))
        for rep in range(3):  # repeated launches reuse the self-resetting counters
            S.ssj_verify_batch_device(ctx, h, d)
            torch.cuda.synchronize()
            for (cand, tn, td, want), (_, _, _, d_out, d_cnt) in zip(reqs, d):
                k = int(d_cnt.item())
                got = oracle.sort_pairs(d_out[:k].cpu().numpy())
                assert np.array_equal(got, want), (plan, tn, td, rep)
    # an id error in one request does not leak into the others
    S.ssj_set_plan(ctx, S.make_plan(inline_lanes=4, defer_from=3, lanes=[4, 16, 64, 256, 256]))
    good, bad = reqs[0], reqs[1][0].copy()
    bad[5] = [c.n_sets, 0]
    d_good = (_dev(torch, good[0]), good[1], good[2],
              torch.empty((good[0].shape[0], 2), dtype=torch.int32, device="cuda:0"),
              torch.zeros(1, dtype=torch.int64, device="cuda:0"))
    d_bad = (_dev(torch, bad), 1, 2, torch.empty((bad.shape[0], 2), dtype=torch.int32, device="cuda:0"),
             torch.zeros(1, dtype=torch.int64, device="cuda:0"))
    S.ssj_verify_batch_device(ctx, h, [d_good, d_bad])
    torch.cuda.synchronize()
    assert int(d_bad[4].item()) == -1
    k = int(d_good[4].item())
    assert np.array_equal(oracle.sort_pairs(d_good[3][:k].cpu().numpy()), good[3])
    S.ssj_free_collection(ctx, h)


def test_graph_replay_matches_eager(S, ctx, data):
    """Library graph replays, with eager work and syncs in between, all match."""
    import torch
    c, reqs = data
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    cand, tn, td, want = reqs[1]
    d_cand = _dev(torch, cand)
    for plan in [dict(inline_lanes=4, defer_from=5, use_graph=1),
                 dict(inline_lanes=4, defer_from=1, lanes=[4, 16, 32, 64, 256], use_graph=1),
                 dict(inline_lanes=1, defer_from=5, spill_iters=1, spill_lanes=16, use_graph=1)]:
        for rep in range(4):
            S.ssj_set_plan(ctx, S.make_plan(**plan))
            d_out = torch.empty((cand.shape[0], 2), dtype=torch.int32, device="cuda:0")
            d_cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
            S.ssj_verify_device(ctx, h, d_cand, tn, td, d_out, d_cnt)
            torch.cuda.synchronize()
            k = int(d_cnt.item())
            assert np.array_equal(oracle.sort_pairs(d_out[:k].cpu().numpy()), want), (plan, rep)
            # eager launch in between
            S.ssj_set_plan(ctx, S.make_plan(**dict(plan, use_graph=0)))
            S.ssj_verify_device(ctx, h, d_cand, tn, td, d_out, d_cnt)
            torch.cuda.synchronize()
            k = int(d_cnt.item())
            assert np.array_equal(oracle.sort_pairs(d_out[:k].cpu().numpy()), want), (plan, rep)
    S.ssj_free_collection(ctx, h)


def test_autotune_plan_is_correct(S, ctx, data):
    import torch
    c, reqs = data
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    cand, tn, td, want = reqs[0]
    d_cand = _dev(torch, cand)
    plan, ms = S.ssj_autotune(ctx, h, d_cand, tn, td, apply=True)
    _log(f"autotuned plan {plan.as_dict()} {ms:.4f} ms")
    assert ms > 0
    got = oracle.sort_pairs(S.ssj_verify(ctx, h, cand, tn, td))
    assert np.array_equal(got, want)
    assert S.ssj_get_plan(ctx).as_dict() == plan.as_dict()
    S.ssj_free_collection(ctx, h)


def test_autotune_cache(S, ctx, data, tmp_path):
    """The tuning cache: a tuned workload is stored and then served without
    measuring (SSJ_CACHED, same plan and time), also to another context; a
    different threshold misses; lines that do not parse are ignored."""
    import torch
    c, reqs = data
    path = str(tmp_path / "tune.jsonl")
    with open(path, "w") as f:
        f.write("not json\n{\"key\": \"broken\n")
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        S.ssj_set_tune_cache(ctx, path)
        cand, tn, td, want = reqs[0]
        d_cand = _dev(torch, cand)
        p1, ms1, hit1 = S.ssj_autotune(ctx, h, d_cand, tn, td, apply=True, with_status=True)
        assert not hit1 and ms1 > 0
        p2, ms2, hit2 = S.ssj_autotune(ctx, h, d_cand, tn, td, apply=False, with_status=True)
        assert hit2 and p2.as_dict() == p1.as_dict() and abs(ms2 - ms1) < 1e-5
        got = oracle.sort_pairs(S.ssj_verify(ctx, h, cand, tn, td))
        assert np.array_equal(got, want)
        lines = open(path).read().splitlines()
        assert len(lines) == 3 and lines[-1].startswith('{"key": "') and "|t=" in lines[-1]
        # the same workload in a second context reads the same file
        ctx2 = S.ssj_init(0)
        try:
            S.ssj_set_tune_cache(ctx2, path)
            h2 = S.ssj_upload_collection(ctx2, c.offsets, c.tokens)
            p3, ms3, hit3 = S.ssj_autotune(ctx2, h2, d_cand, tn, td, apply=True, with_status=True)
            assert hit3 and p3.as_dict() == p1.as_dict()
            assert S.ssj_get_plan(ctx2).as_dict() == p1.as_dict()
            S.ssj_free_collection(ctx2, h2)
        finally:
            S.ssj_shutdown(ctx2)
        # another threshold is another workload
        cand_b, tn_b, td_b, _ = reqs[1]
        if (tn_b, td_b) != (tn, td):
            _, _, hit4 = S.ssj_autotune(ctx, h, _dev(torch, cand_b), tn_b, td_b, apply=False, with_status=True)
            assert not hit4
        S.ssj_set_tune_cache(ctx, None)
        _, _, hit5 = S.ssj_autotune(ctx, h, d_cand, tn, td, apply=False, with_status=True)
        assert not hit5
    finally:
        S.ssj_set_tune_cache(ctx, None)
        S.ssj_free_collection(ctx, h)


def test_timing_counts_launches(S, ctx, data):
    import torch
    c, reqs = data
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    S.ssj_set_plan(ctx, S.make_plan(inline_lanes=4, defer_from=2, lanes=[4, 16, 16, 64, 256]))
    cand, tn, td, want = reqs[2]
    d_cand = _dev(torch, cand)
    d_out = torch.empty((cand.shape[0], 2), dtype=torch.int32, device="cuda:0")
    d_cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    S.ssj_timing_read(ctx, reset=True)
    S.ssj_timing_enable(ctx, 1)
    for _ in range(5):
        S.ssj_verify_device(ctx, h, d_cand, tn, td, d_out, d_cnt)
    torch.cuda.synchronize()
    a, b, n = S.ssj_timing_read(ctx, reset=True)
    assert n == 5 and a > 0 and b > 0
    S.ssj_timing_enable(ctx, 3)
    for _ in range(7):
        S.ssj_verify_device(ctx, h, d_cand, tn, td, d_out, d_cnt)
    torch.cuda.synchronize()
    a, b, n = S.ssj_timing_read(ctx, reset=True)
    assert n == 3 and a > 0
    S.ssj_timing_enable(ctx, 0)
    k = int(d_cnt.item())
    assert np.array_equal(oracle.sort_pairs(d_out[:k].cpu().numpy()), want)
    S.ssj_free_collection(ctx, h)


def _collect(S, ctx, t):
    return oracle.sort_pairs(S.ssj_stream_collect(ctx, t))


def test_run_stream_several_submitters(S, data):
    """The serving replay with several submitting threads, saturated and at a
    Poisson offered load, returns every result (counts against the oracle)."""
    from paper_1812_09141_amd import serving
    c, reqs = data
    ctx = S.ssj_init(0, n_slots=3, queue_depth=16)
    try:
        h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        batches = [(cand, tn, td) for (cand, tn, td, _) in reqs] * 3
        want = 3 * sum(w.shape[0] for (_, _, _, w) in reqs)
        for rate, subs in [(None, 4), (None, 1), (2e8, 3)]:
            _log(f"run_stream rate={rate} submitters={subs}")
            out = serving.run_stream(S, ctx, h, batches, rate, seed=2, n_submitters=subs)
            assert out["results"] == want and out["batches"] == len(batches)
            assert out["submit_threads"] == subs
        S.ssj_free_collection(ctx, h)
    finally:
        S.ssj_shutdown(ctx)


def test_stream_alone_equals_mix(S, data):
    """Each request's result is identical alone and inside a concurrent mix."""
    c, reqs = data
    ctx = S.ssj_init(0, n_slots=3, queue_depth=32)
    try:
        h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        alone = []
        for (cand, tn, td, want) in reqs:
            t = S.ssj_stream_submit(ctx, h, cand, tn, td)
            got = _collect(S, ctx, t)
            assert np.array_equal(got, want), (tn, td)
            alone.append(got)
        # the mix: all requests in flight at once, several times over, from 4 threads
        results = {}
        lock = threading.Lock()

        def worker(wid):
            mine = []
            for rep in range(4):
                for i, (cand, tn, td, _) in enumerate(reqs):
                    mine.append((i, S.ssj_stream_submit(ctx, h, cand, tn, td)))
            for i, t in mine:
                got = _collect(S, ctx, t)
                with lock:
                    results.setdefault(i, []).append(got)

        th = [threading.Thread(target=worker, args=(w,)) for w in range(4)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        for i, outs in results.items():
            assert len(outs) == 16
            for got in outs:
                assert np.array_equal(got, alone[i]), i
        # the engine's statistics: slots grew their buffers, and a reset zeroes them
        st = S.ssj_stream_stats(ctx, reset=True)
        _log(f"engine statistics: {st}")
        assert st["slot_grows"] >= 1 and st["slot_grow_ms"] >= 0.0 and st["longest_pass_ms"] > 0.0
        st = S.ssj_stream_stats(ctx)
        assert st["slot_grows"] == 0 and st["result_grows"] == 0 and st["longest_pass_ms"] < 1e3
    finally:
        S.ssj_shutdown(ctx)


def test_stream_tiny_budget_splits_and_queues(S, data):
    c, reqs = data
    # beyond the collection, room for 4 slots of ~2600 pairs: every request is
    # split into several parts
    ctx = S.ssj_init(0, hbm_budget=synth.device_bytes(c) + 4 * 2600 * 40, n_slots=4, queue_depth=4)
    try:
        h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        tickets = [(i, S.ssj_stream_submit(ctx, h, cand, tn, td)) for i, (cand, tn, td, _) in
                   enumerate(reqs)]
        for i, t in tickets:
            assert np.array_equal(_collect(S, ctx, t), reqs[i][3]), i
    finally:
        S.ssj_shutdown(ctx)


def test_stream_poll_states(S, data):
    c, reqs = data
    ctx = S.ssj_init(0, n_slots=2, queue_depth=2)
    try:
        h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        cand, tn, td, want = reqs[0]
        # unknown ticket
        with pytest.raises(S.SsjError) as e:
            S.ssj_stream_poll(ctx, 987654321, wait=False)
        assert e.value.code == S.SSJ_ENOTFOUND
        t = S.ssj_stream_submit(ctx, h, cand, tn, td)
        r = S.ssj_stream_poll(ctx, t, wait=False, out_cap=cand.shape[0])
        if r is None:  # pending; wait now
            r = S.ssj_stream_poll(ctx, t, wait=True, out_cap=cand.shape[0])
        assert np.array_equal(oracle.sort_pairs(r), want)
        with pytest.raises(S.SsjError) as e:  # retired
            S.ssj_stream_poll(ctx, t, wait=False)
        assert e.value.code == S.SSJ_ENOTFOUND
        # truncation keeps the ticket; retry with room succeeds
        assert want.shape[0] > 1
        t = S.ssj_stream_submit(ctx, h, cand, tn, td)
        with pytest.raises(S.SsjError) as e:
            S.ssj_stream_poll(ctx, t, wait=True, out_cap=1)
        assert e.value.code == S.SSJ_ETRUNC and e.value.n == want.shape[0]
        ts, ta, td_ = S.ssj_stream_times(ctx, t, wait=True)
        assert ts <= ta <= td_
        assert np.array_equal(oracle.sort_pairs(S.ssj_stream_poll(ctx, t, True, want.shape[0])), want)
        # an id out of range fails only its own request
        bad = cand.copy()
        bad[3] = [0, c.n_sets + 5]
        tb = S.ssj_stream_submit(ctx, h, bad, tn, td)
        tg = S.ssj_stream_submit(ctx, h, cand, tn, td)
        with pytest.raises(S.SsjError) as e:
            S.ssj_stream_collect(ctx, tb)
        assert e.value.code == S.SSJ_EINVAL
        assert np.array_equal(_collect(S, ctx, tg), want)
        # with admission held, queue_depth (2) requests queue, the next
        # non-blocking submit is refused, and the collection cannot be freed
        S.ssj_stream_pause(ctx, True)
        big = np.concatenate([cand] * 20)
        held = [S.ssj_stream_submit(ctx, h, big, tn, td, nonblocking=True) for _ in range(2)]
        with pytest.raises(S.SsjError) as e:
            S.ssj_stream_submit(ctx, h, big, tn, td, nonblocking=True)
        assert e.value.code == S.SSJ_EAGAIN
        with pytest.raises(S.SsjError) as e:
            S.ssj_free_collection(ctx, h)
        assert e.value.code == S.SSJ_EAGAIN
        time.sleep(0.05)
        assert all(S.ssj_stream_poll(ctx, t, wait=False) is None for t in held)  # still queued
        # a blocking submit waits for a queue place, which resuming frees
        got = []
        th = threading.Thread(target=lambda: got.append(S.ssj_stream_submit(ctx, h, cand, tn, td)))
        th.start()
        time.sleep(0.05)
        assert not got
        S.ssj_stream_pause(ctx, False)
        th.join(timeout=60)
        assert len(got) == 1
        want_big = oracle.sort_pairs(np.concatenate([want] * 20))
        for t in held:
            assert np.array_equal(oracle.sort_pairs(S.ssj_stream_collect(ctx, t)), want_big)
        assert np.array_equal(_collect(S, ctx, got[0]), want)
        # nothing in flight: the collection is freed
        S.ssj_free_collection(ctx, h)
    finally:
        S.ssj_shutdown(ctx)


def test_stream_shutdown_while_paused(S, data):
    """Shutdown resumes a held engine and finishes its queued requests."""
    c, reqs = data
    ctx = S.ssj_init(0, n_slots=1, queue_depth=4)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    cand, tn, td, want = reqs[1]
    S.ssj_stream_pause(ctx, True)
    S.ssj_stream_submit(ctx, h, cand, tn, td)
    S.ssj_shutdown(ctx)


def test_upload_over_budget_is_enomem(S):
    """Collections must fit the context's HBM budget together: an upload that
    would pass it returns SSJ_ENOMEM and uploads nothing; after a free it fits."""
    rng = np.random.default_rng(4)
    c = synth.random_collection(rng, 2000, 60, 50000)
    one = synth.device_bytes(c)                          # device bytes of one copy
    ctx = S.ssj_init(0, hbm_budget=one + one // 2)
    try:
        h1 = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        with pytest.raises(S.SsjError) as e:
            S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        assert e.value.code == S.SSJ_ENOMEM
        # verification still works within what is left of the budget
        cand = rng.integers(0, c.n_sets, size=(5000, 2)).astype(np.int32)
        want = oracle.sort_pairs(oracle.select(c.offsets, c.tokens, cand, 1, 10))
        assert np.array_equal(oracle.sort_pairs(S.ssj_verify(ctx, h1, cand, 1, 10)), want)
        S.ssj_free_collection(ctx, h1)
        h2 = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        assert np.array_equal(oracle.sort_pairs(S.ssj_verify(ctx, h2, cand, 1, 10)), want)
    finally:
        S.ssj_shutdown(ctx)


def test_null_output_with_capacity_is_einval(S, ctx, data):
    """out_cap > 0 with no output buffer is refused before anything is
    enqueued (single, batched and grouped device calls); the count keeps its
    value."""
    import torch
    c, reqs = data
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        cand, tn, td, want = reqs[0]
        d_cand = _dev(torch, cand)
        d_cnt = torch.full((1,), -7, dtype=torch.int64, device="cuda:0")
        lib = S.load_library()
        rc = lib.ssj_verify_device(ctx, h, d_cand.data_ptr(), cand.shape[0], tn, td, None, 10,
                                   d_cnt.data_ptr(), None)
        assert rc == S.SSJ_EINVAL
        req = S.ssj_request(d_cand.data_ptr(), cand.shape[0], tn, td, None, 10, d_cnt.data_ptr(), 0)
        assert lib.ssj_verify_batch_device(ctx, h, ctypes_ref(req), 1, None) == S.SSJ_EINVAL
        g, si = S.groups_of(cand)
        d_g, d_si = _dev(torch, g), _dev(torch, si)
        rc = lib.ssj_verify_groups_device(ctx, h, h, d_g.data_ptr(), g.shape[0], d_si.data_ptr(), si.shape[0],
                                          0, tn, td, None, 10, d_cnt.data_ptr(), None)
        assert rc == S.SSJ_EINVAL
        torch.cuda.synchronize()
        assert int(d_cnt.item()) == -7
    finally:
        S.ssj_free_collection(ctx, h)


def ctypes_ref(x):
    import ctypes
    return ctypes.byref(x)


def test_stream_64_tickets_8_threads(S, data):
    c, reqs = data
    ctx = S.ssj_init(0, n_slots=4, queue_depth=16)
    try:
        h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        out = {}
        lock = threading.Lock()

        def worker(w):
            mine = []
            for k in range(8):
                i = (w + k) % len(reqs)
                cand, tn, td, _ = reqs[i]
                mine.append((i, S.ssj_stream_submit(ctx, h, cand, tn, td)))
                time.sleep(0.001 * (k % 3))
            for i, t in mine:
                got = _collect(S, ctx, t)
                with lock:
                    out[t] = (i, got)

        th = [threading.Thread(target=worker, args=(w,)) for w in range(8)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        assert len(out) == 64
        for t, (i, got) in out.items():
            assert np.array_equal(got, reqs[i][3])
    finally:
        S.ssj_shutdown(ctx)


def test_count_mode_equals_result_size(S, ctx, data):
    """Output-count mode (no pair writes) reports the result size."""
    import torch
    c, reqs = data
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    for plan in [dict(inline_lanes=1, defer_from=5), dict(inline_lanes=16, defer_from=5),
                 dict(inline_lanes=1, defer_from=1, lanes=[4, 8, 32, 256, 256])]:
        S.ssj_set_plan(ctx, S.make_plan(**plan))
        d = [(_dev(torch, cand), tn, td, None, torch.full((1,), -7, dtype=torch.int64, device="cuda:0"))
             for (cand, tn, td, want) in reqs]
        S.ssj_verify_batch_device(ctx, h, d)
        torch.cuda.synchronize()
        for (cand, tn, td, want), (_, _, _, _, cnt) in zip(reqs, d):
            assert int(cnt.item()) == want.shape[0], (plan, tn, td)
        # and a single request through ssj_verify_device
        cand, tn, td, want = reqs[0]
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        S.ssj_verify_device(ctx, h, _dev(torch, cand), tn, td, None, cnt)
        torch.cuda.synchronize()
        assert int(cnt.item()) == want.shape[0]
    S.ssj_free_collection(ctx, h)
