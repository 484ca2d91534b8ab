"""GPU parity for R-S joins (Definition 1 with two collections) and for the
grouped candidate layout of Sec. 3.3.1 (a probe id and the exclusive end of
its candidates, then 4-byte s ids): libssj through the C ABI against the
oracle, bit-exact."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from ssj_inputs import synth  # noqa: E402
from ssj_inputs import filter as cfilter  # noqa: E402

PLANS = [
    ("inline-1", dict(inline_lanes=1, defer_from=5)),
    ("inline-1-spill", dict(inline_lanes=1, defer_from=5, spill_iters=1, spill_lanes=16)),
    ("inline-1h8", dict(inline_lanes=1, hard_lanes=8, defer_from=5)),
    ("inline-8", dict(inline_lanes=8, defer_from=5)),
    ("deferred-4", dict(inline_lanes=4, defer_from=0, lanes=[4] * 5)),
    ("deferred-256", dict(inline_lanes=4, defer_from=0, lanes=[256] * 5)),
    ("ring", dict(inline_lanes=1, defer_from=5, staged=1)),
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


def _two(seed, max_size):
    """R and S cut from one near-duplicate collection (many similar cross pairs),
    of different sizes and set lengths."""
    rng = np.random.default_rng(9300 + seed)
    c = synth.near_duplicate_collection(rng, n_base=30, copies=5, max_size=max_size,
                                        universe=4 * max_size, change_frac=0.2)
    sets = [c.tokens[c.offsets[i]:c.offsets[i + 1]].tolist() for i in range(c.n_sets)]
    order = rng.permutation(len(sets))
    cut = len(sets) // 3
    R = synth.collection_from_sets([sets[i] for i in order[:cut]])
    Sc = synth.collection_from_sets([sets[i] for i in order[cut:]])
    return rng, R, Sc


def _cross(nr, ns):
    i, j = np.meshgrid(np.arange(nr), np.arange(ns), indexing="ij")
    return np.stack([i.ravel(), j.ravel()], axis=1).astype(np.int32)


@pytest.mark.parametrize("seed,max_size", [(0, 12), (1, 60), (2, 400)])
def test_rs_all_plans(S, ctx, seed, max_size):
    rng, R, Sc = _two(seed, max_size)
    hr = S.ssj_upload_collection(ctx, R.offsets, R.tokens)
    hs = S.ssj_upload_collection(ctx, Sc.offsets, Sc.tokens)
    try:
        cand = _cross(R.n_sets, Sc.n_sets)
        cand = np.concatenate([cand, cand[rng.integers(0, cand.shape[0], 300)]])  # repeats
        for sim, ts in [("jaccard", [(1, 2), (4, 5)]), ("cosine", [(11, 20)]), ("dice", [(3, 5)]),
                        ("overlap", [(5, 1)])]:
            for tn, td in ts:
                want = oracle.sort_pairs(oracle.select_rs(R.offsets, R.tokens, Sc.offsets, Sc.tokens,
                                                          cand, tn, td, sim=sim))
                for name, plan in PLANS:
                    _log(f"rs seed={seed} {sim} t={tn}/{td} plan={name}")
                    S.ssj_set_plan(ctx, S.make_plan(**plan))
                    got = oracle.sort_pairs(S.ssj_verify_rs(ctx, hr, hs, cand, sim, tn, td))
                    assert np.array_equal(got, want), (sim, tn, td, name)
    finally:
        S.ssj_free_collection(ctx, hr)
        S.ssj_free_collection(ctx, hs)


def test_rs_device_count_mode_and_id_errors(S, ctx):
    import torch
    rng, R, Sc = _two(3, 30)
    hr = S.ssj_upload_collection(ctx, R.offsets, R.tokens)
    hs = S.ssj_upload_collection(ctx, Sc.offsets, Sc.tokens)
    try:
        S.ssj_set_plan(ctx, S.make_plan(inline_lanes=1, defer_from=3, lanes=[4, 8, 16, 32, 256]))
        cand = _cross(R.n_sets, Sc.n_sets)
        want = oracle.sort_pairs(oracle.select_rs(R.offsets, R.tokens, Sc.offsets, Sc.tokens,
                                                  cand, 3, 5))
        dev = torch.device("cuda:0")
        d_cand = torch.from_numpy(cand).to(dev)
        d_out = torch.empty_like(d_cand)
        d_cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        _log("rs device")
        S.ssj_verify_rs_device(ctx, hr, hs, d_cand, "jaccard", 3, 5, d_out, d_cnt)
        torch.cuda.synchronize()
        k = int(d_cnt.item())
        assert np.array_equal(oracle.sort_pairs(d_out[:k].cpu().numpy()), want)
        S.ssj_verify_rs_device(ctx, hr, hs, d_cand, "jaccard", 3, 5, None, d_cnt)
        torch.cuda.synchronize()
        assert int(d_cnt.item()) == want.shape[0]
        # an s id valid in R but not in S (and the reverse) is an id error
        assert R.n_sets < Sc.n_sets
        for bad in ([0, Sc.n_sets], [R.n_sets, 0], [-1, 0]):
            with pytest.raises(S.SsjError) as e:
                S.ssj_verify_rs(ctx, hr, hs, np.array([[0, 0], bad], np.int32), "jaccard", 1, 2)
            assert e.value.code == S.SSJ_EINVAL
        # ids of S beyond |R| are fine on the s side
        ok = np.array([[0, Sc.n_sets - 1], [R.n_sets - 1, R.n_sets]], np.int32)
        got = oracle.sort_pairs(S.ssj_verify_rs(ctx, hr, hs, ok, "jaccard", 0, 1))
        assert np.array_equal(got, oracle.sort_pairs(ok))
    finally:
        S.ssj_free_collection(ctx, hr)
        S.ssj_free_collection(ctx, hs)


def _uneven_groups(rng, n_probe, sizes):
    """Grouped candidates with the given group sizes (0 = empty group)."""
    probes = rng.integers(0, n_probe, len(sizes)).astype(np.int32)
    ends = np.cumsum(sizes).astype(np.int32)
    return np.stack([probes, ends], axis=1)


def test_groups_self_join_config2(S, ctx, golden_dir):
    """The filter's probe-grouped candidates of the offline collection, sent as
    groups (4 bytes per candidate), give the flat result."""
    import json
    import torch
    man = json.load(open(os.path.join(golden_dir, "manifest.json")))["2"]
    c = synth.workload_collection(2)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        S.ssj_set_plan(ctx, S.make_plan(inline_lanes=1, defer_from=5))
        for tn, td in [(3, 5), (4, 5)]:
            cand = cfilter.workload_candidates(2, tn, td)
            groups, sids = S.groups_of(cand)
            m = man["thresholds"][f"{tn}/{td}"]
            _log(f"groups config2 t={tn}/{td}: {groups.shape[0]} groups, {sids.shape[0]} candidates")
            got = S.ssj_verify_groups(ctx, h, h, groups, sids, "jaccard", tn, td)
            assert got.shape[0] == m["n_result"] and oracle.result_digest(got) == m["result_sha256"]
            dev = torch.device("cuda:0")
            d_g = torch.from_numpy(groups).to(dev)
            d_s = torch.from_numpy(sids).to(dev)
            d_out = torch.empty((sids.shape[0], 2), dtype=torch.int32, device=dev)
            d_cnt = torch.zeros(1, dtype=torch.int64, device=dev)
            S.ssj_verify_groups_device(ctx, h, h, d_g, d_s, "jaccard", tn, td, d_out, d_cnt)
            torch.cuda.synchronize()
            k = int(d_cnt.item())
            assert k == m["n_result"]
            assert oracle.result_digest(d_out[:k].cpu().numpy()) == m["result_sha256"]
    finally:
        S.ssj_free_collection(ctx, h)


def test_groups_rs_uneven(S, ctx):
    """Empty groups, one-candidate groups, groups across chunk seams, a group of
    thousands of candidates, many groups inside one chunk."""
    import torch
    rng, R, Sc = _two(4, 40)
    hr = S.ssj_upload_collection(ctx, R.offsets, R.tokens)
    hs = S.ssj_upload_collection(ctx, Sc.offsets, Sc.tokens)
    try:
        sizes = ([0, 0, 1, 63, 1, 0, 64, 65, 5000, 0] + [1] * 200 + [0] * 70 + [3] * 40
                 + list(rng.integers(0, 150, 60)) + [0])
        groups = _uneven_groups(rng, R.n_sets, sizes)
        n = int(groups[-1, 1])
        sids = rng.integers(0, Sc.n_sets, n).astype(np.int32)
        flat = np.stack([np.repeat(groups[:, 0], sizes), sids], axis=1).astype(np.int32)
        dev = torch.device("cuda:0")
        for name, plan in PLANS[:3]:
            S.ssj_set_plan(ctx, S.make_plan(**plan))
            for tn, td in [(0, 1), (1, 3), (3, 5)]:
                want = oracle.sort_pairs(oracle.select_rs(R.offsets, R.tokens, Sc.offsets, Sc.tokens,
                                                          flat, tn, td))
                _log(f"groups rs {name} t={tn}/{td} n={n}")
                got = oracle.sort_pairs(S.ssj_verify_groups(ctx, hr, hs, groups, sids, "jaccard",
                                                            tn, td))
                assert np.array_equal(got, want), (name, tn, td)
                d_out = torch.empty((n, 2), dtype=torch.int32, device=dev)
                d_cnt = torch.zeros(1, dtype=torch.int64, device=dev)
                S.ssj_verify_groups_device(ctx, hr, hs, torch.from_numpy(groups).to(dev),
                                           torch.from_numpy(sids).to(dev), "jaccard", tn, td,
                                           d_out, d_cnt)
                torch.cuda.synchronize()
                k = int(d_cnt.item())
                assert np.array_equal(oracle.sort_pairs(d_out[:k].cpu().numpy()), want)
    finally:
        S.ssj_free_collection(ctx, hr)
        S.ssj_free_collection(ctx, hs)


def test_groups_split_across_batches(S):
    """A budget of a few KiB splits the candidates into many batches, with
    groups cut at batch borders."""
    rng, R, Sc = _two(5, 20)
    ctx = S.ssj_init(0, hbm_budget=synth.device_bytes(R) + synth.device_bytes(Sc) + 44 * 1000)
    try:
        hr = S.ssj_upload_collection(ctx, R.offsets, R.tokens)
        hs = S.ssj_upload_collection(ctx, Sc.offsets, Sc.tokens)
        sizes = [3000, 0, 1, 2500, 999, 1001, 0, 4000]
        groups = _uneven_groups(rng, R.n_sets, sizes)
        n = int(groups[-1, 1])
        sids = rng.integers(0, Sc.n_sets, n).astype(np.int32)
        flat = np.stack([np.repeat(groups[:, 0], sizes), sids], axis=1).astype(np.int32)
        want = oracle.sort_pairs(oracle.select_rs(R.offsets, R.tokens, Sc.offsets, Sc.tokens,
                                                  flat, 1, 3))
        _log("groups batches")
        got = oracle.sort_pairs(S.ssj_verify_groups(ctx, hr, hs, groups, sids, "jaccard", 1, 3))
        assert np.array_equal(got, want)
        S.ssj_free_collection(ctx, hr)
        S.ssj_free_collection(ctx, hs)
    finally:
        S.ssj_shutdown(ctx)


def test_groups_malformed(S, ctx):
    import torch
    rng, R, Sc = _two(6, 20)
    hr = S.ssj_upload_collection(ctx, R.offsets, R.tokens)
    hs = S.ssj_upload_collection(ctx, Sc.offsets, Sc.tokens)
    try:
        S.ssj_set_plan(ctx, S.make_plan(inline_lanes=1, defer_from=5))
        sids = rng.integers(0, Sc.n_sets, 300).astype(np.int32)
        good = np.array([[0, 100], [1, 250], [2, 300]], np.int32)
        assert S.ssj_verify_groups(ctx, hr, hs, good, sids, "jaccard", 0, 1).shape[0] == 300
        host_bad = [np.array([[0, 200], [1, 100], [2, 300]], np.int32),   # decreasing ends
                    np.array([[0, 100], [1, 250]], np.int32),               # short of n_cand
                    np.array([[0, 100], [1, 301]], np.int32)]               # past n_cand
        for g in host_bad:
            with pytest.raises(S.SsjError) as e:
                S.ssj_verify_groups(ctx, hr, hs, g, sids, "jaccard", 1, 2)
            assert e.value.code == S.SSJ_EINVAL
        bad_probe = np.array([[0, 100], [R.n_sets, 300]], np.int32)
        with pytest.raises(S.SsjError) as e:
            S.ssj_verify_groups(ctx, hr, hs, bad_probe, sids, "jaccard", 1, 2)
        assert e.value.code == S.SSJ_EINVAL
        dev = torch.device("cuda:0")
        d_s = torch.from_numpy(sids).to(dev)
        d_out = torch.empty((300, 2), dtype=torch.int32, device=dev)
        d_cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        for g in host_bad[:2] + [bad_probe, np.zeros((0, 2), np.int32)]:
            _log(f"groups malformed device {g.tolist()}")
            d_g = torch.from_numpy(g).to(dev) if g.shape[0] else torch.zeros((1, 2), dtype=torch.int32, device=dev)[:0]
            S.ssj_verify_groups_device(ctx, hr, hs, d_g, d_s, "jaccard", 1, 2, d_out, d_cnt)
            torch.cuda.synchronize()
            assert int(d_cnt.item()) == -1, g.tolist()
        # the context keeps working
        d_g = torch.from_numpy(good).to(dev)
        S.ssj_verify_groups_device(ctx, hr, hs, d_g, d_s, "jaccard", 0, 1, d_out, d_cnt)
        torch.cuda.synchronize()
        assert int(d_cnt.item()) == 300
    finally:
        S.ssj_free_collection(ctx, hr)
        S.ssj_free_collection(ctx, hs)


def test_groups_many_and_malformed_large(S, ctx):
    """Tens of thousands of groups (several rounds of the chunk's group search)
    with runs of hundreds of empty groups; then malformed ends deep inside the
    list, where no chunk's own groups reach them, still give -1, and a
    well-formed call afterwards is unaffected."""
    import torch
    rng, R, Sc = _two(7, 30)
    hr = S.ssj_upload_collection(ctx, R.offsets, R.tokens)
    hs = S.ssj_upload_collection(ctx, Sc.offsets, Sc.tokens)
    try:
        S.ssj_set_plan(ctx, S.make_plan(inline_lanes=1, defer_from=5))
        sizes = []
        while len(sizes) < 30000:
            kind = rng.integers(0, 10)
            if kind == 0:
                sizes += [0] * int(rng.integers(64, 400))
            elif kind == 1:
                sizes.append(int(rng.integers(100, 300)))
            else:
                sizes += rng.integers(0, 6, 50).tolist()
        groups = _uneven_groups(rng, R.n_sets, sizes)
        n = int(groups[-1, 1])
        sids = rng.integers(0, Sc.n_sets, n).astype(np.int32)
        flat = np.stack([np.repeat(groups[:, 0], sizes), sids], axis=1).astype(np.int32)
        want = oracle.sort_pairs(oracle.select_rs(R.offsets, R.tokens, Sc.offsets, Sc.tokens, flat, 0, 1))
        dev = torch.device("cuda:0")
        d_s = torch.from_numpy(sids).to(dev)
        d_out = torch.empty((n, 2), dtype=torch.int32, device=dev)
        d_cnt = torch.zeros(1, dtype=torch.int64, device=dev)

        def run(g):
            S.ssj_verify_groups_device(ctx, hr, hs, torch.from_numpy(g).to(dev), d_s, "jaccard", 0, 1,
                                       d_out, d_cnt)
            torch.cuda.synchronize()
            return int(d_cnt.item())

        _log(f"groups many: {groups.shape[0]} groups, {n} candidates")
        assert run(groups) == want.shape[0]
        assert np.array_equal(oracle.sort_pairs(d_out[:want.shape[0]].cpu().numpy()), want)
        mid = int(np.flatnonzero((groups[:, 1] > 0) & (np.arange(groups.shape[0]) > 15000))[0]) + 1
        bad = []
        g = groups.copy()
        g[mid, 1] = g[mid - 1, 1] - 1           # one end below the one before
        bad.append(("decrease", g))
        g = groups.copy()
        g[mid, 1] = n + 7                       # an end past n_cand
        bad.append(("past n", g))
        g = groups.copy()
        g[-1, 1] = n - 1                        # the last end short of n_cand
        bad.append(("short", g))
        g = groups.copy()
        g[mid, 1] = -5                          # a negative end
        bad.append(("negative", g))
        for name, g in bad:
            _log(f"groups many malformed: {name} at group {mid}")
            assert run(g) == -1, name
        assert run(groups) == want.shape[0]
    finally:
        S.ssj_free_collection(ctx, hr)
        S.ssj_free_collection(ctx, hs)


def test_groups_batch_one_launch(S, ctx, golden_dir):
    """The offline step's four threshold lists as grouped requests of one
    batched launch give the manifest results; a malformed request inside a
    batch gets -1 and leaves the others exact; a mixed-function batch equals
    the single calls."""
    import json
    import torch
    man = json.load(open(os.path.join(golden_dir, "manifest.json")))["2"]
    c = synth.workload_collection(2)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    dev = torch.device("cuda:0")
    try:
        S.ssj_set_plan(ctx, S.make_plan(inline_lanes=1, defer_from=5))
        reqs, meta = [], []
        for tn, td in synth.WORKLOADS[2].thresholds:
            g, si = S.groups_of(cfilter.workload_candidates(2, tn, td))
            d_out = torch.empty((si.shape[0], 2), dtype=torch.int32, device=dev)
            d_cnt = torch.full((1,), -7, dtype=torch.int64, device=dev)
            reqs.append((torch.from_numpy(g).to(dev), torch.from_numpy(si).to(dev), tn, td, d_out, d_cnt))
            meta.append(man["thresholds"][f"{tn}/{td}"])
        _log("groups batch: four thresholds")
        S.ssj_verify_groups_batch_device(ctx, h, h, reqs)
        torch.cuda.synchronize()
        for (_, _, tn, td, d_out, d_cnt), m in zip(reqs, meta):
            k = int(d_cnt.item())
            assert k == m["n_result"], (tn, td)
            assert oracle.result_digest(d_out[:k].cpu().numpy()) == m["result_sha256"]
        # a malformed request (decreasing ends) in the middle of the batch
        bad_g = reqs[1][0].clone()
        bad_g[5, 1] = bad_g[4, 1] - 1
        mixed = [reqs[0], (bad_g,) + reqs[1][1:], reqs[2], reqs[3]]
        for r in mixed:
            r[5].fill_(-7)
        _log("groups batch: malformed second request")
        S.ssj_verify_groups_batch_device(ctx, h, h, mixed)
        torch.cuda.synchronize()
        assert int(mixed[1][5].item()) == -1
        for i in (0, 2, 3):
            k = int(mixed[i][5].item())
            assert k == meta[i]["n_result"]
            assert oracle.result_digest(mixed[i][4][:k].cpu().numpy()) == meta[i]["result_sha256"]
        # other similarity functions in one batch, against single grouped calls
        g0, s0 = reqs[1][0], reqs[1][1]
        sims = [("dice", 7, 10), ("cosine", 3, 5), ("overlap", 8, 1), ("jaccard", 1, 2)]
        outs = [(torch.empty((s0.numel(), 2), dtype=torch.int32, device=dev),
                 torch.zeros(1, dtype=torch.int64, device=dev)) for _ in sims]
        S.ssj_verify_groups_batch_device(ctx, h, h, [(g0, s0, tn, td, o, n, sim)
                                                     for (sim, tn, td), (o, n) in zip(sims, outs)])
        torch.cuda.synchronize()
        for (sim, tn, td), (o, n) in zip(sims, outs):
            o1 = torch.empty_like(o)
            n1 = torch.zeros(1, dtype=torch.int64, device=dev)
            S.ssj_verify_groups_device(ctx, h, h, g0, s0, sim, tn, td, o1, n1)
            torch.cuda.synchronize()
            k = int(n.item())
            assert k == int(n1.item()) >= 0, sim
            assert np.array_equal(oracle.sort_pairs(o[:k].cpu().numpy()), oracle.sort_pairs(o1[:k].cpu().numpy()))
        with pytest.raises(S.SsjError):
            S.ssj_verify_groups_batch_device(ctx, h, h, [reqs[0]] * 17)
    finally:
        S.ssj_free_collection(ctx, h)


# Every mapping family on grouped candidates: the in-order kernel's
# thread-per-pair pipeline, its lane groups (pairs handed on by permutes),
# the staged kernel, and the deferred kernel, which reads the probe ids
# that the in-order kernel stored for the pairs it queued.
GROUP_PLANS = PLANS + [
    ("inline-1h16-defer", dict(inline_lanes=1, hard_lanes=16, defer_from=1, lanes=[4, 16, 32, 64, 256])),
    ("inline-32", dict(inline_lanes=32, defer_from=5)),
    ("inline-64", dict(inline_lanes=64, defer_from=5)),
    ("deferred-1", dict(inline_lanes=4, defer_from=0, lanes=[1] * 5)),
    ("deferred-64", dict(inline_lanes=16, defer_from=0, lanes=[64] * 5)),
    ("spill-2x1-defer", dict(inline_lanes=1, defer_from=2, lanes=[4, 8, 32, 64, 256], spill_iters=2,
                             spill_lanes=1)),
    ("spill-1x256", dict(inline_lanes=1, defer_from=5, spill_iters=1, spill_lanes=256)),
    ("staged", dict(inline_lanes=1, defer_from=5, staged=1)),
    ("staged-spill-1x16", dict(inline_lanes=1, defer_from=5, staged=1, spill_iters=1, spill_lanes=16)),
    ("staged-defer", dict(inline_lanes=1, defer_from=2, lanes=[4, 8, 32, 64, 256], staged=1)),
    ("graph", dict(inline_lanes=8, defer_from=2, lanes=[4, 16, 16, 64, 256], use_graph=1)),
    ("inline-1-wg1", dict(inline_lanes=1, defer_from=5, wg_per_cu=1)),
]


def test_groups_every_mapping(S, ctx):
    """Grouped candidates over long near-duplicate sets (merges past the set
    records, deferred classes, spilled merges) with empty groups, runs of more
    than 64 empty groups inside one chunk, one-candidate groups and a group of
    thousands, in every mapping; two grouped requests of one batched launch."""
    import torch
    rng, R, Sc = _two(8, 400)
    hr = S.ssj_upload_collection(ctx, R.offsets, R.tokens)
    hs = S.ssj_upload_collection(ctx, Sc.offsets, Sc.tokens)
    try:
        sizes = ([0, 3, 0] + [0] * 150 + [2, 1] + [0] * 70 + [1] * 130 + [64, 65, 63, 0, 2500]
                 + list(rng.integers(0, 40, 80)) + [0] * 65 + [7] + list(rng.integers(0, 3, 300)) + [0])
        groups = _uneven_groups(rng, R.n_sets, sizes)
        n = int(groups[-1, 1])
        # half of each probe's candidates among the S sets similar to it at
        # t = 1/2 (found by the oracle over all cross pairs), so that many pass
        cross = _cross(R.n_sets, Sc.n_sets)
        close = oracle.select_rs(R.offsets, R.tokens, Sc.offsets, Sc.tokens, cross, 1, 2)
        near = [close[close[:, 0] == r, 1] for r in range(R.n_sets)]
        probe_of = np.repeat(groups[:, 0], sizes)
        sids = rng.integers(0, Sc.n_sets, n).astype(np.int32)
        for k in range(n):
            nb = near[probe_of[k]]
            if nb.shape[0] and rng.random() < 0.5:
                sids[k] = nb[rng.integers(0, nb.shape[0])]
        flat = np.stack([probe_of, sids], axis=1).astype(np.int32)
        dev = torch.device("cuda:0")
        d_g = torch.from_numpy(groups).to(dev)
        d_s = torch.from_numpy(sids).to(dev)
        # the second request: the first half of the groups, cut to end where they end
        half = groups.shape[0] // 2
        g2 = groups[:half].copy()
        n2 = int(g2[-1, 1])
        d_g2 = torch.from_numpy(g2).to(dev)
        d_s2 = d_s[:n2].contiguous()
        wants = {}
        for tn, td in [(1, 4), (3, 5)]:
            wants[(tn, td)] = oracle.sort_pairs(oracle.select_rs(R.offsets, R.tokens, Sc.offsets, Sc.tokens,
                                                                 flat, tn, td))
        want2 = oracle.sort_pairs(oracle.select_rs(R.offsets, R.tokens, Sc.offsets, Sc.tokens, flat[:n2], 1, 2))
        assert wants[(3, 5)].shape[0] > 50 and want2.shape[0] > 50
        d_out = torch.empty((n, 2), dtype=torch.int32, device=dev)
        d_out2 = torch.empty((n2, 2), dtype=torch.int32, device=dev)
        d_cnt = torch.zeros(2, dtype=torch.int64, device=dev)
        for name, plan in GROUP_PLANS:
            S.ssj_set_plan(ctx, S.make_plan(**plan))
            for (tn, td), want in wants.items():
                _log(f"groups every mapping {name} t={tn}/{td} n={n}")
                S.ssj_verify_groups_device(ctx, hr, hs, d_g, d_s, "jaccard", tn, td, d_out, d_cnt[:1])
                torch.cuda.synchronize()
                k = int(d_cnt[0].item())
                assert k == want.shape[0], (name, tn, td)
                assert np.array_equal(oracle.sort_pairs(d_out[:k].cpu().numpy()), want), (name, tn, td)
            _log(f"groups every mapping {name}: two grouped requests in one launch")
            S.ssj_verify_groups_batch_device(ctx, hr, hs, [(d_g, d_s, 3, 5, d_out, d_cnt[0:1]),
                                                          (d_g2, d_s2, 1, 2, d_out2, d_cnt[1:2])])
            torch.cuda.synchronize()
            k1, k2 = (int(x) for x in d_cnt.cpu().numpy())
            assert k1 == wants[(3, 5)].shape[0] and k2 == want2.shape[0], name
            assert np.array_equal(oracle.sort_pairs(d_out[:k1].cpu().numpy()), wants[(3, 5)]), name
            assert np.array_equal(oracle.sort_pairs(d_out2[:k2].cpu().numpy()), want2), name
    finally:
        S.ssj_free_collection(ctx, hr)
        S.ssj_free_collection(ctx, hs)
