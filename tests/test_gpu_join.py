"""GPU candidate generation (prefix, length and positional filters) and the
whole self-join on the GPU, against the CPU filters of the candidate
generator (element by element, order included) and the oracle."""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import brute  # noqa: E402
from ssj_inputs import synth  # noqa: E402
from ssj_inputs import filter as cfilter  # noqa: E402


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
    S.ssj_set_plan(c, S.make_plan(inline_lanes=1, defer_from=5))
    yield c
    S.ssj_shutdown(c)


def _gpu_candidates(S, ctx, h, tn, td, positional, cap):
    import torch
    dev = torch.device("cuda:0")
    d_out = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=dev)
    d_cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    S.ssj_candidates_device(ctx, h, tn, td, positional, d_out, d_cnt)
    torch.cuda.synchronize()
    k = int(d_cnt.item())
    return k, d_out[:min(k, cap)].cpu().numpy()


def _small_collections():
    out = []
    for seed in range(4):
        rng = np.random.default_rng(9500 + seed)
        out.append(synth.random_collection(rng, n_sets=400, max_size=16, universe=90))
        out.append(synth.near_duplicate_collection(rng, n_base=40, copies=5, max_size=20, universe=100,
                                                   change_frac=0.25))
    return out


def test_candidates_equal_cpu_filters_small(S, ctx):
    for ci, c in enumerate(_small_collections()):
        h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        try:
            for tn, td in [(1, 3), (1, 2), (3, 5), (4, 5), (9, 10), (1, 1)]:
                for pos in (False, True):
                    want = cfilter.candidates(c.offsets, c.tokens, tn, td, positional=pos)
                    _log(f"candidates small #{ci} t={tn}/{td} positional={pos}: {want.shape[0]}")
                    k, got = _gpu_candidates(S, ctx, h, tn, td, pos, want.shape[0] + 8)
                    assert k == want.shape[0] and np.array_equal(got, want), (ci, tn, td, pos)
                # the join itself = brute force
                got = oracle.sort_pairs(S.ssj_join(ctx, h, tn, td, positional=True))
                bj = brute.brute_join(c.offsets, c.tokens, tn, td)
                want = oracle.sort_pairs(np.array(bj, np.int32).reshape(-1, 2))
                assert np.array_equal(got, want), (ci, tn, td)
        finally:
            S.ssj_free_collection(ctx, h)


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_candidates_and_join_on_workloads(S, ctx, golden_dir, cfg):
    import torch
    man = json.load(open(os.path.join(golden_dir, "manifest.json")))[str(cfg)]
    c = synth.workload_collection(cfg)
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        for (tn, td) in synth.WORKLOADS[cfg].thresholds:
            m = man["thresholds"][f"{tn}/{td}"]
            for pos in (False, True):
                want = cfilter.workload_candidates(cfg, tn, td, positional=pos)
                _log(f"candidates config{cfg} t={tn}/{td} positional={pos}: {want.shape[0]}")
                k, got = _gpu_candidates(S, ctx, h, tn, td, pos, want.shape[0])
                assert k == want.shape[0] and np.array_equal(got, want)
            dev = torch.device("cuda:0")
            d_out = torch.empty((max(m["n_result"], 1) + 16, 2), dtype=torch.int32, device=dev)
            d_cnt = torch.zeros(1, dtype=torch.int64, device=dev)
            S.ssj_join_device(ctx, h, tn, td, True, d_out, d_cnt)
            torch.cuda.synchronize()
            k = int(d_cnt.item())
            assert k == m["n_result"]
            assert oracle.result_digest(d_out[:k].cpu().numpy()) == m["result_sha256"]
            got = S.ssj_join(ctx, h, tn, td, positional=False)
            assert got.shape[0] == m["n_result"] and oracle.result_digest(got) == m["result_sha256"]
    finally:
        S.ssj_free_collection(ctx, h)


def test_heavy_tail_candidate_count(S, ctx, golden_dir):
    """The heavy-tail collection's ~1.7e8 prefix-filter candidates: the count the
    CPU filter recorded in the manifest, and a sample of them in order."""
    man = json.load(open(os.path.join(golden_dir, "manifest.json")))["4"]
    c = synth.workload_collection(4)
    (tn, td), = synth.WORKLOADS[4].thresholds
    m = man["thresholds"][f"{tn}/{td}"]
    h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
    try:
        _log("candidates config4")
        k, head = _gpu_candidates(S, ctx, h, tn, td, False, 1 << 20)
        assert k == m["n_candidates"]
        want = cfilter.workload_candidates(4, tn, td)
        assert np.array_equal(head, want[:1 << 20])
    finally:
        S.ssj_free_collection(ctx, h)


def test_join_edges_and_errors(S, ctx):
    # one set, sets of one token, identical sets
    for sets in ([[5]], [[1], [1], [2]], [[1, 2, 3], [1, 2, 3], [1, 2, 4]]):
        c = synth.collection_from_sets(sets)
        h = S.ssj_upload_collection(ctx, c.offsets, c.tokens)
        try:
            for tn, td in [(1, 2), (1, 1)]:
                got = oracle.sort_pairs(S.ssj_join(ctx, h, tn, td))
                bj = brute.brute_join(c.offsets, c.tokens, tn, td)
                assert np.array_equal(got, oracle.sort_pairs(np.array(bj, np.int32).reshape(-1, 2)))
            for tn, td in [(0, 1), (3, 2), (1, 0)]:
                with pytest.raises(S.SsjError) as e:
                    S.ssj_join(ctx, h, tn, td)
                assert e.value.code == S.SSJ_EINVAL
        finally:
            S.ssj_free_collection(ctx, h)
