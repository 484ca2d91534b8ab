"""Host logic of bench.py (no GPU): plan specs, the result digest the bench
compares with the manifest, the committed traffic lookup, and the one-GPU
guard."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import oracle  # noqa: E402
from paper_1812_09141_amd import ssj as S  # noqa: E402


def test_plan_specs():
    assert bench.plan_of(S, "auto") is None
    p = bench.plan_of(S, "inline:1w5").as_dict()
    assert p["inline_lanes"] == 1 and p["defer_from"] == 5 and p["wg_per_cu"] == 5 and p["spill_iters"] == 0
    p = bench.plan_of(S, "inline:1h16").as_dict()
    assert p["hard_lanes"] == 16 and p["wg_per_cu"] == 0
    p = bench.plan_of(S, "defer:1s32x16w4,4,4,8,16,32,64").as_dict()
    assert (p["inline_lanes"], p["spill_iters"], p["spill_lanes"], p["wg_per_cu"], p["defer_from"]) == (1, 32, 16, 4, 4)
    assert list(p["lanes"]) == [4, 8, 16, 32, 64]
    p = bench.plan_of(S, "inline:8").as_dict()
    assert p["inline_lanes"] == 8 and p["spill_lanes"] == 16 and p["staged"] == 0
    p = bench.plan_of(S, "inline:1bs6x64w2").as_dict()
    assert (p["staged"], p["spill_iters"], p["spill_lanes"], p["wg_per_cu"], p["defer_from"]) == (1, 6, 64, 2, 5)
    p = bench.plan_of(S, "defer:1b,3,4,8,16,32,64").as_dict()
    assert p["staged"] == 1 and p["defer_from"] == 3 and p["spill_iters"] == 0
    for bad in ["inline:x", "inline:", "foo:1", "defer:1", "defer:1,2,4,4", "inline:1q3"]:
        with pytest.raises(SystemExit):
            bench.plan_of(S, bad)


def test_pairs_digest_matches_the_oracle_digest():
    """bench.py checks results against manifest digests written with the
    oracle's digest function: the two must agree and ignore order."""
    rng = np.random.default_rng(3)
    pr = rng.integers(0, 1 << 31, (500, 2)).astype(np.int32)
    pr[:50, 0] = pr[50:100, 0]                      # equal r, different s
    d = bench.pairs_digest(pr)
    assert d == oracle.result_digest(pr)
    assert d == bench.pairs_digest(pr[rng.permutation(500)])
    assert d != bench.pairs_digest(pr[:-1])
    assert bench.pairs_digest(np.zeros((0, 2), np.int32)) == oracle.result_digest(np.zeros((0, 2), np.int32))


def test_traffic_lookup_requires_matching_source():
    p = os.path.join(ROOT, "profiles", "verify_tiles_offline_traffic.json")
    d = json.load(open(p))
    assert bench.traffic_from_profiles(d["kernel_source_sha256"], d["workload_key"], d["kernel"]) == d["bytes_per_launch"]
    assert bench.traffic_from_profiles("0" * 64, d["workload_key"], d["kernel"]) is None
    assert bench.traffic_from_profiles(d["kernel_source_sha256"], "heavytail", d["kernel"]) is None
    assert bench.traffic_from_profiles(d["kernel_source_sha256"], d["workload_key"], "k_other") is None


def test_kernel_names_follow_the_plan():
    """The kernel names the bench reports (and looks traffic up by) are the
    instances a plan launches."""
    assert bench.kernel_name_of(bench.plan_of(S, "inline:1w5")) == \
        "k_verify_tiles<1,0,false,false,false,false>"
    assert bench.kernel_name_of(bench.plan_of(S, "inline:1bs6x16")) == \
        "k_verify_tiles<1,0,true,false,true,false> + k_verify_deferred<false,false>"
    assert bench.kernel_name_of(bench.plan_of(S, "inline:1b")) == "k_verify_tiles<1,0,false,false,true,false>"
    assert bench.kernel_name_of(bench.plan_of(S, "defer:16,3,4,8,16,32,64")) == \
        "k_verify_tiles<16,0,true,false,false,false> + k_verify_deferred<false,false>"


def test_default_workloads_lead_with_the_largest():
    """The headline is the heavy-tail workload (the largest configuration),
    with the long-set and offline workloads in the same line."""
    a = bench.parse([])
    assert a.workload.split(",") == ["heavytail", "longsets", "offline"]
    assert a.steps == 20 and a.gpus == 1


def test_host_cpu_reports_threads():
    c = bench.host_cpu()
    assert c["nproc"] >= 1 and c["cpu_count"] >= 1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
