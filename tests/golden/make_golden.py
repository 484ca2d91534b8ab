"""Writes tests/golden/manifest.json: per workload and threshold, the
collection digest, the candidate count, and the oracle's result count and
SHA-256 of the sorted result.  Calls only the input generators and the
oracle (never the GPU library).

    python tests/golden/make_golden.py [cfg ...]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from ssj_inputs import filter as cfilter  # noqa: E402
from ssj_inputs import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "manifest.json")

# Other similarity functions of Table 1 over the offline workload's t = 0.6
# candidates (the overlap threshold is a count).
SIM_CASES = {2: ((3, 5), (("dice", 7, 10), ("cosine", 3, 5), ("overlap", 8, 1)))}
# Lower thresholds where the random collections have passing pairs: a
# workload's own filter and verification at that threshold ("extra"), or its
# stated threshold's candidates verified at a lower one ("verify_at").
EXTRA_THRESHOLDS = {1: ((1, 2),)}
VERIFY_AT = {3: ((7, 10), ((1, 10), (1, 5), (3, 10)))}
# Streamed batches (count, schedule seed) of the serving workload, as the
# benchmark draws them: per batch the oracle's result count and digest.
STREAM_CASES = {5: (200, 0)}
# Buckets of |r| + |s| for per-bucket figures on the heavy-tail workload
# (inclusive upper bounds; the last bucket is open).
SIZE_BUCKETS = {4: (32, 128, 512, 2048)}


def bucket_stats(c, cand, res, cr, cs, bounds):
    """Candidates, consumed tokens, results and the result digest per bucket of |r| + |s|."""
    sizes = np.diff(c.offsets)
    b_cand = np.searchsorted(np.asarray(bounds), sizes[cand[:, 0]] + sizes[cand[:, 1]], side="left")
    b_res = np.searchsorted(np.asarray(bounds), sizes[res[:, 0]] + sizes[res[:, 1]], side="left")
    consumed = cr.astype(np.int64) + cs.astype(np.int64)
    out = []
    for q in range(len(bounds) + 1):
        rq = res[b_res == q]
        out.append({"upper_bound": int(bounds[q]) if q < len(bounds) else None,
                    "n_candidates": int((b_cand == q).sum()),
                    "sum_consumed_tokens": int(consumed[b_cand == q].sum()),
                    "n_result": int(rq.shape[0]), "result_sha256": oracle.result_digest(rq)})
    return out


def main(cfgs):
    man = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            man = json.load(f)
    nt = os.cpu_count() or 1
    for cfg in cfgs:
        w = synth.WORKLOADS[cfg]
        c = synth.workload_collection(cfg)
        entry = {"collection_sha256": c.digest(), "n_sets": c.n_sets, "n_tokens": c.n_tokens,
                 "generator_version": synth.GEN_VERSION, "numpy": np.__version__, "thresholds": {}}
        extra = EXTRA_THRESHOLDS.get(cfg, ())
        for (tn, td) in tuple(w.thresholds) + tuple(extra):
            t0 = time.time()
            cand = cfilter.workload_candidates(cfg, tn, td)
            res = oracle.select(c.offsets, c.tokens, cand, tn, td, n_threads=nt)
            cr, cs, _ = oracle.merge_trace(c.offsets, c.tokens, cand, tn, td, n_threads=nt)
            key = "extra_thresholds" if (tn, td) in extra else "thresholds"
            entry.setdefault(key, {})[f"{tn}/{td}"] = {
                "n_candidates": int(cand.shape[0]),
                "candidates_sha256": oracle.result_digest(cand),
                "n_result": int(res.shape[0]),
                "result_sha256": oracle.result_digest(res),
                "sum_consumed_tokens": int(cr.astype(np.int64).sum() + cs.astype(np.int64).sum()),
            }
            if cfg in SIZE_BUCKETS:
                entry["thresholds"][f"{tn}/{td}"]["buckets"] = bucket_stats(c, cand, res, cr, cs,
                                                                            SIZE_BUCKETS[cfg])
            print(cfg, tn, td, entry[key][f"{tn}/{td}"], round(time.time() - t0, 1), flush=True)
        if cfg in VERIFY_AT:
            (tn, td), lower = VERIFY_AT[cfg]
            cand = cfilter.workload_candidates(cfg, tn, td)
            entry["verify_at"] = {"candidates": f"{tn}/{td}"}
            for (vn, vd) in lower:
                res = oracle.select(c.offsets, c.tokens, cand, vn, vd, n_threads=nt)
                cr, cs, _ = oracle.merge_trace(c.offsets, c.tokens, cand, vn, vd, n_threads=nt)
                entry["verify_at"][f"{vn}/{vd}"] = {
                    "n_result": int(res.shape[0]), "result_sha256": oracle.result_digest(res),
                    "sum_consumed_tokens": int(cr.astype(np.int64).sum() + cs.astype(np.int64).sum())}
            print(cfg, entry["verify_at"], flush=True)
        if cfg in SIM_CASES:
            (tn, td), cases = SIM_CASES[cfg]
            cand = cfilter.workload_candidates(cfg, tn, td)
            entry["sims"] = {"candidates": f"{tn}/{td}"}
            for sim, sn, sd in cases:
                res = oracle.select(c.offsets, c.tokens, cand, sn, sd, n_threads=nt, sim=sim)
                entry["sims"][f"{sim} {sn}/{sd}"] = {"n_result": int(res.shape[0]),
                                                      "result_sha256": oracle.result_digest(res)}
            print(cfg, entry["sims"], flush=True)
        if cfg in STREAM_CASES:
            n_b, seed = STREAM_CASES[cfg]
            from paper_1812_09141_amd import serving
            sizes, ts, _ = synth.stream_schedule(n_b, seed=seed, thresholds=w.thresholds)
            batches = serving.build_batches(c.offsets, c.tokens, sizes, ts, n_threads=nt)
            per = []
            for (b, tn, td) in batches:
                res = oracle.select(c.offsets, c.tokens, b, tn, td, n_threads=nt)
                per.append({"t": f"{tn}/{td}", "n_candidates": int(b.shape[0]), "n_result": int(res.shape[0]),
                            "result_sha256": oracle.result_digest(res)})
            entry["stream"] = {"n_batches": n_b, "seed": seed, "batches": per}
            print(cfg, "stream", n_b, sum(x["n_result"] for x in per), flush=True)
        man[str(cfg)] = entry
    with open(OUT, "w") as f:
        json.dump(man, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [1, 2, 3, 4, 5])
