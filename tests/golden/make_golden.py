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
        for (tn, td) in w.thresholds:
            t0 = time.time()
            cand = cfilter.workload_candidates(cfg, tn, td)
            res = oracle.select(c.offsets, c.tokens, cand, tn, td, n_threads=nt)
            cr, cs, _ = oracle.merge_trace(c.offsets, c.tokens, cand, tn, td, n_threads=nt)
            entry["thresholds"][f"{tn}/{td}"] = {
                "n_candidates": int(cand.shape[0]),
                "candidates_sha256": oracle.result_digest(cand),
                "n_result": int(res.shape[0]),
                "result_sha256": oracle.result_digest(res),
                "sum_consumed_tokens": int(cr.astype(np.int64).sum() + cs.astype(np.int64).sum()),
            }
            print(cfg, tn, td, entry["thresholds"][f"{tn}/{td}"], round(time.time() - t0, 1), flush=True)
        man[str(cfg)] = entry
    with open(OUT, "w") as f:
        json.dump(man, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [1, 2, 3, 4])
