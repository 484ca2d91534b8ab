"""Serving driver: CPU filter threads feed candidate batches to the stream API.

The paper's host side runs the filtering thread H0 next to a device handler
H1 and a post-processing thread H2, so that verification of one chunk
overlaps the filtering of the next (Sec. 3.2, Sec. 4.1.2).  Here the device
handler is libssj's stream engine (ssj_stream_submit / ssj_stream_poll);
this module supplies the producer side -- AllPairs filter threads that cut
the candidate stream into batches -- and a replay loop that submits batches
at Poisson arrival times and records per-batch latency from the engine's own
timestamps (submit entry to results on the host).
"""
from __future__ import annotations

import threading
import time
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from ssj_inputs import filter as cfilter


class CandidateStream:
    """Candidate pairs of one collection at one threshold, cut into batches of
    whole probes (the filter emits a probe's candidates together).  The stream
    wraps around at the end of the collection."""

    def __init__(self, offsets, tokens, t_num: int, t_den: int, n_threads: int = 8):
        self.t = (int(t_num), int(t_den))
        self.index = cfilter.PrefixIndex(offsets, tokens, t_num, t_den)
        lib = cfilter._load()
        counts = np.zeros(self.index.n_sets, dtype=np.int64)
        self.total = int(lib.ssjf_count(self.index._h, n_threads, counts.ctypes.data))
        self.cum = np.zeros(self.index.n_sets + 1, dtype=np.int64)
        np.cumsum(counts, out=self.cum[1:])
        self.cursor = 0

    def next_range(self, want: int) -> Tuple[int, int, int]:
        """Probe range [a, b) holding about `want` candidates (at least one probe)."""
        if self.total == 0:
            return 0, 0, 0
        a = self.cursor
        if self.cum[a] == self.total:  # no candidates left after a: wrap
            a = 0
        target = self.cum[a] + max(1, want)
        b = int(np.searchsorted(self.cum, target, side="left"))
        b = max(a + 1, min(b, self.index.n_sets))
        self.cursor = b if b < self.index.n_sets else 0
        return a, b, int(self.cum[b] - self.cum[a])

    def fill(self, a: int, b: int, n: int) -> np.ndarray:
        out = np.empty((n, 2), dtype=np.int32)
        got, nxt = self.index.probe(a, b, out)
        if got != n or nxt != b:
            raise RuntimeError("filter produced an unexpected batch")
        return out

    def close(self):
        self.index.close()


def build_batches(offsets, tokens, sizes: Sequence[int], thresholds: Sequence[Tuple[int, int]],
                  n_threads: int = 8) -> List[Tuple[np.ndarray, int, int]]:
    """Cuts the candidate streams into batches of about sizes[i] pairs at
    thresholds[i]; the filter work runs on n_threads threads."""
    streams: Dict[Tuple[int, int], CandidateStream] = {}
    plan = []
    for size, t in zip(sizes, thresholds):
        if t not in streams:
            streams[t] = CandidateStream(offsets, tokens, t[0], t[1], n_threads)
        a, b, n = streams[t].next_range(int(size))
        plan.append((t, a, b, n))
    with ThreadPoolExecutor(max_workers=n_threads) as ex:
        futs = [ex.submit(streams[t].fill, a, b, n) for (t, a, b, n) in plan]
        batches = [(f.result(), t[0], t[1]) for f, (t, a, b, n) in zip(futs, plan)]
    for s in streams.values():
        s.close()
    return batches


def run_stream(S, ctx, coll, batches, rate_pairs_per_s: Optional[float] = None, seed: int = 0,
               timeout_s: float = 120.0, n_submitters: int = 1, results: Optional[list] = None) -> dict:
    """Submits the batches (at Poisson arrivals of the given offered load, or
    as fast as admission allows when rate is None) and collects them.

    n_submitters threads share the arrivals (batch i goes to thread
    i % n_submitters at its arrival time), as several filter threads each
    submit the batches they produce; each submit copies its batch into the
    engine's pinned staging in the submitting thread.

    Returns per-batch latency percentiles and maximum (ms), the slowest
    batch's submit / admission / completion times (ms after the first
    submit), the end-to-end rate (pairs/s from the first submit to the last
    completion) and the result count.  With a list in `results`, batch i's
    result pairs are stored in results[i].
    """
    n = len(batches)
    tickets: List[Optional[int]] = [None] * n
    ready = [threading.Event() for _ in range(n)]
    mean = float(np.mean([b[0].shape[0] for b in batches])) if n else 1.0
    rng = np.random.default_rng(seed)
    gaps = (rng.exponential(mean / rate_pairs_per_s, size=n) if rate_pairs_per_s else np.zeros(n))
    arrival = np.cumsum(gaps)
    errors: List[BaseException] = []
    t0 = time.perf_counter()

    def submitter(k):
        try:
            for i in range(k, n, n_submitters):
                cand, tn, td = batches[i]
                delay = t0 + arrival[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tickets[i] = S.ssj_stream_submit(ctx, coll, cand, tn, td)
                ready[i].set()
        except BaseException as e:  # surfaced by the caller
            errors.append(e)
            for ev in ready:
                ev.set()

    lat = np.zeros(n)
    t_sub = np.zeros(n)
    t_adm = np.zeros(n)
    t_done = np.zeros(n)
    if results is not None:
        results[:] = [None] * n
    n_result = 0
    ths = [threading.Thread(target=submitter, args=(k,), daemon=True) for k in range(max(1, n_submitters))]
    n_submitters = len(ths)
    for th in ths:
        th.start()
    deadline = time.perf_counter() + timeout_s
    for i in range(n):
        if not ready[i].wait(max(0.0, deadline - time.perf_counter())) or errors:
            break
        ts, ta, td = S.ssj_stream_times(ctx, tickets[i], wait=True)
        res = S.ssj_stream_collect(ctx, tickets[i])
        n_result += res.shape[0]
        if results is not None:
            results[i] = res
        t_sub[i], t_adm[i], t_done[i] = ts, ta, td
        lat[i] = (td - ts) / 1e6
    for th in ths:
        th.join(timeout=max(0.0, deadline - time.perf_counter()))
    if errors:
        raise errors[0]
    pairs = int(sum(b[0].shape[0] for b in batches))
    span = (t_done.max() - t_sub.min()) / 1e9 if n else 0.0
    slow = int(np.argmax(lat)) if n else 0
    base = t_sub.min() if n else 0.0
    return {
        "batches": n,
        "pairs": pairs,
        "mean_batch_pairs": round(mean, 1),
        "p50_ms": round(float(np.percentile(lat, 50)), 4) if n else None,
        "p99_ms": round(float(np.percentile(lat, 99)), 4) if n else None,
        "max_ms": round(float(lat.max()), 4) if n else None,
        "slowest": ({"batch": slow, "pairs": int(batches[slow][0].shape[0]),
                     "submit_ms": round((t_sub[slow] - base) / 1e6, 4),
                     "admit_ms": round((t_adm[slow] - base) / 1e6, 4),
                     "done_ms": round((t_done[slow] - base) / 1e6, 4)} if n else None),
        "pairs_per_s": round(pairs / span, 1) if span > 0 else None,
        "offered_pairs_per_s": rate_pairs_per_s,
        "results": n_result,
        "submit_threads": n_submitters,
    }
