"""Host logic of the serving replay (paper_1812_09141_amd/serving.py) against
a fake stream API on the CPU: every batch is submitted exactly once, no
earlier than its arrival time, spread over the submitting threads, and the
results and latencies are collected per ticket."""
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1812_09141_amd import serving  # noqa: E402


class FakeStream:
    """ssj_stream_submit / ssj_stream_times / ssj_stream_collect with fixed
    1 ms service and one result pair per 1,000 candidates."""

    def __init__(self):
        self.mu = threading.Lock()
        self.next = 1
        self.req = {}
        self.threads = {}

    def ssj_stream_submit(self, ctx, coll, cand, tn, td):
        with self.mu:
            t = self.next
            self.next += 1
            now = time.monotonic_ns()
            self.req[t] = (cand.shape[0], tn, td, now)
            self.threads.setdefault(id(threading.current_thread()), []).append(t)
        return t

    def ssj_stream_times(self, ctx, ticket, wait=True):
        n, _, _, ts = self.req[ticket]
        return ts, ts + 100_000, ts + 1_000_000

    def ssj_stream_collect(self, ctx, ticket):
        n = self.req[ticket][0]
        return np.zeros((n // 1000, 2), np.int32)


def _batches(rng, k):
    return [(np.zeros((int(n), 2), np.int32), 3, 5) for n in rng.integers(1000, 20000, k)]


def test_saturated_every_batch_once_over_threads():
    rng = np.random.default_rng(0)
    b = _batches(rng, 60)
    for subs in (1, 3, 4):
        S = FakeStream()
        out = serving.run_stream(S, None, None, b, None, n_submitters=subs)
        assert out["batches"] == 60 and out["submit_threads"] == subs
        assert out["pairs"] == sum(x[0].shape[0] for x in b)
        assert out["results"] == sum(x[0].shape[0] // 1000 for x in b)
        assert sorted(n for n, _, _, _ in S.req.values()) == sorted(x[0].shape[0] for x in b)
        assert len(S.threads) == subs
        assert abs(out["p50_ms"] - 1.0) < 1e-9 and abs(out["p99_ms"] - 1.0) < 1e-9


def test_offered_load_respects_arrivals():
    rng = np.random.default_rng(1)
    b = _batches(rng, 40)
    mean = np.mean([x[0].shape[0] for x in b])
    rate = mean / 0.002  # one batch every 2 ms on average
    S = FakeStream()
    t0 = time.monotonic_ns()
    out = serving.run_stream(S, None, None, b, rate, seed=7, n_submitters=3)
    gaps = np.random.default_rng(7).exponential(mean / rate, size=len(b))
    arrival_ns = np.cumsum(gaps) * 1e9
    # each batch i went out no earlier than its arrival (tickets follow submit order, so match by size)
    sub = sorted(S.req.values(), key=lambda v: v[3])
    assert len(sub) == 40
    total_span = (sub[-1][3] - t0)
    assert total_span >= 0.9 * arrival_ns[-1]
    assert out["offered_pairs_per_s"] == rate and out["results"] == sum(x[0].shape[0] // 1000 for x in b)
