"""Seeded synthetic token-set collections for the verification workloads.

This module only *draws inputs*: it holds none of the verification
arithmetic (no overlap, no threshold test).  It is shared by the oracle
tests, the GPU parity tests, the benchmark and the streaming driver, so both
sides of every comparison see byte-identical collections.

What the collections reproduce (paper Sec. 2.2, "Data layout"): every set
holds unique integer tokens; token ids ascend with global document frequency
(rarest token = id 0); the tokens of a set are sorted ascending; the sets of a
collection are sorted by size and, among equal sizes, lexicographically.  The
set id is the position after that sort.  The paper's seven real datasets
(Sec. 5.1, Table 3) are not available; these synthetic shapes stand in for
them (short sets, long sets, Zipf-like heavy-tailed sizes).

Generation recipe (deterministic for a given numpy bit generator):
  * sizes: uniform integers, or a lognormal whose *arithmetic* mean is m
    (mu = ln m - sigma^2/2) rounded to the nearest integer and clipped, or a
    classical Pareto-I draw floor(x_m * U^(-1/alpha)) clipped;
  * tokens: a bounded Zipf law P(k) ~ k^-s over ranks 1..U, sampled by
    inverse CDF on the cumulative weights; a set keeps the first `size`
    distinct ranks of its successive draws (repeats are skipped);
  * relabelling: ranks that occur are renumbered 0..D-1 by ascending
    document frequency, ties broken by ascending Zipf rank;
  * seeds: numpy SeedSequence([seed, config, purpose]).
"""
from __future__ import annotations

import dataclasses
import hashlib
import os
from typing import Optional, Tuple

import numpy as np

GEN_VERSION = 1

PURPOSE_SIZES = 0
PURPOSE_TOKENS = 1
PURPOSE_STREAM = 2


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic collection plus the thresholds it is joined at."""

    cfg: int
    name: str
    n_sets: int
    size_law: Tuple  # ("uniform", lo, hi) | ("lognormal", mean, sigma, lo, hi) | ("pareto", alpha, xm, hi)
    zipf_s: float
    universe: int
    thresholds: Tuple[Tuple[int, int], ...]  # rational t = t_num / t_den
    seed: int = 0


WORKLOADS = {
    1: Workload(1, "tiny", 2_000, ("uniform", 5, 15), 1.0, 5_000, ((4, 5),)),
    2: Workload(2, "offline", 100_000, ("lognormal", 12.0, 0.5, 2, 200), 1.0, 200_000,
                ((3, 5), (7, 10), (4, 5), (9, 10))),
    3: Workload(3, "longsets", 50_000, ("lognormal", 130.0, 0.8, 10, 2_000), 0.9, 1_000_000,
                ((7, 10),)),
    4: Workload(4, "heavytail", 500_000, ("pareto", 1.5, 3, 5_000), 1.2, 2_000_000, ((3, 4),)),
    5: Workload(5, "stream", 1_000_000, ("lognormal", 12.0, 0.5, 2, 200), 1.0, 1_000_000,
                ((3, 5), (4, 5), (9, 10))),
}


@dataclasses.dataclass
class Collection:
    """CSR collection: set i owns tokens[offsets[i]:offsets[i+1]]."""

    offsets: np.ndarray  # int64, n_sets + 1
    tokens: np.ndarray  # int32, nnz

    @property
    def n_sets(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_tokens(self) -> int:
        return int(self.tokens.shape[0])

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)

    def set(self, i: int) -> np.ndarray:
        return self.tokens[self.offsets[i]:self.offsets[i + 1]]

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.offsets, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.tokens, dtype=np.int32).tobytes())
        return h.hexdigest()


def _rng(seed: int, cfg: int, purpose: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([seed, cfg, purpose]))


def draw_sizes(law: Tuple, n: int, rng: np.random.Generator) -> np.ndarray:
    kind = law[0]
    if kind == "uniform":
        _, lo, hi = law
        return rng.integers(lo, hi + 1, size=n, dtype=np.int64)
    if kind == "lognormal":
        _, mean, sigma, lo, hi = law
        mu = np.log(mean) - sigma * sigma / 2.0
        x = np.rint(rng.lognormal(mu, sigma, size=n))
        return np.clip(x, lo, hi).astype(np.int64)
    if kind == "pareto":
        _, alpha, xm, hi = law
        u = 1.0 - rng.random(n)  # (0, 1]
        x = np.floor(xm * u ** (-1.0 / alpha))
        return np.clip(x, xm, hi).astype(np.int64)
    raise ValueError(f"unknown size law {law!r}")


def zipf_cdf(universe: int, s: float) -> np.ndarray:
    w = np.arange(1, universe + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    c /= c[-1]
    return c


def _distinct_first(set_idx: np.ndarray, pos: np.ndarray, tok: np.ndarray):
    """Keep, per set, the first draw of each distinct token.

    The inputs are ordered by draw position within each set, so a stable sort
    on the (set, token) key keeps the earliest draw of a token first.
    """
    key = (set_idx << 24) | tok
    order = np.argsort(key, kind="stable")
    key = key[order]
    keep = np.ones(key.shape[0], dtype=bool)
    keep[1:] = key[1:] != key[:-1]
    sel = order[keep]
    return set_idx[sel], pos[sel], tok[sel]


def draw_token_ranks(sizes: np.ndarray, universe: int, s: float,
                     rng: np.random.Generator) -> Tuple[np.ndarray, np.ndarray]:
    """Per set, the first sizes[i] distinct Zipf ranks of successive draws.

    Returns (set_idx, rank) sorted by set, then by draw order.
    """
    n = sizes.shape[0]
    if int(sizes.max(initial=0)) > universe:
        raise ValueError("a set is larger than the token universe")
    if universe >= (1 << 24) or n >= (1 << 27):
        raise ValueError("universe or set count too large for the packed sort keys")
    cdf = zipf_cdf(universe, s)
    set_idx = np.zeros(0, dtype=np.int64)
    pos = np.zeros(0, dtype=np.int64)
    tok = np.zeros(0, dtype=np.int64)
    next_pos = np.zeros(n, dtype=np.int64)
    have = np.zeros(n, dtype=np.int64)
    factor = 1.25
    while True:
        deficit = sizes - have
        need = np.nonzero(deficit > 0)[0]
        if need.size == 0:
            break
        m = np.ceil(deficit[need] * factor).astype(np.int64) + 2
        total = int(m.sum())
        new_set = np.repeat(need, m)
        start = np.repeat(np.cumsum(m) - m, m)
        new_pos = np.repeat(next_pos[need], m) + (np.arange(total, dtype=np.int64) - start)
        next_pos[need] += m
        u = rng.random(total)
        new_tok = np.searchsorted(cdf, u, side="right").astype(np.int64) + 1
        new_tok = np.minimum(new_tok, universe)
        set_idx, pos, tok = _distinct_first(
            np.concatenate([set_idx, new_set]), np.concatenate([pos, new_pos]),
            np.concatenate([tok, new_tok]))
        have = np.bincount(set_idx, minlength=n)
        factor *= 2.0
    # Per set, keep the sizes[i] earliest distinct draws.
    order = np.argsort((set_idx << 36) | pos, kind="stable")
    set_idx, tok = set_idx[order], tok[order]
    first = np.searchsorted(set_idx, np.arange(n))
    rank_in_set = np.arange(set_idx.shape[0]) - first[set_idx]
    keep = rank_in_set < sizes[set_idx]
    return set_idx[keep], tok[keep]


def relabel_by_frequency(rank: np.ndarray, universe: int) -> np.ndarray:
    """Map Zipf ranks to ids ordered by (document frequency, rank) ascending."""
    df = np.bincount(rank, minlength=universe + 1)
    occurring = np.nonzero(df)[0]
    order = np.lexsort((occurring, df[occurring]))
    new_id = np.full(universe + 1, -1, dtype=np.int64)
    new_id[occurring[order]] = np.arange(occurring.shape[0], dtype=np.int64)
    return new_id[rank]


def canonical_order(offsets: np.ndarray, tokens: np.ndarray) -> Collection:
    """Sort sets by size, then lexicographically among equal sizes."""
    sizes = np.diff(offsets)
    n = sizes.shape[0]
    perm_parts = []
    for L in np.unique(sizes):
        ids = np.nonzero(sizes == L)[0]
        if ids.shape[0] > 1:
            rows = tokens[(offsets[ids][:, None] + np.arange(L)[None, :])]
            keys = tuple(rows[:, c] for c in range(L - 1, -1, -1))
            ids = ids[np.lexsort(keys)]
        perm_parts.append(ids)
    perm = np.concatenate(perm_parts) if perm_parts else np.zeros(0, dtype=np.int64)
    new_sizes = sizes[perm]
    new_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(new_sizes, out=new_off[1:])
    nnz = int(new_off[-1])
    gather = np.repeat(offsets[:-1][perm] - new_off[:-1], new_sizes) + np.arange(nnz, dtype=np.int64)
    return Collection(new_off, np.ascontiguousarray(tokens[gather], dtype=np.int32))


def make_collection(n_sets: int, size_law: Tuple, zipf_s: float, universe: int,
                    seed: int = 0, cfg: int = 0) -> Collection:
    sizes = draw_sizes(size_law, n_sets, _rng(seed, cfg, PURPOSE_SIZES))
    set_idx, rank = draw_token_ranks(sizes, universe, zipf_s, _rng(seed, cfg, PURPOSE_TOKENS))
    ids = relabel_by_frequency(rank, universe)
    order = np.lexsort((ids, set_idx))
    ids = ids[order]
    offsets = np.zeros(n_sets + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    return canonical_order(offsets, ids.astype(np.int32))


def _cache_dir() -> Optional[str]:
    d = os.environ.get("SSJ_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "ssj_inputs")
    try:
        os.makedirs(d, exist_ok=True)
        return d
    except OSError:
        return None


def workload_collection(cfg: int, use_cache: bool = True) -> Collection:
    """The collection of one of the five workload configurations."""
    w = WORKLOADS[cfg]
    d = _cache_dir() if use_cache else None
    path = None
    if d is not None:
        path = os.path.join(d, f"cfg{cfg}_s{w.seed}_v{GEN_VERSION}_np{np.__version__}.npz")
        if os.path.exists(path):
            try:
                z = np.load(path, allow_pickle=False)
                return Collection(z["offsets"], z["tokens"])
            except Exception:
                pass
    c = make_collection(w.n_sets, w.size_law, w.zipf_s, w.universe, w.seed, w.cfg)
    if path is not None:
        tmp = path + f".tmp{os.getpid()}.npz"
        try:
            np.savez(tmp, offsets=c.offsets, tokens=c.tokens)
            os.replace(tmp, path)
        except OSError:
            pass
    return c


def random_collection(rng: np.random.Generator, n_sets: int, max_size: int, universe: int,
                      zipf_s: float = 1.0, min_size: int = 1) -> Collection:
    """Small random collection for property tests (same contract as the workloads)."""
    sizes = rng.integers(min_size, max_size + 1, size=n_sets).astype(np.int64)
    set_idx, rank = draw_token_ranks(sizes, universe, zipf_s, rng)
    ids = relabel_by_frequency(rank, universe)
    order = np.lexsort((ids, set_idx))
    offsets = np.zeros(n_sets + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    return canonical_order(offsets, ids[order].astype(np.int32))


def near_duplicate_collection(rng: np.random.Generator, n_base: int, copies: int, max_size: int,
                              universe: int, change_frac: float = 0.1, min_size: int = 2,
                              zipf_s: float = 1.0) -> Collection:
    """Collection rich in similar pairs: every base set appears `copies` times,
    each copy with about change_frac of its tokens swapped for fresh ones and
    a few tokens dropped or added.  Used to exercise passing pairs, which the
    random workloads rarely contain."""
    sizes = rng.integers(min_size, max_size + 1, size=n_base).astype(np.int64)
    set_idx, rank = draw_token_ranks(sizes, universe, zipf_s, rng)
    bases = np.split(rank, np.cumsum(sizes)[:-1])
    out = []
    for b in bases:
        for _ in range(copies):
            x = set(int(v) for v in b)
            k = int(rng.binomial(len(b), change_frac))
            for v in rng.choice(b, size=k, replace=False):
                x.discard(int(v))
            add = k + int(rng.integers(-1, 2))
            while add > 0:
                v = int(rng.integers(1, universe + 1))
                if v not in x:
                    x.add(v)
                    add -= 1
            if not x:
                x.add(int(b[0]))
            out.append(np.array(sorted(x), dtype=np.int64))
    sz = np.array([len(v) for v in out], dtype=np.int64)
    offsets = np.zeros(len(out) + 1, dtype=np.int64)
    np.cumsum(sz, out=offsets[1:])
    flat = np.concatenate(out)
    ids = relabel_by_frequency(flat, universe)
    sidx = np.repeat(np.arange(len(out)), sz)
    order = np.lexsort((ids, sidx))
    return canonical_order(offsets, ids[order].astype(np.int32))


def device_bytes(c: Collection) -> int:
    """Device bytes of a collection in the verification library's layout
    (each set padded to a multiple of 4 int32 tokens, a 32-byte record per
    set): what an upload takes from a context's HBM budget."""
    padded = int(((np.diff(c.offsets) + 3) // 4 * 4).sum())
    return 4 * max(padded, 4) + 32 * max(c.n_sets, 1)


def collection_from_sets(sets) -> Collection:
    """CSR from an explicit list of token lists (each sorted and unique)."""
    sizes = np.array([len(s) for s in sets], dtype=np.int64)
    offsets = np.zeros(len(sets) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    flat = np.array([t for s in sets for t in s], dtype=np.int32)
    return Collection(offsets, flat)


def stream_schedule(n_batches: int, seed: int = 0, lo: float = 1e3, hi: float = 1e6,
                    thresholds=((3, 5), (4, 5), (9, 10))):
    """Batch sizes (log-uniform in [lo, hi]) and per-batch thresholds for streaming."""
    rng = _rng(seed, 5, PURPOSE_STREAM)
    sizes = np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_batches))).astype(np.int64)
    tidx = rng.integers(0, len(thresholds), size=n_batches)
    return sizes, [thresholds[i] for i in tidx], rng
