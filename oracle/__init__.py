"""Verification oracle -- TEST INFRASTRUCTURE ONLY.

Plain CPU references for the verification phase of an exact set-similarity
join (paper Sec. 3, Definition 1; the similarity functions of Table 1).  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import this package.
It shares no code with the GPU library and imports nothing from it.

  * ``verify`` / ``select`` / ``merge_trace``: ctypes wrappers of the plain C
    oracle (``verify_ref.c``): full-merge overlap + the exact integer test of
    Jaccard, Cosine, Dice or Overlap (``sim``), and the early-terminating
    Jaccard merge replayed for token accounting.
  * ``select_rs``: the same for an R-S join (Definition 1 with two
    collections): r ids index R, s ids index S.
  * ``brute``: pure-Python all-pairs join and per-pair verification with
    ``frozenset`` and ``fractions.Fraction`` (tiny inputs only).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssj_oracle.so")
SRC_PATH = os.path.join(_HERE, "verify_ref.c")

_lib = None

# similarity functions of Table 1 (the threshold of "overlap" is a count)
SIMS = {"jaccard": 0, "cosine": 1, "dice": 2, "overlap": 3}


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-shared", "-fPIC", "-o", LIB_PATH + ".tmp",
           SRC_PATH]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    p = ctypes.c_void_p
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    lib.ssjref_verify_sim.argtypes = [p, i64, p, p, i64, ci, i64, i64, p, p, ci]
    lib.ssjref_verify_sim.restype = ctypes.c_int
    lib.ssjref_select_sim.argtypes = [p, i64, p, p, i64, ci, i64, i64, p, p, ci]
    lib.ssjref_select_sim.restype = i64
    lib.ssjref_merge_trace.argtypes = [p, i64, p, p, i64, i64, i64, p, p, p, ctypes.c_int]
    lib.ssjref_merge_trace.restype = ctypes.c_int
    lib.ssjref_max_threads.argtypes = []
    lib.ssjref_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


class OracleError(ValueError):
    pass


def max_threads() -> int:
    return int(_load().ssjref_max_threads())


def _prep(offsets, tokens, pairs):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    tok = np.ascontiguousarray(tokens, dtype=np.int32)
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    if tok.size == 0:
        tok = np.zeros(1, dtype=np.int32)
    return off, tok, pr


def _sim_code(sim: str) -> int:
    if sim not in SIMS:
        raise OracleError(f"unknown similarity function {sim!r}")
    return SIMS[sim]


def verify(offsets, tokens, pairs, t_num: int, t_den: int, n_threads: int = 1,
           with_overlap: bool = False, sim: str = "jaccard"):
    """pass flags (uint8 per pair) and optionally the exact overlaps."""
    off, tok, pr = _prep(offsets, tokens, pairs)
    n = pr.shape[0]
    passed = np.zeros(max(n, 1), dtype=np.uint8)
    ov = np.zeros(max(n, 1), dtype=np.int32) if with_overlap else None
    rc = _load().ssjref_verify_sim(off.ctypes.data, off.shape[0] - 1, tok.ctypes.data,
                                   pr.ctypes.data, n, _sim_code(sim), int(t_num), int(t_den),
                                   passed.ctypes.data, ov.ctypes.data if ov is not None else None,
                                   int(n_threads))
    if rc != 0:
        raise OracleError("invalid threshold, id out of range or empty set")
    if with_overlap:
        return passed[:n], ov[:n]
    return passed[:n]


def select(offsets, tokens, pairs, t_num: int, t_den: int, n_threads: int = 1,
           sim: str = "jaccard") -> np.ndarray:
    """The passing pairs (int32 [k, 2]) in input order."""
    off, tok, pr = _prep(offsets, tokens, pairs)
    n = pr.shape[0]
    scratch = np.zeros(max(n, 1), dtype=np.uint8)
    out = np.zeros((max(n, 1), 2), dtype=np.int32)
    k = _load().ssjref_select_sim(off.ctypes.data, off.shape[0] - 1, tok.ctypes.data,
                                  pr.ctypes.data, n, _sim_code(sim), int(t_num), int(t_den),
                                  scratch.ctypes.data, out.ctypes.data, int(n_threads))
    if k < 0:
        raise OracleError("invalid threshold, id out of range or empty set")
    return out[:k].copy()


def select_rs(offsets_r, tokens_r, offsets_s, tokens_s, pairs, t_num: int, t_den: int,
              n_threads: int = 1, sim: str = "jaccard") -> np.ndarray:
    """The passing pairs of an R-S join (r in R, s in S), in input order.

    The two collections are laid out as one (the sets of S after those of R,
    so S's set s becomes set |R| + s), and each pair is verified by select;
    the ids returned are the caller's."""
    off_r = np.asarray(offsets_r, dtype=np.int64)
    off_s = np.asarray(offsets_s, dtype=np.int64)
    n_r, n_s = off_r.shape[0] - 1, off_s.shape[0] - 1
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    if pr.shape[0] and (pr[:, 0].min() < 0 or pr[:, 0].max() >= n_r or pr[:, 1].min() < 0
                        or pr[:, 1].max() >= n_s):
        raise OracleError("id out of range")
    off = np.concatenate([off_r, off_r[-1] + off_s[1:]])
    tok = np.concatenate([np.asarray(tokens_r, dtype=np.int32), np.asarray(tokens_s, dtype=np.int32)])
    shifted = pr.copy()
    shifted[:, 1] += n_r
    keep = select(off, tok, shifted, t_num, t_den, n_threads=n_threads, sim=sim)
    keep[:, 1] -= n_r
    return keep


def merge_trace(offsets, tokens, pairs, t_num: int, t_den: int, n_threads: int = 1):
    """(c_r, c_s, decided) of the early-terminating merge, per pair."""
    off, tok, pr = _prep(offsets, tokens, pairs)
    n = pr.shape[0]
    cr = np.zeros(max(n, 1), dtype=np.int32)
    cs = np.zeros(max(n, 1), dtype=np.int32)
    dec = np.zeros(max(n, 1), dtype=np.uint8)
    rc = _load().ssjref_merge_trace(off.ctypes.data, off.shape[0] - 1, tok.ctypes.data,
                                    pr.ctypes.data, n, int(t_num), int(t_den), cr.ctypes.data,
                                    cs.ctypes.data, dec.ctypes.data, int(n_threads))
    if rc != 0:
        raise OracleError("invalid threshold, id out of range or empty set")
    return cr[:n], cs[:n], dec[:n]


def sort_pairs(pairs) -> np.ndarray:
    """Canonical multiset order: ascending (r << 32 | s) as unsigned keys."""
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    key = (pr[:, 0].astype(np.int64) << 32) | (pr[:, 1].astype(np.int64) & 0xFFFFFFFF)
    return pr[np.argsort(key, kind="stable")]


def result_digest(pairs) -> str:
    import hashlib
    return hashlib.sha256(sort_pairs(pairs).tobytes()).hexdigest()
