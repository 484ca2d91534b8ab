"""ctypes binding of the CPU candidate generators: the AllPairs prefix + length
filter, optionally with PPJoin's positional filter.

The filters are the paper's filtering phase (Sec. 2.2 "Filters", Sec. 3.1
AllPairs and PPJoin); they produce the candidate pairs that verification
consumes.  They are input generation: they decide no pair, they only drop pairs
that cannot pass.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssj_allpairs.so")
SRC_PATH = os.path.join(_HERE, "csrc", "allpairs.cpp")

_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-O3", "-march=x86-64-v2", "-std=c++17", "-shared", "-fPIC", "-pthread",
           "-o", LIB_PATH + ".tmp", SRC_PATH]
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
    lib.ssjf_build.argtypes = [p, i64, p, i64, i64, ctypes.POINTER(p)]
    lib.ssjf_build.restype = ctypes.c_int
    lib.ssjf_build2.argtypes = [p, i64, p, i64, i64, ctypes.c_int, ctypes.POINTER(p)]
    lib.ssjf_build2.restype = ctypes.c_int
    lib.ssjf_free.argtypes = [p]
    lib.ssjf_free.restype = None
    lib.ssjf_probe.argtypes = [p, i64, i64, p, i64, ctypes.POINTER(i64)]
    lib.ssjf_probe.restype = i64
    lib.ssjf_count.argtypes = [p, ctypes.c_int, p]
    lib.ssjf_count.restype = i64
    lib.ssjf_fill.argtypes = [p, ctypes.c_int, p, p]
    lib.ssjf_fill.restype = ctypes.c_int
    _lib = lib
    return lib


def default_threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(n, 16))


class PrefixIndex:
    """Prefix inverted index over one collection at one threshold
    (positional=True adds PPJoin's positional filter)."""

    def __init__(self, offsets: np.ndarray, tokens: np.ndarray, t_num: int, t_den: int,
                 positional: bool = False):
        lib = _load()
        self._off = np.ascontiguousarray(offsets, dtype=np.int64)
        self._tok = np.ascontiguousarray(tokens, dtype=np.int32)
        self.n_sets = int(self._off.shape[0] - 1)
        h = ctypes.c_void_p()
        rc = lib.ssjf_build2(self._off.ctypes.data, self.n_sets, self._tok.ctypes.data,
                             int(t_num), int(t_den), int(bool(positional)), ctypes.byref(h))
        if rc != 0:
            raise ValueError("ssjf_build rejected the collection or threshold")
        self._h = h
        self.t = (int(t_num), int(t_den))

    def close(self):
        if getattr(self, "_h", None):
            _load().ssjf_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def probe(self, r_begin: int, r_end: int, out: np.ndarray) -> Tuple[int, int]:
        """Fill out (int32 [cap, 2]) with candidates of probes from r_begin on.

        Returns (pairs written, next probe).  Releases the GIL while it runs.
        """
        nxt = ctypes.c_int64()
        n = _load().ssjf_probe(self._h, int(r_begin), int(r_end), out.ctypes.data,
                               int(out.shape[0]), ctypes.byref(nxt))
        if n < 0:
            raise ValueError("ssjf_probe: bad arguments")
        return int(n), int(nxt.value)

    def all_candidates(self, n_threads: Optional[int] = None) -> np.ndarray:
        """Every candidate (r, s), grouped by probe r in ascending order."""
        lib = _load()
        nt = n_threads or default_threads()
        counts = np.zeros(self.n_sets, dtype=np.int64)
        total = lib.ssjf_count(self._h, nt, counts.ctypes.data)
        starts = np.zeros(self.n_sets, dtype=np.int64)
        if self.n_sets > 1:
            np.cumsum(counts[:-1], out=starts[1:])
        out = np.empty((int(total), 2), dtype=np.int32)
        if total > 0:
            lib.ssjf_fill(self._h, nt, starts.ctypes.data, out.ctypes.data)
        return out


def candidates(offsets: np.ndarray, tokens: np.ndarray, t_num: int, t_den: int,
               n_threads: Optional[int] = None, positional: bool = False) -> np.ndarray:
    ix = PrefixIndex(offsets, tokens, t_num, t_den, positional=positional)
    try:
        return ix.all_candidates(n_threads)
    finally:
        ix.close()


def _cache_path(cfg: int, t_num: int, t_den: int, positional: bool = False) -> Optional[str]:
    from . import synth
    d = synth._cache_dir()
    if d is None:
        return None
    kind = "ppj" if positional else "cand"
    return os.path.join(d, f"{kind}_cfg{cfg}_t{t_num}_{t_den}_v{synth.GEN_VERSION}_np{np.__version__}.npy")


def workload_candidates(cfg: int, t_num: int, t_den: int, use_cache: bool = True,
                        positional: bool = False) -> np.ndarray:
    """Candidates of a workload collection at one threshold (cached on disk);
    positional=True adds PPJoin's positional filter."""
    from . import synth
    path = _cache_path(cfg, t_num, t_den, positional) if use_cache else None
    if path and os.path.exists(path):
        try:
            return np.load(path, allow_pickle=False)
        except Exception:
            pass
    c = synth.workload_collection(cfg, use_cache=use_cache)
    cand = candidates(c.offsets, c.tokens, t_num, t_den, positional=positional)
    if path:
        tmp = path + f".tmp{os.getpid()}.npy"
        try:
            np.save(tmp, cand)
            os.replace(tmp, path)
        except OSError:
            pass
    return cand
