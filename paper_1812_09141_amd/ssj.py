"""Thin ctypes binding of libssj (include/ssj.h).

Argument marshalling only: every step of verification runs in the HIP
library.  The functions carry the C names.  PyTorch is imported first so that
the library binds to the HIP runtime torch already loaded (one runtime per
process); torch supplies device buffers and streams for ``ssj_verify_device``.
There is no CPU fallback: if libssj.so is missing or cannot load, this module
raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np
import torch  # noqa: F401  (shared HIP runtime, device memory, streams)

_PKG = os.path.dirname(os.path.abspath(__file__))
# SSJ_LIB may name another build of the same library (e.g. for comparisons)
LIB_PATH = os.environ.get("SSJ_LIB") or os.path.join(_PKG, "libssj.so")

SSJ_OK = 0
SSJ_PENDING = 1
SSJ_CACHED = 2
SSJ_EINVAL = -1
SSJ_ENOMEM = -2
SSJ_ETRUNC = -3
SSJ_EAGAIN = -4
SSJ_EDEVICE = -5
SSJ_ENOTFOUND = -6

# similarity functions (paper Table 1); Overlap's threshold is a count
SSJ_SIM_JACCARD = 0
SSJ_SIM_COSINE = 1
SSJ_SIM_DICE = 2
SSJ_SIM_OVERLAP = 3
SIMS = {"jaccard": SSJ_SIM_JACCARD, "cosine": SSJ_SIM_COSINE, "dice": SSJ_SIM_DICE,
        "overlap": SSJ_SIM_OVERLAP}

SSJ_N_CLASSES = 5
SSJ_CLASS_BOUNDS = (32, 128, 512, 2048, 0x7FFFFFFF)
SSJ_MAX_BATCH = 16
SSJ_NOALLOC_MAX_PAIRS = 1 << 20

EXPORTED = (
    "ssj_init", "ssj_shutdown", "ssj_last_error", "ssj_upload_collection",
    "ssj_free_collection", "ssj_verify", "ssj_verify_device", "ssj_stream_submit",
    "ssj_stream_poll", "ssj_stream_times", "ssj_get_plan", "ssj_set_plan",
    "ssj_collection_info", "ssj_timing_enable", "ssj_timing_read", "ssj_verify_batch_device",
    "ssj_autotune", "ssj_verify_sim", "ssj_verify_device_sim", "ssj_stream_submit_sim",
    "ssj_verify_rs", "ssj_verify_rs_device", "ssj_verify_groups", "ssj_verify_groups_device",
    "ssj_verify_groups_batch_device",
    "ssj_candidates_device", "ssj_join_device", "ssj_join", "ssj_stream_pause",
    "ssj_verify_device_noalloc", "ssj_set_tune_cache", "ssj_stream_stats",
)

_NAMES = {
    SSJ_OK: "SSJ_OK", SSJ_PENDING: "SSJ_PENDING", SSJ_CACHED: "SSJ_CACHED", SSJ_EINVAL: "SSJ_EINVAL",
    SSJ_ENOMEM: "SSJ_ENOMEM", SSJ_ETRUNC: "SSJ_ETRUNC", SSJ_EAGAIN: "SSJ_EAGAIN",
    SSJ_EDEVICE: "SSJ_EDEVICE", SSJ_ENOTFOUND: "SSJ_ENOTFOUND",
}


class SsjError(RuntimeError):
    def __init__(self, code: int, msg: str, n: Optional[int] = None):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code
        self.n = n


class ssj_pair(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("s", ctypes.c_int32)]


class ssj_opts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hbm_budget", ctypes.c_uint64),
                ("n_slots", ctypes.c_int), ("queue_depth", ctypes.c_int)]


class ssj_plan(ctypes.Structure):
    _fields_ = [("inline_lanes", ctypes.c_int), ("hard_lanes", ctypes.c_int),
                ("defer_from", ctypes.c_int), ("lanes", ctypes.c_int * SSJ_N_CLASSES),
                ("use_graph", ctypes.c_int), ("spill_iters", ctypes.c_int),
                ("spill_lanes", ctypes.c_int), ("wg_per_cu", ctypes.c_int), ("staged", ctypes.c_int)]

    def as_dict(self):
        return {"inline_lanes": self.inline_lanes, "hard_lanes": self.hard_lanes,
                "defer_from": self.defer_from, "lanes": list(self.lanes),
                "use_graph": self.use_graph, "spill_iters": self.spill_iters,
                "spill_lanes": self.spill_lanes, "wg_per_cu": self.wg_per_cu, "staged": self.staged}


class ssj_request(ctypes.Structure):
    _fields_ = [("d_cand", ctypes.c_void_p), ("n_cand", ctypes.c_int64),
                ("t_num", ctypes.c_int64), ("t_den", ctypes.c_int64),
                ("d_out", ctypes.c_void_p), ("out_cap", ctypes.c_int64),
                ("d_count", ctypes.c_void_p), ("sim", ctypes.c_int32)]


class ssj_group_request(ctypes.Structure):
    _fields_ = [("d_groups", ctypes.c_void_p), ("n_groups", ctypes.c_int64),
                ("d_cand", ctypes.c_void_p), ("n_cand", ctypes.c_int64),
                ("t_num", ctypes.c_int64), ("t_den", ctypes.c_int64),
                ("d_out", ctypes.c_void_p), ("out_cap", ctypes.c_int64),
                ("d_count", ctypes.c_void_p), ("sim", ctypes.c_int32)]


class ssj_stream_stats_t(ctypes.Structure):
    _fields_ = [("slot_grows", ctypes.c_uint64), ("slot_grow_ms", ctypes.c_double),
                ("result_grows", ctypes.c_uint64), ("result_grow_ms", ctypes.c_double),
                ("longest_pass_ms", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libssj.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    p, i64, u64, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "ssj_init": ([P(ssj_opts), P(p)], c_int),
        "ssj_shutdown": ([p], c_int),
        "ssj_last_error": ([p], ctypes.c_char_p),
        "ssj_upload_collection": ([p, p, i64, p, i64, P(p)], c_int),
        "ssj_free_collection": ([p, p], c_int),
        "ssj_verify": ([p, p, p, i64, i64, i64, p, i64, P(i64)], c_int),
        "ssj_verify_device": ([p, p, p, i64, i64, i64, p, i64, p, p], c_int),
        "ssj_verify_device_noalloc": ([p, p, p, i64, i64, i64, p, i64, p, p], c_int),
        "ssj_stream_submit": ([p, p, p, i64, i64, i64, c_int, P(u64)], c_int),
        "ssj_stream_poll": ([p, u64, c_int, p, i64, P(i64)], c_int),
        "ssj_stream_times": ([p, u64, c_int, P(u64), P(u64), P(u64)], c_int),
        "ssj_stream_stats": ([p, P(ssj_stream_stats_t), c_int], c_int),
        "ssj_stream_pause": ([p, c_int], c_int),
        "ssj_get_plan": ([p, P(ssj_plan)], c_int),
        "ssj_set_plan": ([p, P(ssj_plan)], c_int),
        "ssj_collection_info": ([p, P(i64), P(i64), P(i64)], c_int),
        "ssj_timing_enable": ([p, c_int], c_int),
        "ssj_timing_read": ([p, c_int, P(ctypes.c_double), P(ctypes.c_double), P(i64)], c_int),
        "ssj_verify_batch_device": ([p, p, P(ssj_request), c_int, p], c_int),
        "ssj_autotune": ([p, p, p, i64, i64, i64, c_int, P(ssj_plan), P(ctypes.c_double)], c_int),
        "ssj_set_tune_cache": ([p, ctypes.c_char_p], c_int),
        "ssj_verify_sim": ([p, p, p, i64, c_int, i64, i64, p, i64, P(i64)], c_int),
        "ssj_verify_device_sim": ([p, p, p, i64, c_int, i64, i64, p, i64, p, p], c_int),
        "ssj_stream_submit_sim": ([p, p, p, i64, c_int, i64, i64, c_int, P(u64)], c_int),
        "ssj_verify_rs": ([p, p, p, p, i64, c_int, i64, i64, p, i64, P(i64)], c_int),
        "ssj_verify_rs_device": ([p, p, p, p, i64, c_int, i64, i64, p, i64, p, p], c_int),
        "ssj_verify_groups": ([p, p, p, p, i64, p, i64, c_int, i64, i64, p, i64, P(i64)], c_int),
        "ssj_verify_groups_device": ([p, p, p, p, i64, p, i64, c_int, i64, i64, p, i64, p, p], c_int),
        "ssj_verify_groups_batch_device": ([p, p, p, P(ssj_group_request), c_int, p], c_int),
        "ssj_candidates_device": ([p, p, i64, i64, c_int, p, i64, p, p], c_int),
        "ssj_join_device": ([p, p, i64, i64, c_int, p, i64, p, p], c_int),
        "ssj_join": ([p, p, i64, i64, c_int, p, i64, P(i64)], c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _err(ctx, code: int, n: Optional[int] = None):
    msg = load_library().ssj_last_error(ctx).decode(errors="replace")
    raise SsjError(code, msg, n)


def _pairs(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32).reshape(-1, 2)


# --- C-named entry points -------------------------------------------------

def ssj_init(device: int = 0, hbm_budget: int = 0, n_slots: int = 0, queue_depth: int = 0):
    lib = load_library()
    o = ssj_opts(device, hbm_budget, n_slots, queue_depth)
    h = ctypes.c_void_p()
    rc = lib.ssj_init(ctypes.byref(o), ctypes.byref(h))
    if rc != SSJ_OK:
        _err(None, rc)
    return h


def ssj_shutdown(ctx) -> None:
    load_library().ssj_shutdown(ctx)


def ssj_last_error(ctx=None) -> str:
    return load_library().ssj_last_error(ctx).decode(errors="replace")


def ssj_upload_collection(ctx, offsets, tokens):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    tok = np.ascontiguousarray(tokens, dtype=np.int32)
    h = ctypes.c_void_p()
    rc = load_library().ssj_upload_collection(ctx, off.ctypes.data, off.shape[0] - 1,
                                              tok.ctypes.data if tok.size else None,
                                              tok.shape[0], ctypes.byref(h))
    if rc != SSJ_OK:
        _err(ctx, rc)
    return h


def ssj_free_collection(ctx, coll) -> None:
    rc = load_library().ssj_free_collection(ctx, coll)
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_collection_info(coll) -> Tuple[int, int, int]:
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    rc = load_library().ssj_collection_info(coll, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    if rc != SSJ_OK:
        _err(None, rc)
    return a.value, b.value, c.value


def ssj_verify(ctx, coll, cand, t_num: int, t_den: int, out_cap: Optional[int] = None) -> np.ndarray:
    """Passing pairs (int32 [k, 2]); raises SsjError (code SSJ_ETRUNC carries .n)."""
    c = _pairs(cand)
    n = c.shape[0]
    cap = n if out_cap is None else int(out_cap)
    out = np.zeros((max(cap, 1), 2), dtype=np.int32)
    out_n = ctypes.c_int64()
    rc = load_library().ssj_verify(ctx, coll, c.ctypes.data if n else None, n, int(t_num), int(t_den),
                                   out.ctypes.data, cap, ctypes.byref(out_n))
    if rc != SSJ_OK:
        _err(ctx, rc, out_n.value)
    return out[:out_n.value].copy()


def sim_code(sim) -> int:
    """SSJ_SIM_* code of a similarity function given by code or name."""
    if isinstance(sim, str):
        if sim not in SIMS:
            raise ValueError(f"unknown similarity function {sim!r}")
        return SIMS[sim]
    return int(sim)


def ssj_verify_sim(ctx, coll, cand, sim, t_num: int, t_den: int,
                   out_cap: Optional[int] = None) -> np.ndarray:
    """ssj_verify with a similarity function of Table 1 (code or name)."""
    c = _pairs(cand)
    n = c.shape[0]
    cap = n if out_cap is None else int(out_cap)
    out = np.zeros((max(cap, 1), 2), dtype=np.int32)
    out_n = ctypes.c_int64()
    rc = load_library().ssj_verify_sim(ctx, coll, c.ctypes.data if n else None, n, sim_code(sim),
                                       int(t_num), int(t_den), out.ctypes.data, cap,
                                       ctypes.byref(out_n))
    if rc != SSJ_OK:
        _err(ctx, rc, out_n.value)
    return out[:out_n.value].copy()


def ssj_verify_device_sim(ctx, coll, d_cand: "torch.Tensor", sim, t_num: int, t_den: int,
                          d_out: "torch.Tensor", d_count: "torch.Tensor", stream=None) -> None:
    """ssj_verify_device with a similarity function of Table 1 (code or name)."""
    assert d_cand.is_cuda and d_cand.dtype == torch.int32 and d_cand.is_contiguous()
    if d_out is not None:
        assert d_out.is_cuda and d_out.dtype == torch.int32 and d_out.is_contiguous()
    assert d_count.is_cuda and d_count.dtype == torch.int64 and d_count.numel() >= 1
    n = d_cand.numel() // 2
    cap = d_out.numel() // 2 if d_out is not None else 0
    st = stream if stream is not None else torch.cuda.current_stream(d_cand.device)
    rc = load_library().ssj_verify_device_sim(ctx, coll, d_cand.data_ptr() if n else None, n,
                                              sim_code(sim), int(t_num), int(t_den),
                                              d_out.data_ptr() if cap else None, cap,
                                              d_count.data_ptr(), ctypes.c_void_p(st.cuda_stream))
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_verify_rs(ctx, coll_r, coll_s, cand, sim, t_num: int, t_den: int,
                  out_cap: Optional[int] = None) -> np.ndarray:
    """R-S join verification: r ids index coll_r, s ids coll_s (host buffers)."""
    c = _pairs(cand)
    n = c.shape[0]
    cap = n if out_cap is None else int(out_cap)
    out = np.zeros((max(cap, 1), 2), dtype=np.int32)
    out_n = ctypes.c_int64()
    rc = load_library().ssj_verify_rs(ctx, coll_r, coll_s, c.ctypes.data if n else None, n,
                                      sim_code(sim), int(t_num), int(t_den), out.ctypes.data, cap,
                                      ctypes.byref(out_n))
    if rc != SSJ_OK:
        _err(ctx, rc, out_n.value)
    return out[:out_n.value].copy()


def ssj_verify_rs_device(ctx, coll_r, coll_s, d_cand: "torch.Tensor", sim, t_num: int, t_den: int,
                         d_out: "torch.Tensor", d_count: "torch.Tensor", stream=None) -> None:
    """ssj_verify_device_sim for an R-S join."""
    assert d_cand.is_cuda and d_cand.dtype == torch.int32 and d_cand.is_contiguous()
    if d_out is not None:
        assert d_out.is_cuda and d_out.dtype == torch.int32 and d_out.is_contiguous()
    assert d_count.is_cuda and d_count.dtype == torch.int64 and d_count.numel() >= 1
    n = d_cand.numel() // 2
    cap = d_out.numel() // 2 if d_out is not None else 0
    st = stream if stream is not None else torch.cuda.current_stream(d_cand.device)
    rc = load_library().ssj_verify_rs_device(ctx, coll_r, coll_s, d_cand.data_ptr() if n else None,
                                             n, sim_code(sim), int(t_num), int(t_den),
                                             d_out.data_ptr() if cap else None, cap,
                                             d_count.data_ptr(), ctypes.c_void_p(st.cuda_stream))
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_verify_groups(ctx, coll_r, coll_s, groups, cand, sim, t_num: int, t_den: int,
                      out_cap: Optional[int] = None) -> np.ndarray:
    """Grouped candidates: groups (n_groups, 2) int32 rows (probe id, exclusive end into
    cand), cand the s ids (host buffers)."""
    gr = np.ascontiguousarray(groups, dtype=np.int32).reshape(-1, 2)
    c = np.ascontiguousarray(cand, dtype=np.int32).reshape(-1)
    n = c.shape[0]
    cap = n if out_cap is None else int(out_cap)
    out = np.zeros((max(cap, 1), 2), dtype=np.int32)
    out_n = ctypes.c_int64()
    rc = load_library().ssj_verify_groups(ctx, coll_r, coll_s, gr.ctypes.data if gr.shape[0] else None,
                                          gr.shape[0], c.ctypes.data if n else None, n, sim_code(sim),
                                          int(t_num), int(t_den), out.ctypes.data, cap,
                                          ctypes.byref(out_n))
    if rc != SSJ_OK:
        _err(ctx, rc, out_n.value)
    return out[:out_n.value].copy()


def ssj_verify_groups_device(ctx, coll_r, coll_s, d_groups: "torch.Tensor", d_cand: "torch.Tensor",
                             sim, t_num: int, t_den: int, d_out: "torch.Tensor",
                             d_count: "torch.Tensor", stream=None) -> None:
    """Grouped candidates on the device: d_groups (n_groups, 2) int32, d_cand int32 s ids."""
    assert d_groups.is_cuda and d_groups.dtype == torch.int32 and d_groups.is_contiguous()
    assert d_cand.is_cuda and d_cand.dtype == torch.int32 and d_cand.is_contiguous()
    if d_out is not None:
        assert d_out.is_cuda and d_out.dtype == torch.int32 and d_out.is_contiguous()
    assert d_count.is_cuda and d_count.dtype == torch.int64 and d_count.numel() >= 1
    ng = d_groups.numel() // 2
    n = d_cand.numel()
    cap = d_out.numel() // 2 if d_out is not None else 0
    st = stream if stream is not None else torch.cuda.current_stream(d_cand.device)
    rc = load_library().ssj_verify_groups_device(
        ctx, coll_r, coll_s, d_groups.data_ptr() if ng else None, ng, d_cand.data_ptr() if n else None,
        n, sim_code(sim), int(t_num), int(t_den), d_out.data_ptr() if cap else None, cap,
        d_count.data_ptr(), ctypes.c_void_p(st.cuda_stream))
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_verify_groups_batch_device(ctx, coll_r, coll_s, requests, stream=None) -> None:
    """requests: list of (d_groups, d_cand, t_num, t_den, d_out, d_count[, sim]) with
    d_groups (n_groups, 2) int32 and d_cand int32 s ids on the device; one launch."""
    n = len(requests)
    arr = (ssj_group_request * max(n, 1))()
    dev = None
    for i, req in enumerate(requests):
        d_groups, d_cand, tn, td, d_out, d_count = req[:6]
        sim = sim_code(req[6]) if len(req) > 6 else SSJ_SIM_JACCARD
        assert d_groups.is_cuda and d_groups.dtype == torch.int32 and d_groups.is_contiguous()
        assert d_cand.is_cuda and d_cand.dtype == torch.int32 and d_cand.is_contiguous()
        if d_out is not None:
            assert d_out.is_cuda and d_out.dtype == torch.int32 and d_out.is_contiguous()
        assert d_count.is_cuda and d_count.dtype == torch.int64
        ng = d_groups.numel() // 2
        nc = d_cand.numel()
        cap = d_out.numel() // 2 if d_out is not None else 0
        arr[i] = ssj_group_request(d_groups.data_ptr() if ng else None, ng, d_cand.data_ptr() if nc else None, nc,
                                   int(tn), int(td), d_out.data_ptr() if cap else None, cap, d_count.data_ptr(), sim)
        dev = d_cand.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    rc = load_library().ssj_verify_groups_batch_device(ctx, coll_r, coll_s, arr, n, ctypes.c_void_p(st.cuda_stream))
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_candidates_device(ctx, coll, t_num: int, t_den: int, positional: bool,
                          d_out: "torch.Tensor", d_count: "torch.Tensor", stream=None) -> None:
    """GPU prefix-filter candidates (with PPJoin's positional filter if positional)."""
    if d_out is not None:
        assert d_out.is_cuda and d_out.dtype == torch.int32 and d_out.is_contiguous()
    assert d_count.is_cuda and d_count.dtype == torch.int64 and d_count.numel() >= 1
    cap = d_out.numel() // 2 if d_out is not None else 0
    st = stream if stream is not None else torch.cuda.current_stream(d_count.device)
    rc = load_library().ssj_candidates_device(ctx, coll, int(t_num), int(t_den), int(bool(positional)),
                                              d_out.data_ptr() if cap else None, cap, d_count.data_ptr(),
                                              ctypes.c_void_p(st.cuda_stream))
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_join_device(ctx, coll, t_num: int, t_den: int, positional: bool, d_out: "torch.Tensor",
                    d_count: "torch.Tensor", stream=None) -> None:
    """The whole self-join on the GPU (filter, then verification)."""
    if d_out is not None:
        assert d_out.is_cuda and d_out.dtype == torch.int32 and d_out.is_contiguous()
    assert d_count.is_cuda and d_count.dtype == torch.int64 and d_count.numel() >= 1
    cap = d_out.numel() // 2 if d_out is not None else 0
    st = stream if stream is not None else torch.cuda.current_stream(d_count.device)
    rc = load_library().ssj_join_device(ctx, coll, int(t_num), int(t_den), int(bool(positional)),
                                        d_out.data_ptr() if cap else None, cap, d_count.data_ptr(),
                                        ctypes.c_void_p(st.cuda_stream))
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_join(ctx, coll, t_num: int, t_den: int, positional: bool = True,
             out_cap: Optional[int] = None) -> np.ndarray:
    """The whole self-join on the GPU, results in host memory (grows the buffer once
    when out_cap is too small)."""
    cap = 1 << 16 if out_cap is None else int(out_cap)
    for _ in range(2):
        out = np.zeros((max(cap, 1), 2), dtype=np.int32)
        out_n = ctypes.c_int64()
        rc = load_library().ssj_join(ctx, coll, int(t_num), int(t_den), int(bool(positional)),
                                     out.ctypes.data, cap, ctypes.byref(out_n))
        if rc == SSJ_ETRUNC and out_cap is None:
            cap = int(out_n.value)
            continue
        if rc != SSJ_OK:
            _err(ctx, rc, out_n.value)
        return out[:out_n.value].copy()
    _err(ctx, SSJ_ETRUNC, out_n.value)


def groups_of(pairs) -> tuple:
    """Grouped form (groups, s ids) of flat pairs: one group per run of equal r."""
    c = _pairs(pairs)
    if c.shape[0] == 0:
        return np.zeros((0, 2), np.int32), np.zeros(0, np.int32)
    starts = np.flatnonzero(np.r_[True, c[1:, 0] != c[:-1, 0]])
    ends = np.r_[starts[1:], c.shape[0]]
    return np.stack([c[starts, 0], ends], axis=1).astype(np.int32), c[:, 1].copy()


def ssj_stream_submit_sim(ctx, coll, cand, sim, t_num: int, t_den: int,
                          nonblocking: bool = False) -> int:
    """ssj_stream_submit with a similarity function of Table 1 (code or name)."""
    c = _pairs(cand)
    t = ctypes.c_uint64()
    rc = load_library().ssj_stream_submit_sim(ctx, coll, c.ctypes.data if c.shape[0] else None,
                                              c.shape[0], sim_code(sim), int(t_num), int(t_den),
                                              int(bool(nonblocking)), ctypes.byref(t))
    if rc != SSJ_OK:
        _err(ctx, rc)
    return t.value


def ssj_verify_device(ctx, coll, d_cand: "torch.Tensor", t_num: int, t_den: int,
                      d_out: "torch.Tensor", d_count: "torch.Tensor", stream=None) -> None:
    """Enqueues verification of device pairs on a torch stream (no sync).

    d_out=None selects the output-count mode: only *d_count is produced."""
    assert d_cand.is_cuda and d_cand.dtype == torch.int32 and d_cand.is_contiguous()
    if d_out is not None:
        assert d_out.is_cuda and d_out.dtype == torch.int32 and d_out.is_contiguous()
    assert d_count.is_cuda and d_count.dtype == torch.int64 and d_count.numel() >= 1
    n = d_cand.numel() // 2
    cap = d_out.numel() // 2 if d_out is not None else 0
    st = stream if stream is not None else torch.cuda.current_stream(d_cand.device)
    rc = load_library().ssj_verify_device(ctx, coll, d_cand.data_ptr() if n else None, n,
                                          int(t_num), int(t_den), d_out.data_ptr() if cap else None,
                                          cap, d_count.data_ptr(), ctypes.c_void_p(st.cuda_stream))
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_verify_device_noalloc(ctx, coll, d_cand: "torch.Tensor", t_num: int, t_den: int,
                              d_out: "torch.Tensor", d_count: "torch.Tensor", stream=None) -> None:
    """ssj_verify_device through the allocation-free entry point (at most
    SSJ_NOALLOC_MAX_PAIRS pairs; the library's fixed per-device scratch)."""
    assert d_cand.is_cuda and d_cand.dtype == torch.int32 and d_cand.is_contiguous()
    if d_out is not None:
        assert d_out.is_cuda and d_out.dtype == torch.int32 and d_out.is_contiguous()
    assert d_count.is_cuda and d_count.dtype == torch.int64 and d_count.numel() >= 1
    n = d_cand.numel() // 2
    cap = d_out.numel() // 2 if d_out is not None else 0
    st = stream if stream is not None else torch.cuda.current_stream(d_cand.device)
    rc = load_library().ssj_verify_device_noalloc(ctx, coll, d_cand.data_ptr() if n else None, n,
                                                  int(t_num), int(t_den), d_out.data_ptr() if cap else None,
                                                  cap, d_count.data_ptr(), ctypes.c_void_p(st.cuda_stream))
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_stream_submit(ctx, coll, cand, t_num: int, t_den: int, nonblocking: bool = False) -> int:
    c = _pairs(cand)
    t = ctypes.c_uint64()
    rc = load_library().ssj_stream_submit(ctx, coll, c.ctypes.data if c.shape[0] else None,
                                          c.shape[0], int(t_num), int(t_den), int(bool(nonblocking)),
                                          ctypes.byref(t))
    if rc != SSJ_OK:
        _err(ctx, rc)
    return t.value


def ssj_stream_poll(ctx, ticket: int, wait: bool = True, out_cap: int = 0):
    """Returns the passing pairs, or None while pending (wait=False)."""
    out = np.zeros((max(out_cap, 1), 2), dtype=np.int32)
    out_n = ctypes.c_int64()
    rc = load_library().ssj_stream_poll(ctx, ticket, int(bool(wait)), out.ctypes.data, out_cap,
                                        ctypes.byref(out_n))
    if rc == SSJ_PENDING:
        return None
    if rc != SSJ_OK:
        _err(ctx, rc, out_n.value)
    return out[:out_n.value].copy()


def ssj_stream_pause(ctx, pause: bool = True) -> None:
    """Holds (True) or resumes (False) admission of queued stream requests."""
    rc = load_library().ssj_stream_pause(ctx, int(bool(pause)))
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_stream_times(ctx, ticket: int, wait: bool = False):
    """(t_submit, t_admit, t_done) in ns of CLOCK_MONOTONIC, or None while pending."""
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    rc = load_library().ssj_stream_times(ctx, ticket, int(bool(wait)), ctypes.byref(a),
                                         ctypes.byref(b), ctypes.byref(c))
    if rc == SSJ_PENDING:
        return None
    if rc != SSJ_OK:
        _err(ctx, rc)
    return a.value, b.value, c.value


def ssj_stream_stats(ctx, reset: bool = False) -> dict:
    """The streaming engine's buffer regrowths and longest engine-loop pass."""
    st = ssj_stream_stats_t()
    rc = load_library().ssj_stream_stats(ctx, ctypes.byref(st), int(bool(reset)))
    if rc != SSJ_OK:
        _err(ctx, rc)
    return {"slot_grows": st.slot_grows, "slot_grow_ms": round(st.slot_grow_ms, 4),
            "result_grows": st.result_grows, "result_grow_ms": round(st.result_grow_ms, 4),
            "longest_pass_ms": round(st.longest_pass_ms, 4)}


def ssj_get_plan(ctx) -> ssj_plan:
    p = ssj_plan()
    rc = load_library().ssj_get_plan(ctx, ctypes.byref(p))
    if rc != SSJ_OK:
        _err(ctx, rc)
    return p


def make_plan(inline_lanes: int = 1, defer_from: int = SSJ_N_CLASSES, lanes=(4, 16, 64, 256, 256),
              use_graph: int = 0, hard_lanes: int = 0, spill_iters: int = 0,
              spill_lanes: int = 16, wg_per_cu: int = 0, staged: int = 0) -> ssj_plan:
    p = ssj_plan()
    p.inline_lanes = int(inline_lanes)
    p.hard_lanes = int(hard_lanes)
    p.defer_from = int(defer_from)
    for q in range(SSJ_N_CLASSES):
        p.lanes[q] = int(lanes[q])
    p.use_graph = int(use_graph)
    p.spill_iters = int(spill_iters)
    p.spill_lanes = int(spill_lanes)
    p.wg_per_cu = int(wg_per_cu)
    p.staged = int(staged)
    return p


def ssj_set_plan(ctx, plan: ssj_plan) -> None:
    rc = load_library().ssj_set_plan(ctx, ctypes.byref(plan))
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_verify_batch_device(ctx, coll, requests, stream=None) -> None:
    """requests: list of (d_cand, t_num, t_den, d_out, d_count[, sim]) torch tensors/ints
    (sim, a code or name of a Table 1 function, defaults to Jaccard)."""
    n = len(requests)
    arr = (ssj_request * max(n, 1))()
    dev = None
    for i, req in enumerate(requests):
        d_cand, tn, td, d_out, d_count = req[:5]
        sim = sim_code(req[5]) if len(req) > 5 else SSJ_SIM_JACCARD
        assert d_cand.is_cuda and d_cand.dtype == torch.int32 and d_cand.is_contiguous()
        if d_out is not None:
            assert d_out.is_cuda and d_out.dtype == torch.int32 and d_out.is_contiguous()
        assert d_count.is_cuda and d_count.dtype == torch.int64
        nc = d_cand.numel() // 2
        cap = d_out.numel() // 2 if d_out is not None else 0
        arr[i] = ssj_request(d_cand.data_ptr() if nc else None, nc, int(tn), int(td),
                             d_out.data_ptr() if cap else None, cap, d_count.data_ptr(), sim)
        dev = d_cand.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    rc = load_library().ssj_verify_batch_device(ctx, coll, arr, n, ctypes.c_void_p(st.cuda_stream))
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_autotune(ctx, coll, d_cand: "torch.Tensor", t_num: int, t_den: int, apply: bool = True,
                 with_status: bool = False):
    """Best plan for the given device candidates and its kernel time (ms);
    with_status also returns whether it came from the tuning cache."""
    p = ssj_plan()
    ms = ctypes.c_double()
    n = d_cand.numel() // 2
    rc = load_library().ssj_autotune(ctx, coll, d_cand.data_ptr(), n, int(t_num), int(t_den),
                                     int(bool(apply)), ctypes.byref(p), ctypes.byref(ms))
    if rc not in (SSJ_OK, SSJ_CACHED):
        _err(ctx, rc)
    if with_status:
        return p, ms.value, rc == SSJ_CACHED
    return p, ms.value


def ssj_set_tune_cache(ctx, path) -> None:
    """Tuning cache file of ssj_autotune (None turns it off)."""
    rc = load_library().ssj_set_tune_cache(ctx, os.fsencode(path) if path else None)
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_timing_enable(ctx, period: int = 1) -> None:
    """Time every period-th launch (0 = off)."""
    rc = load_library().ssj_timing_enable(ctx, int(period))
    if rc != SSJ_OK:
        _err(ctx, rc)


def ssj_timing_read(ctx, reset: bool = False):
    """(in-order ms, rest-of-launch ms, timed launches) summed since the last reset."""
    a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    rc = load_library().ssj_timing_read(ctx, int(bool(reset)), ctypes.byref(a), ctypes.byref(b),
                                        ctypes.byref(n))
    if rc != SSJ_OK:
        _err(ctx, rc)
    return a.value, b.value, n.value


def ssj_stream_collect(ctx, ticket: int):
    """poll(wait) with a retry at the size the library reports."""
    try:
        return ssj_stream_poll(ctx, ticket, True, 0)
    except SsjError as e:
        if e.code != SSJ_ETRUNC:
            raise
        return ssj_stream_poll(ctx, ticket, True, int(e.n))
