"""Python binding of the gfx950 AHPP library (include/ahpp.h).

Argument marshalling only: every step of a query runs in the HIP library
``libahpp.so``.  Torch is used for device buffers and streams.  If the
library has not been built this module raises at import of the library; there
is no fallback path.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libahpp.so")

OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_NOT_CONVERGED = 0, -1, -2, -3, -4

EXPORTED = ("ahpp_graph_load", "ahpp_graph_info", "ahpp_graph_key", "ahpp_graph_free", "ahpp_query", "ahpp_query_noalloc",
            "ahpp_query_schedule",
            "ahpp_query_batch", "ahpp_topk",
            "ahpp_server_create", "ahpp_server_free", "ahpp_server_submit", "ahpp_server_step",
            "ahpp_server_results", "ahpp_server_info", "ahpp_server_set_solo", "ahpp_graph_tune", "ahpp_query_mc", "ahpp_profile_enable",
            "ahpp_profile_read", "ahpp_last_error")

# Kernel kinds of ahpp_profile_read.
PROF_SINGLE_BACK, PROF_SINGLE_FWD, PROF_BATCH_BACK, PROF_BATCH_FWD, PROF_BATCH_HOT = 0, 1, 2, 3, 4


class AhppError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class GraphDesc(ctypes.Structure):
    _fields_ = [("n_u", ctypes.c_int64), ("n_v", ctypes.c_int64), ("n_attr", ctypes.c_int64),
                ("n_edges", ctypes.c_int64), ("edge_u", ctypes.c_void_p), ("edge_v", ctypes.c_void_p),
                ("edge_w", ctypes.c_void_p), ("n_assoc", ctypes.c_int64), ("assoc_u", ctypes.c_void_p),
                ("assoc_a", ctypes.c_void_p), ("assoc_w", ctypes.c_void_p), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("lam", ctypes.c_double), ("lambda_iters", ctypes.c_int32),
                ("device", ctypes.c_int32), ("cache_dir", ctypes.c_char_p)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("n_u", ctypes.c_int64), ("n_v", ctypes.c_int64), ("n_attr", ctypes.c_int64),
                ("n_edges", ctypes.c_int64), ("n_assoc", ctypes.c_int64), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("lam", ctypes.c_double), ("lambda_iters", ctypes.c_int32),
                ("device", ctypes.c_int32), ("dangling_u", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("load_ms", ctypes.c_double), ("lambda_ms", ctypes.c_double), ("key", ctypes.c_uint64 * 2),
                ("lambda_cached", ctypes.c_int32), ("hot_rows", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("sync_switch_iter", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n_push", ctypes.c_int64), ("max_residual", ctypes.c_double),
                ("sum_residual", ctypes.c_double), ("ms", ctypes.c_float), ("pad", ctypes.c_float)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f not in ("reserved", "pad")}


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libahpp.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() or "
                          "python paper_2512_11606_amd/build.py")
    # torch and this library both link libamdhip64.so.7, and the process keeps
    # whichever copy is loaded first.  torch's device memory and streams must
    # live in the runtime the library's kernels use, and torch cannot start
    # its own on a runtime another build loaded, so torch goes first.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.ahpp_graph_load.restype = ctypes.c_int
    lib.ahpp_graph_load.argtypes = [ctypes.POINTER(GraphDesc), ctypes.POINTER(ctypes.c_void_p)]
    lib.ahpp_graph_info.restype = ctypes.c_int
    lib.ahpp_graph_info.argtypes = [P, ctypes.POINTER(GraphInfo)]
    lib.ahpp_graph_key.restype = ctypes.c_int
    lib.ahpp_graph_key.argtypes = [ctypes.POINTER(GraphDesc), ctypes.POINTER(ctypes.c_uint64)]
    lib.ahpp_graph_free.restype = None
    lib.ahpp_graph_free.argtypes = [P]
    lib.ahpp_query.restype = ctypes.c_int
    lib.ahpp_query.argtypes = [P, i32, dbl, i32, P, P, i32, P, P, P, P, P]
    lib.ahpp_query_noalloc.restype = ctypes.c_int
    lib.ahpp_query_noalloc.argtypes = [P, i32, dbl, i32, P, P, i32, P, P, P, P, P]
    lib.ahpp_query_batch.restype = ctypes.c_int
    lib.ahpp_query_batch.argtypes = [P, i32, P, P, i32, P, i32, P, P, P, P, P]
    lib.ahpp_topk.restype = ctypes.c_int
    lib.ahpp_topk.argtypes = [P, P, i32, i32, P, P, P, P]
    lib.ahpp_server_create.restype = ctypes.c_int
    lib.ahpp_server_create.argtypes = [P, i64, i32, i32, i32, i32, ctypes.POINTER(ctypes.c_void_p)]
    lib.ahpp_server_free.restype = None
    lib.ahpp_server_free.argtypes = [P]
    lib.ahpp_server_submit.restype = ctypes.c_int
    lib.ahpp_server_submit.argtypes = [P, i64, i32, dbl]
    lib.ahpp_server_step.restype = ctypes.c_int
    lib.ahpp_server_step.argtypes = [P, i32, P, P]
    lib.ahpp_server_results.restype = ctypes.c_int
    lib.ahpp_server_results.argtypes = [P, i32, P, P, P, P, P, P, P, P]
    lib.ahpp_server_info.restype = ctypes.c_int
    lib.ahpp_server_info.argtypes = [P, P, P, P, P]
    lib.ahpp_server_set_solo.restype = ctypes.c_int
    lib.ahpp_server_set_solo.argtypes = [P, i32]
    lib.ahpp_query_schedule.restype = ctypes.c_int
    lib.ahpp_query_schedule.argtypes = [P, i32, dbl, i32, i32, P, P, i32, P, P, P, P, P]
    lib.ahpp_query_mc.restype = ctypes.c_int
    lib.ahpp_query_mc.argtypes = [P, i32, i64, ctypes.c_uint64, P, i32, P, P, P, P, P]
    lib.ahpp_graph_tune.restype = ctypes.c_int
    lib.ahpp_graph_tune.argtypes = [P, i32, P, P]
    lib.ahpp_profile_enable.restype = ctypes.c_int
    lib.ahpp_profile_enable.argtypes = [P, i32]
    lib.ahpp_profile_read.restype = ctypes.c_int
    lib.ahpp_profile_read.argtypes = [P, i32, P, P, P, P]
    lib.ahpp_last_error.restype = ctypes.c_char_p
    lib.ahpp_last_error.argtypes = []
    _lib = lib
    return lib


def _check(status: int, allow_not_converged: bool = False) -> int:
    if status == OK or (allow_not_converged and status == ERR_NOT_CONVERGED):
        return status
    raise AhppError(status, load_library().ahpp_last_error().decode())


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _as_i32(x, what: str) -> np.ndarray:
    """Contiguous int32 copy of an id array; ids of a wider integer type must
    fit, since a silent wrap could land on a valid id."""
    a = np.asarray(x)
    if a.dtype != np.int32:
        if a.size and not np.issubdtype(a.dtype, np.integer):
            raise ValueError(f"{what}: ids must be integers, got {a.dtype}")
        if a.size and (int(a.min()) < np.iinfo(np.int32).min or int(a.max()) > np.iinfo(np.int32).max):
            raise ValueError(f"{what}: ids outside the int32 range")
        a = a.astype(np.int32)
    return np.ascontiguousarray(a)


def _dev_ptr(t) -> Optional[int]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device: int, stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class QueryResult:
    pi: object                # torch float32 [n_u] (or [n_q, n_u]) on the device, or None
    resid: object             # torch float32 [n_u] or None
    topk_idx: object          # torch int32 [k] (or [n_q, k]) or None
    topk_val: object
    topk_n: object
    stats: list               # list of dicts (one per query)
    status: int


class Graph:
    """Handle of a graph loaded on one device (owns its device memory)."""

    def __init__(self, handle: ctypes.c_void_p, device: int):
        self._h = handle
        self.device = device
        self.info = ahpp_graph_info(self)

    @property
    def n_u(self) -> int:
        return int(self.info["n_u"])

    @property
    def lam(self) -> float:
        return float(self.info["lam"])

    def free(self):
        if self._h:
            load_library().ahpp_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _graph_desc(n_u: int, n_v: int, n_attr: int, edge_u, edge_v, edge_w, assoc_u, assoc_a, assoc_w,
                alpha: float, beta: float, lam: float, lambda_iters: int, device: int, cache_dir: Optional[str]):
    """A GraphDesc and the arrays it points at (which must outlive it)."""
    eu, ev = _as_i32(edge_u, "edge_u"), _as_i32(edge_v, "edge_v")
    ew = None if edge_w is None else np.ascontiguousarray(edge_w, dtype=np.float32)
    au, aa = _as_i32(assoc_u, "assoc_u"), _as_i32(assoc_a, "assoc_a")
    aw = None if assoc_w is None else np.ascontiguousarray(assoc_w, dtype=np.float32)
    if eu.shape != ev.shape or (ew is not None and ew.shape != eu.shape):
        raise ValueError("edge arrays differ in length")
    if au.shape != aa.shape or (aw is not None and aw.shape != au.shape):
        raise ValueError("association arrays differ in length")
    d = GraphDesc(int(n_u), int(n_v), int(n_attr), int(eu.size), _np_ptr(eu), _np_ptr(ev), _np_ptr(ew),
                  int(au.size), _np_ptr(au), _np_ptr(aa), _np_ptr(aw), float(alpha), float(beta), float(lam),
                  int(lambda_iters), int(device), None if not cache_dir else os.fsencode(cache_dir))
    return d, (eu, ev, ew, au, aa, aw)


def ahpp_graph_load(n_u: int, n_v: int, n_attr: int, edge_u, edge_v, edge_w, assoc_u, assoc_a, assoc_w,
                    alpha: float = 0.15, beta: float = 0.35, lam: float = 0.0, lambda_iters: int = 0,
                    device: int = 0, cache_dir: Optional[str] = None) -> Graph:
    """Loads COO lists (host arrays) onto `device`; see ahpp_graph_load in ahpp.h."""
    d, keep = _graph_desc(n_u, n_v, n_attr, edge_u, edge_v, edge_w, assoc_u, assoc_a, assoc_w, alpha, beta, lam,
                          lambda_iters, device, cache_dir)
    h = ctypes.c_void_p()
    _check(load_library().ahpp_graph_load(ctypes.byref(d), ctypes.byref(h)))
    del keep
    return Graph(h, int(device))


def load_graph(g, alpha: float = 0.15, beta: float = 0.35, lam: float = 0.0, lambda_iters: int = 0,
               device: int = 0, cache_dir: Optional[str] = None) -> Graph:
    """ahpp_graph_load for an object with the fields of synth.AttributedBipartiteGraph."""
    return ahpp_graph_load(g.n_u, g.n_v, g.n_attr, g.edge_u, g.edge_v, g.edge_w, g.assoc_u, g.assoc_a, g.assoc_w,
                           alpha, beta, lam, lambda_iters, device, cache_dir)


def ahpp_graph_key(g, alpha: float = 0.15, beta: float = 0.35, lam: float = 0.0, lambda_iters: int = 0) -> tuple:
    """Host-side key of a graph's inputs (ahpp_graph_key in ahpp.h), as two ints."""
    d, keep = _graph_desc(g.n_u, g.n_v, g.n_attr, g.edge_u, g.edge_v, g.edge_w, g.assoc_u, g.assoc_a, g.assoc_w,
                          alpha, beta, lam, lambda_iters, 0, None)
    key = (ctypes.c_uint64 * 2)()
    _check(load_library().ahpp_graph_key(ctypes.byref(d), key))
    del keep
    return int(key[0]), int(key[1])


def ahpp_graph_info(g: Graph) -> dict:
    info = GraphInfo()
    _check(load_library().ahpp_graph_info(g._h, ctypes.byref(info)))
    out = {f: getattr(info, f) for f, _ in info._fields_ if f != "reserved"}
    out["key"] = (int(info.key[0]), int(info.key[1]))
    return out


def ahpp_query(g: Graph, source: int, eps: float, k: int = 0, max_iters: int = 0, want_pi: bool = True,
               want_resid: bool = False, want_stats: bool = True, stream=None,
               allow_not_converged: bool = False) -> QueryResult:
    """One eps-approximate query; outputs are torch tensors on the graph's device."""
    import torch
    dev = torch.device("cuda", g.device)
    pi = torch.empty(g.n_u, dtype=torch.float32, device=dev) if want_pi else None
    resid = torch.empty(g.n_u, dtype=torch.float32, device=dev) if want_resid else None
    ti = torch.empty(max(k, 1), dtype=torch.int32, device=dev) if k > 0 else None
    tv = torch.empty(max(k, 1), dtype=torch.float32, device=dev) if k > 0 else None
    tn = torch.empty(1, dtype=torch.int32, device=dev) if k > 0 else None
    st = Stats()
    status = _check(load_library().ahpp_query(g._h, int(source), float(eps), int(max_iters), _dev_ptr(pi),
                                              _dev_ptr(resid), int(k), _dev_ptr(ti), _dev_ptr(tv), _dev_ptr(tn),
                                              ctypes.byref(st) if want_stats else None, _stream(g.device, stream)),
                    allow_not_converged)
    return QueryResult(pi, resid, ti, tv, tn, [st.as_dict()] if want_stats else [], status)


def ahpp_query_noalloc(g: Graph, source: int, eps: float, k: int = 0, max_iters: int = 0, want_pi: bool = True,
                       want_resid: bool = False, want_stats: bool = True, stream=None,
                       allow_not_converged: bool = False) -> QueryResult:
    """ahpp_query whose per-query buffers live in the library's fixed device
    scratch (no device allocation inside the call; see ahpp.h).  The output
    tensors are allocated here, by the caller side."""
    import torch
    dev = torch.device("cuda", g.device)
    pi = torch.empty(g.n_u, dtype=torch.float32, device=dev) if want_pi else None
    resid = torch.empty(g.n_u, dtype=torch.float32, device=dev) if want_resid else None
    ti = torch.empty(max(k, 1), dtype=torch.int32, device=dev) if k > 0 else None
    tv = torch.empty(max(k, 1), dtype=torch.float32, device=dev) if k > 0 else None
    tn = torch.empty(1, dtype=torch.int32, device=dev) if k > 0 else None
    st = Stats()
    status = _check(load_library().ahpp_query_noalloc(g._h, int(source), float(eps), int(max_iters), _dev_ptr(pi),
                                                      _dev_ptr(resid), int(k), _dev_ptr(ti), _dev_ptr(tv),
                                                      _dev_ptr(tn), ctypes.byref(st) if want_stats else None,
                                                      _stream(g.device, stream)),
                    allow_not_converged)
    return QueryResult(pi, resid, ti, tv, tn, [st.as_dict()] if want_stats else [], status)


SCHEDULE_ASRP, SCHEDULE_APP, SCHEDULE_APP_S, SCHEDULE_APP_E = 0, 1, 2, 3


def ahpp_query_schedule(g: Graph, source: int, eps: float, schedule: int, k: int = 0, max_iters: int = 0,
                        want_pi: bool = True, want_resid: bool = False, stream=None,
                        allow_not_converged: bool = False) -> QueryResult:
    """One query under an Exp-2 push schedule (0 ASRP, 1 APP, 2 APP(S), 3 APP(E))."""
    import torch
    dev = torch.device("cuda", g.device)
    pi = torch.empty(g.n_u, dtype=torch.float32, device=dev) if want_pi else None
    resid = torch.empty(g.n_u, dtype=torch.float32, device=dev) if want_resid else None
    ti = torch.empty(max(k, 1), dtype=torch.int32, device=dev) if k > 0 else None
    tv = torch.empty(max(k, 1), dtype=torch.float32, device=dev) if k > 0 else None
    tn = torch.empty(1, dtype=torch.int32, device=dev) if k > 0 else None
    st = Stats()
    status = _check(load_library().ahpp_query_schedule(g._h, int(source), float(eps), int(schedule), int(max_iters),
                                                       _dev_ptr(pi), _dev_ptr(resid), int(k), _dev_ptr(ti),
                                                       _dev_ptr(tv), _dev_ptr(tn), ctypes.byref(st),
                                                       _stream(g.device, stream)),
                    allow_not_converged)
    return QueryResult(pi, resid, ti, tv, tn, [st.as_dict()], status)


def ahpp_query_batch(g: Graph, sources: Sequence[int], eps, k: int = 0, max_iters: int = 0, want_pi: bool = True,
                     want_stats: bool = True, stream=None, allow_not_converged: bool = False) -> QueryResult:
    """n_q queries answered together; row q of every output belongs to query q."""
    import torch
    src = _as_i32(sources, "sources")
    n_q = int(src.size)
    e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (n_q,)))
    dev = torch.device("cuda", g.device)
    pi = torch.empty((n_q, g.n_u), dtype=torch.float32, device=dev) if want_pi else None
    ti = torch.empty((n_q, max(k, 1)), dtype=torch.int32, device=dev) if k > 0 else None
    tv = torch.empty((n_q, max(k, 1)), dtype=torch.float32, device=dev) if k > 0 else None
    tn = torch.empty(n_q, dtype=torch.int32, device=dev) if k > 0 else None
    st = (Stats * max(n_q, 1))()
    status = _check(load_library().ahpp_query_batch(g._h, n_q, _np_ptr(src), _np_ptr(e), int(max_iters),
                                                    _dev_ptr(pi), int(k), _dev_ptr(ti), _dev_ptr(tv), _dev_ptr(tn),
                                                    ctypes.cast(st, ctypes.c_void_p) if want_stats else None,
                                                    _stream(g.device, stream)), allow_not_converged)
    return QueryResult(pi, None, ti, tv, tn, [s.as_dict() for s in st[:n_q]] if want_stats else [], status)


def ahpp_topk(g: Graph, pi, k: int, exclude: int = -1, stream=None):
    """Top-k of a device score vector (torch float32 [n_u]): (idx, val, n) tensors."""
    import torch
    if (pi.dtype != torch.float32 or not pi.is_cuda or pi.device.index != g.device or pi.numel() != g.n_u
            or not pi.is_contiguous()):
        raise ValueError("pi must be a contiguous float32 tensor of length n_u on the graph's device")
    ti = torch.empty(max(k, 1), dtype=torch.int32, device=pi.device)
    tv = torch.empty(max(k, 1), dtype=torch.float32, device=pi.device)
    tn = torch.empty(1, dtype=torch.int32, device=pi.device)
    _check(load_library().ahpp_topk(g._h, _dev_ptr(pi), int(k), int(exclude), _dev_ptr(ti), _dev_ptr(tv),
                                    _dev_ptr(tn), _stream(g.device, stream)))
    return ti, tv, tn


def ahpp_profile_enable(g: Graph, on: bool = True) -> None:
    """Starts (clearing totals) or stops HIP-event timing of the gather kernels."""
    _check(load_library().ahpp_profile_enable(g._h, 1 if on else 0))


class McStats(ctypes.Structure):
    _fields_ = [("walks", ctypes.c_int64), ("lost", ctypes.c_int64), ("truncated", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("ms", ctypes.c_float), ("pad", ctypes.c_float)]


def ahpp_query_mc(g: Graph, source: int, n_walks: int, seed: int = 0, k: int = 0, want_pi: bool = True,
                  stream=None) -> dict:
    """Monte Carlo estimate of one AHPP row from n_walks walks (see ahpp.h):
    dict with pi, topk_idx, topk_val, topk_n (torch tensors on the graph's
    device, or None) and stats."""
    import torch
    dev = torch.device("cuda", g.device)
    pi = torch.empty(g.n_u, dtype=torch.float32, device=dev) if want_pi else None
    ti = torch.empty(max(k, 1), dtype=torch.int32, device=dev) if k > 0 else None
    tv = torch.empty(max(k, 1), dtype=torch.float32, device=dev) if k > 0 else None
    tn = torch.empty(1, dtype=torch.int32, device=dev) if k > 0 else None
    st = McStats()
    _check(load_library().ahpp_query_mc(g._h, int(source), int(n_walks), ctypes.c_uint64(int(seed) & (2**64 - 1)),
                                        _dev_ptr(pi), int(k), _dev_ptr(ti), _dev_ptr(tv), _dev_ptr(tn),
                                        ctypes.byref(st), _stream(g.device, stream)))
    return {"pi": pi, "topk_idx": ti, "topk_val": tv, "topk_n": tn,
            "stats": {f: getattr(st, f) for f, _ in st._fields_ if f != "pad"}}


class TuneInfo(ctypes.Structure):
    _fields_ = [("tiles_in_flight", ctypes.c_int32), ("workgroup_multiplier", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("reserved", ctypes.c_int32), ("ms_per_tile_round", ctypes.c_double),
                ("default_ms_per_tile_round", ctypes.c_double)]


def ahpp_graph_tune(g: Graph, max_tiles: int = 0, stream=None) -> dict:
    """Times candidate batch schedules and keeps the fastest (see ahpp.h)."""
    info = TuneInfo()
    _check(load_library().ahpp_graph_tune(g._h, int(max_tiles), ctypes.byref(info), _stream(g.device, stream)))
    return {f: getattr(info, f) for f, _ in info._fields_ if f != "reserved"}


def ahpp_profile_read(g: Graph, kind: int) -> dict:
    """Launch count, summed elapsed ms, gathered-model bytes and compulsory
    bytes of one kernel kind (see ahpp.h)."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    by = ctypes.c_double(0.0)
    comp = ctypes.c_double(0.0)
    _check(load_library().ahpp_profile_read(g._h, int(kind), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                            ctypes.byref(comp)))
    return {"launches": int(n.value), "ms": float(ms.value), "bytes": float(by.value),
            "compulsory": float(comp.value)}


class Server:
    """Continuous-batching server over a loaded graph (ahpp_server_* in ahpp.h)."""

    def __init__(self, g: Graph, k: int, max_device_bytes: int = 0, max_iters: int = 0, keep_pi: bool = False,
                 max_slots: int = 0):
        self.g = g
        self.k = int(k)
        self.keep_pi = bool(keep_pi)
        h = ctypes.c_void_p()
        _check(load_library().ahpp_server_create(g._h, int(max_device_bytes), int(max_slots), self.k,
                                                 int(max_iters), 1 if keep_pi else 0, ctypes.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            load_library().ahpp_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, tag: int, source: int, eps: float) -> None:
        _check(load_library().ahpp_server_submit(self._h, int(tag), int(source), float(eps)))

    def step(self, rounds: int, stream=None) -> int:
        n = ctypes.c_int32(0)
        _check(load_library().ahpp_server_step(self._h, int(rounds), ctypes.byref(n), _stream(self.g.device, stream)))
        return int(n.value)

    def set_solo(self, solo_max: int) -> None:
        """Lone queries on the single-query engine when no query runs in the
        tiles and at most solo_max wait (0: off; see ahpp_server_set_solo)."""
        _check(load_library().ahpp_server_set_solo(self._h, int(solo_max)))

    def info(self) -> dict:
        v = [ctypes.c_int32(0) for _ in range(4)]
        _check(load_library().ahpp_server_info(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("slots", "running", "queued", "ready"), (int(x.value) for x in v)))

    def results(self, max_n: int = 1024, want_pi: bool = False, stream=None) -> list:
        """Finished queries: list of dicts (tag, topk_idx, topk_val, stats, pi)."""
        import torch
        max_n = int(max_n)
        tags = np.zeros(max_n, np.int64)
        idx = np.zeros((max_n, self.k), np.int32)
        val = np.zeros((max_n, self.k), np.float32)
        tn = np.zeros(max_n, np.int32)
        st = (Stats * max(max_n, 1))()
        pi = None
        if want_pi:
            if not self.keep_pi:
                raise ValueError("server was created without keep_pi")
            # Only as many vectors as are waiting (each is n_u floats).
            max_n = min(max_n, self.info()["ready"])
            pi = torch.empty((max(max_n, 1), self.g.n_u), dtype=torch.float32,
                             device=torch.device("cuda", self.g.device))
        n = ctypes.c_int32(0)
        _check(load_library().ahpp_server_results(self._h, max_n, _np_ptr(tags), _np_ptr(idx), _np_ptr(val),
                                                  _np_ptr(tn), ctypes.cast(st, ctypes.c_void_p), _dev_ptr(pi),
                                                  ctypes.byref(n), _stream(self.g.device, stream)))
        out = []
        for i in range(int(n.value)):
            m = int(tn[i])
            out.append({"tag": int(tags[i]), "topk_idx": idx[i, :m].copy(), "topk_val": val[i, :m].copy(),
                        "stats": st[i].as_dict(), "pi": None if pi is None else pi[i]})
        return out
