"""ctypes binding of libpathsamp.so (the C ABI of include/pathsamp.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device buffers are torch tensors (``data_ptr()``), streams are torch streams
(``cuda_stream``); host buffers are numpy arrays.  There is no fallback: if the
library cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpathsamp.so")

PM_OK, PM_EINVAL, PM_EGRAPH, PM_EOVERFLOW, PM_ENOMEM, PM_EDEVICE, PM_EBUSY, PM_ECANCELED = 0, -1, -2, -3, -4, -5, -6, -7
PM_VALIDATE, PM_CHECK_SYMMETRY = 1, 2
NUM_TALLIES = 8


class PathSampError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


class CsrView(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("row_offsets", ctypes.c_void_p), ("cols", ctypes.c_void_p),
                ("on_device", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("k_path", ctypes.c_uint64), ("k_cent", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("first_id_path", ctypes.c_uint64), ("first_id_cent", ctypes.c_uint64), ("delta", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("tally_path", ctypes.c_uint64 * NUM_TALLIES), ("tally_cent", ctypes.c_uint64 * NUM_TALLIES),
                ("W", ctypes.c_uint64), ("Lambda", ctypes.c_uint64), ("N1", ctypes.c_uint64),
                ("k_path", ctypes.c_uint64), ("k_cent", ctypes.c_uint64),
                ("est", ctypes.c_double * 7), ("lo", ctypes.c_double * 7), ("hi", ctypes.c_double * 7),
                ("est_basic", ctypes.c_double * 7)]

    def to_dict(self) -> dict:
        return {
            "tally_path": [int(x) for x in self.tally_path],
            "tally_cent": [int(x) for x in self.tally_cent],
            "W": int(self.W), "Lambda": int(self.Lambda), "N1": int(self.N1),
            "k_path": int(self.k_path), "k_cent": int(self.k_cent),
            "est": list(self.est), "lo": list(self.lo), "hi": list(self.hi), "est_basic": list(self.est_basic),
        }


class ProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


class Exact(ctypes.Structure):
    _fields_ = [("C", ctypes.c_uint64 * 7), ("N", ctypes.c_uint64 * 7), ("triangles", ctypes.c_uint64)]


class EdgeView(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("num_edges", ctypes.c_int64), ("src", ctypes.c_void_p),
                ("dst", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class Tune(ctypes.Structure):
    _fields_ = [("samples_per_tile", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_active", ctypes.c_int32), ("max_graphs", ctypes.c_int32),
                ("step_samples", ctypes.c_uint64), ("k_pilot", ctypes.c_uint64), ("k_max", ctypes.c_uint64),
                ("samples_per_tile", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_uint32), ("motif_mask", ctypes.c_uint32), ("rel_err", ctypes.c_double),
                ("delta", ctypes.c_double), ("seed", ctypes.c_uint64), ("k_path", ctypes.c_uint64),
                ("k_cent", ctypes.c_uint64)]


class ReqStats(ctypes.Structure):
    _fields_ = [("queued_ms", ctypes.c_double), ("latency_ms", ctypes.c_double), ("k_path", ctypes.c_uint64),
                ("k_cent", ctypes.c_uint64), ("steps", ctypes.c_uint32), ("capped_mask", ctypes.c_uint32),
                ("unseen_mask", ctypes.c_uint32), ("prepared", ctypes.c_int32)]

    def to_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint64), ("samples", ctypes.c_uint64), ("requests_done", ctypes.c_uint64),
                ("resident_bytes", ctypes.c_uint64), ("resident_graphs", ctypes.c_uint64),
                ("preparations", ctypes.c_uint64), ("evictions", ctypes.c_uint64), ("busy_ms", ctypes.c_double)]

    def to_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("dmax", ctypes.c_int64), ("isolated", ctypes.c_int64),
                ("W", ctypes.c_uint64), ("Lambda", ctypes.c_uint64), ("N1", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64)]


_lib = None

# name -> (restype, argtypes); kept in step with include/pathsamp.h
_P = ctypes.c_void_p
_SIGNATURES = {
    "pm_count_motifs": (ctypes.c_int32, [ctypes.POINTER(CsrView), ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.POINTER(Result)]),
    "pm_graph_create": (ctypes.c_int32, [ctypes.POINTER(CsrView), ctypes.c_uint32, _P, ctypes.POINTER(_P)]),
    "pm_graph_info_get": (ctypes.c_int32, [_P, ctypes.POINTER(GraphInfo)]),
    "pm_graph_export": (ctypes.c_int32, [_P, _P, _P, _P, _P, _P, _P]),
    "pm_graph_destroy": (ctypes.c_int32, [_P]),
    "pm_count": (ctypes.c_int32, [_P, ctypes.POINTER(Params), ctypes.POINTER(Result), _P]),
    "pm_graph_build_alias": (ctypes.c_int32, [_P, _P]),
    "pm_count_alias": (ctypes.c_int32, [_P, ctypes.POINTER(Params), ctypes.POINTER(Result), _P]),
    "pm_graph_alias_export": (ctypes.c_int32, [_P, ctypes.c_int32, _P, _P, _P]),
    "pm_sample_async": (ctypes.c_int32, [_P, ctypes.POINTER(Params), _P, _P]),
    "pm_finalize": (ctypes.c_int32, [_P, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(Result)]),
    "pm_chernoff_interval": (ctypes.c_int32, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "pm_samples_for_error": (ctypes.c_int32, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                              ctypes.POINTER(ctypes.c_uint64)]),
    "pm_philox_device": (ctypes.c_int32, [_P, _P, ctypes.c_int64]),
    "pm_device_copy": (ctypes.c_int32, [_P, _P, ctypes.c_uint64, _P]),
    "pm_device_gather": (ctypes.c_int32, [_P, ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint64, _P]),
    "pm_set_sampler_shape": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32]),
    "pm_set_draw_order": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_uint64]),
    "pm_set_search_mode": (ctypes.c_int32, [ctypes.c_int32]),
    "pm_count_noalloc": (ctypes.c_int32, [_P, ctypes.POINTER(Params), ctypes.POINTER(Result), _P]),
    "pm_static_scratch_bytes": (ctypes.c_uint64, []),
    "pm_adjacent": (ctypes.c_int32, [_P, _P, _P, ctypes.c_int64, _P, ctypes.c_int32, _P]),
    "pm_draw_order": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _P,
                                       _P]),
    "pm_release_cached_memory": (ctypes.c_int32, []),
    "pm_profile_enable": (ctypes.c_int32, [ctypes.c_int32]),
    "pm_profile_read": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "pm_profile_select": (ctypes.c_int32, [ctypes.c_char_p]),
    "pm_batch_create": (ctypes.c_int32, [_P, _P, ctypes.c_int32, _P, _P, ctypes.POINTER(_P)]),
    "pm_batch_set_params": (ctypes.c_int32, [_P, _P]),
    "pm_batch_run": (ctypes.c_int32, [_P, _P, _P]),
    "pm_batch_get_tune": (ctypes.c_int32, [_P, ctypes.POINTER(Tune)]),
    "pm_batch_destroy": (ctypes.c_int32, [_P]),
    "pm_count_batch": (ctypes.c_int32, [_P, _P, _P, ctypes.c_int32, _P, _P]),
    "pm_samples_for_request": (ctypes.c_int32, [_P, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                                ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64),
                                                ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32),
                                                ctypes.POINTER(ctypes.c_uint32)]),
    "pm_server_create": (ctypes.c_int32, [ctypes.POINTER(ServerCfg), ctypes.POINTER(_P)]),
    "pm_server_add_graph": (ctypes.c_int32, [_P, ctypes.POINTER(CsrView), ctypes.c_uint32,
                                             ctypes.POINTER(ctypes.c_uint32)]),
    "pm_server_preload": (ctypes.c_int32, [_P, ctypes.c_uint32]),
    "pm_server_submit": (ctypes.c_int32, [_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "pm_server_wait": (ctypes.c_int32, [_P, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(Result),
                                        ctypes.POINTER(ReqStats)]),
    "pm_server_cancel": (ctypes.c_int32, [_P, ctypes.c_uint64]),
    "pm_server_get_stats": (ctypes.c_int32, [_P, ctypes.POINTER(ServerStats)]),
    "pm_server_destroy": (ctypes.c_int32, [_P]),
    "pm_exact_counts": (ctypes.c_int32, [_P, ctypes.POINTER(Exact), _P]),
    "pm_csr_from_edges": (ctypes.c_int32, [ctypes.POINTER(EdgeView), _P, _P, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_int64), _P]),
    "pm_graph_from_edges": (ctypes.c_int32, [ctypes.POINTER(EdgeView), ctypes.c_uint32, _P, ctypes.POINTER(_P)]),
    "pm_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "pm_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libpathsamp.so (building it first only if it does not exist)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build

        _build.build()
    handle = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(handle, name)
        fn.restype = res
        fn.argtypes = args
    _lib = handle
    return handle


def _check(status: int, where: str):
    if status != PM_OK:
        msg = lib().pm_last_error().decode(errors="replace")
        raise PathSampError(status, where, msg)


def _stream_ptr(stream):
    if stream is None:
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _csr_view(off, col):
    """CsrView over torch CUDA tensors or host numpy arrays; returns the
    view and the objects that keep the memory alive."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(off, torch.Tensor):
        if off.dtype != torch.int64 or col.dtype != torch.int32:
            raise TypeError("row_offsets must be int64 and cols int32")
        if not (off.is_cuda and col.is_cuda):
            off_np = off.cpu().numpy()
            col_np = col.cpu().numpy()
            return _csr_view(off_np, col_np)
        off = off.contiguous()
        col = col.contiguous()
        v = CsrView(off.numel() - 1, off.data_ptr(), col.data_ptr() if col.numel() else None, 1)
        return v, (off, col)
    off = np.ascontiguousarray(off, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    v = CsrView(off.size - 1, off.ctypes.data, col.ctypes.data if col.size else None, 0)
    return v, (off, col)


def _edge_view(n, src, dst):
    """EdgeView over torch CUDA tensors or host arrays (int32); returns the
    view and the objects that keep the memory alive."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        torch = None
    if torch is not None and isinstance(src, torch.Tensor):
        if src.dtype != torch.int32 or dst.dtype != torch.int32 or src.numel() != dst.numel():
            raise TypeError("src and dst must be int32 tensors of one length")
        if src.is_cuda and dst.is_cuda:
            src, dst = src.contiguous(), dst.contiguous()
            return EdgeView(n, src.numel(), src.data_ptr() if src.numel() else None,
                            dst.data_ptr() if dst.numel() else None, 1), (src, dst)
        src, dst = src.cpu().numpy(), dst.cpu().numpy()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.size != dst.size:
        raise ValueError("src and dst differ in length")
    return EdgeView(n, src.size, src.ctypes.data if src.size else None, dst.ctypes.data if dst.size else None,
                    0), (src, dst)


def csr_from_edges(n: int, src, dst, stream=None):
    """pm_csr_from_edges: (row_offsets int64[n+1], cols int32[2m]) as CUDA tensors."""
    import torch

    view, keep = _edge_view(n, src, dst)
    cap = 2 * view.num_edges
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    col = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    slots = ctypes.c_int64()
    _check(lib().pm_csr_from_edges(ctypes.byref(view), off.data_ptr(), col.data_ptr(), cap, ctypes.byref(slots),
                                   _stream_ptr(stream)), "pm_csr_from_edges")
    del keep
    return off, col[:slots.value].clone()


class Graph:
    """A prepared graph resident on the current device (pm_graph handle)."""

    def __init__(self, off, col, flags: int = PM_VALIDATE | PM_CHECK_SYMMETRY, stream=None):
        L = lib()
        view, self._keep = _csr_view(off, col)
        h = ctypes.c_void_p()
        _check(L.pm_graph_create(ctypes.byref(view), flags, _stream_ptr(stream), ctypes.byref(h)),
               "pm_graph_create")
        self._keep = None
        self._h = h

    @property
    def handle(self):
        return self._h

    @classmethod
    def from_edges(cls, n: int, src, dst, flags: int = PM_VALIDATE | PM_CHECK_SYMMETRY, stream=None):
        """pm_graph_from_edges: ingest an edge list and prepare it in one call."""
        view, keep = _edge_view(n, src, dst)
        g = cls.__new__(cls)
        h = ctypes.c_void_p()
        _check(lib().pm_graph_from_edges(ctypes.byref(view), flags, _stream_ptr(stream), ctypes.byref(h)),
               "pm_graph_from_edges")
        g._h = h
        del keep
        return g

    def info(self) -> dict:
        gi = GraphInfo()
        _check(lib().pm_graph_info_get(self._h, ctypes.byref(gi)), "pm_graph_info_get")
        return {f: int(getattr(gi, f)) for f, _ in GraphInfo._fields_}

    def export(self, stream=None) -> dict:
        gi = self.info()
        n, slots = gi["n"], 2 * gi["m"]
        off = np.zeros(n + 1, np.int64)
        col = np.zeros(max(slots, 1), np.int32)
        rank = np.zeros(max(n, 1), np.int32)
        pt = np.zeros(max(slots, 1), np.uint64)
        pl = np.zeros(max(slots, 1), np.uint64)
        _check(lib().pm_graph_export(self._h, off.ctypes.data, col.ctypes.data, rank.ctypes.data, pt.ctypes.data,
                                     pl.ctypes.data, _stream_ptr(stream)), "pm_graph_export")
        return {"off": off, "col": col[:slots], "rank": rank[:n], "p_tau": pt[:slots], "p_lam": pl[:slots]}

    def count(self, k_path: int, k_cent: int | None = None, seed: int = 1, first_path: int = 0,
              first_cent: int = 0, delta: float = 0.01, stream=None) -> dict:
        p = Params(k_path, k_path if k_cent is None else k_cent, seed, first_path, first_cent, delta)
        r = Result()
        _check(lib().pm_count(self._h, ctypes.byref(p), ctypes.byref(r), _stream_ptr(stream)), "pm_count")
        return r.to_dict()

    def count_noalloc(self, k_path: int, k_cent: int | None = None, seed: int = 1, first_path: int = 0,
                      first_cent: int = 0, delta: float = 0.01, stream=None) -> dict:
        """pm_count_noalloc: pm_count with the library's fixed device scratch."""
        p = Params(k_path, k_path if k_cent is None else k_cent, seed, first_path, first_cent, delta)
        r = Result()
        _check(lib().pm_count_noalloc(self._h, ctypes.byref(p), ctypes.byref(r), _stream_ptr(stream)),
               "pm_count_noalloc")
        return r.to_dict()

    def build_alias(self, stream=None):
        """pm_graph_build_alias: the alias-draw tables of both samplers."""
        _check(lib().pm_graph_build_alias(self._h, _stream_ptr(stream)), "pm_graph_build_alias")

    def count_alias(self, k_path: int, k_cent: int | None = None, seed: int = 1, first_path: int = 0,
                    first_cent: int = 0, delta: float = 0.01, stream=None) -> dict:
        """pm_count_alias: both samplers through the alias tables."""
        p = Params(k_path, k_path if k_cent is None else k_cent, seed, first_path, first_cent, delta)
        r = Result()
        _check(lib().pm_count_alias(self._h, ctypes.byref(p), ctypes.byref(r), _stream_ptr(stream)),
               "pm_count_alias")
        return r.to_dict()

    def alias_export(self, centered: bool, stream=None):
        """(K uint64[2m], alias int64[2m]) of one sampler's alias table."""
        slots = 2 * self.info()["m"]
        K = np.zeros(max(slots, 1), np.uint64)
        A = np.zeros(max(slots, 1), np.int64)
        _check(lib().pm_graph_alias_export(self._h, 1 if centered else 0, K.ctypes.data, A.ctypes.data,
                                           _stream_ptr(stream)), "pm_graph_alias_export")
        return K[:slots], A[:slots]

    def exact(self, stream=None) -> dict:
        """pm_exact_counts: {"C": [0, C1..C6], "N": [0, N1..N6], "triangles": T}."""
        e = Exact()
        _check(lib().pm_exact_counts(self._h, ctypes.byref(e), _stream_ptr(stream)), "pm_exact_counts")
        return {"C": [int(x) for x in e.C], "N": [int(x) for x in e.N], "triangles": int(e.triangles)}

    def sample_async(self, tallies, k_path: int, k_cent: int, seed: int, first_path: int = 0, first_cent: int = 0,
                     stream=None):
        """Enqueue both samplers; tallies is a CUDA uint64/int64 tensor of 16."""
        if tallies.numel() < 2 * NUM_TALLIES or not tallies.is_cuda:
            raise ValueError("tallies must be a CUDA tensor of at least 16 64-bit integers")
        p = Params(k_path, k_cent, seed, first_path, first_cent, 0.01)
        _check(lib().pm_sample_async(self._h, ctypes.byref(p), ctypes.c_void_p(tallies.data_ptr()),
                                     _stream_ptr(stream)), "pm_sample_async")

    def adjacent(self, a, b, mode: int = 2, stream=None):
        """pm_adjacent: uint8 tensor, 1 where relabelled ids a[i], b[i] are
        adjacent (a, b int32 CUDA tensors of one length)."""
        import torch

        assert a.is_cuda and b.is_cuda and a.dtype == torch.int32 and b.dtype == torch.int32
        assert a.numel() == b.numel()
        a, b = a.contiguous(), b.contiguous()
        out = torch.empty(a.numel(), dtype=torch.uint8, device=a.device)
        _check(lib().pm_adjacent(self._h, a.data_ptr(), b.data_ptr(), a.numel(), out.data_ptr(), mode,
                                 _stream_ptr(stream)), "pm_adjacent")
        return out

    def draw_order(self, centered: bool, seed: int, k: int, first: int = 0, stream=None):
        """pm_draw_order: int32 CUDA tensor of the k sample offsets (id - first)
        of one sort chunk in the order a draw-ordered launch runs them."""
        import torch

        out = torch.empty(k, dtype=torch.int32, device="cuda")
        _check(lib().pm_draw_order(self._h, 1 if centered else 0, seed, first, k, out.data_ptr(),
                                   _stream_ptr(stream)), "pm_draw_order")
        return out

    def destroy(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().pm_graph_destroy(self._h), "pm_graph_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def make_params(k_path: int, k_cent: int | None = None, seed: int = 1, first_path: int = 0, first_cent: int = 0,
                delta: float = 0.01) -> Params:
    return Params(k_path, k_path if k_cent is None else k_cent, seed, first_path, first_cent, delta)


def _params_array(params):
    arr = (Params * len(params))()
    for i, p in enumerate(params):
        arr[i] = p if isinstance(p, Params) else make_params(**p)
    return arr


def _graph_array(graphs):
    arr = (ctypes.c_void_p * len(graphs))()
    for i, g in enumerate(graphs):
        arr[i] = g.handle.value
    return arr


class Batch:
    """pm_batch: many prepared graphs sampled by one captured persistent launch."""

    def __init__(self, graphs, params, tune=None, stream=None):
        self._graphs = list(graphs)  # keep the handles alive
        self.count = len(self._graphs)
        ga, pa = _graph_array(self._graphs), _params_array(params)
        t = None if tune is None else ctypes.byref(Tune(*tune))
        h = ctypes.c_void_p()
        _check(lib().pm_batch_create(ga, pa, self.count, t, _stream_ptr(stream), ctypes.byref(h)), "pm_batch_create")
        self._h = h

    def set_params(self, params):
        _check(lib().pm_batch_set_params(self._h, _params_array(params)), "pm_batch_set_params")

    def run(self, stream=None) -> list:
        out = (Result * self.count)()
        _check(lib().pm_batch_run(self._h, out, _stream_ptr(stream)), "pm_batch_run")
        return [r.to_dict() for r in out]

    def tune(self):
        t = Tune()
        _check(lib().pm_batch_get_tune(self._h, ctypes.byref(t)), "pm_batch_get_tune")
        return (t.samples_per_tile, t.blocks_per_cu)

    def destroy(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().pm_batch_destroy(self._h), "pm_batch_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def count_batch(graphs, params, tune=None, stream=None) -> list:
    """pm_count_batch: one-shot batched count."""
    ga, pa = _graph_array(graphs), _params_array(params)
    out = (Result * len(graphs))()
    t = None if tune is None else ctypes.byref(Tune(*tune))
    _check(lib().pm_count_batch(ga, pa, out, len(graphs), t, _stream_ptr(stream)), "pm_count_batch")
    return [r.to_dict() for r in out]


def samples_for_request(tally_path, tally_cent, k0: int, W: int, Lambda: int, N1: int, motif_mask: int,
                        rel_err: float, delta: float, k_max: int):
    """pm_samples_for_request: (k_path, k_cent, capped_mask, unseen_mask)."""
    tp = (ctypes.c_uint64 * NUM_TALLIES)(*[int(x) for x in tally_path])
    tc = (ctypes.c_uint64 * NUM_TALLIES)(*[int(x) for x in tally_cent])
    kp, kc = ctypes.c_uint64(), ctypes.c_uint64()
    cap, uns = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().pm_samples_for_request(tp, tc, k0, W, Lambda, N1, motif_mask, rel_err, delta, k_max,
                                        ctypes.byref(kp), ctypes.byref(kc), ctypes.byref(cap), ctypes.byref(uns)),
           "pm_samples_for_request")
    return kp.value, kc.value, cap.value, uns.value


class Server:
    """pm_server: continuous batching of motif-count requests over registered graphs.

    Registered CSR buffers (torch tensors or numpy arrays) are kept referenced
    here, since the server may read them again after an eviction."""

    def __init__(self, hbm_budget: int = 0, max_active: int = 0, max_graphs: int = 0, step_samples: int = 0,
                 k_pilot: int = 0, k_max: int = 0, samples_per_tile: int = 0, blocks_per_cu: int = 0):
        cfg = ServerCfg(hbm_budget, max_active, max_graphs, step_samples, k_pilot, k_max, samples_per_tile,
                        blocks_per_cu)
        h = ctypes.c_void_p()
        _check(lib().pm_server_create(ctypes.byref(cfg), ctypes.byref(h)), "pm_server_create")
        self._h = h
        self._keep = []

    def add_graph(self, off, col, flags: int = PM_VALIDATE | PM_CHECK_SYMMETRY) -> int:
        view, keep = _csr_view(off, col)
        gid = ctypes.c_uint32()
        _check(lib().pm_server_add_graph(self._h, ctypes.byref(view), flags, ctypes.byref(gid)),
               "pm_server_add_graph")
        self._keep.append(keep)
        return gid.value

    def preload(self, gid: int):
        _check(lib().pm_server_preload(self._h, gid), "pm_server_preload")

    def submit(self, graph: int, rel_err: float = 0.01, delta: float = 0.01, seed: int = 1, motif_mask: int = 0,
               k_path: int = 0, k_cent: int = 0) -> int:
        rq = Request(graph, motif_mask, rel_err, delta, seed, k_path, k_cent)
        t = ctypes.c_uint64()
        _check(lib().pm_server_submit(self._h, ctypes.byref(rq), ctypes.byref(t)), "pm_server_submit")
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        """(result dict, stats dict); raises PathSampError with the request's status."""
        r, st = Result(), ReqStats()
        _check(lib().pm_server_wait(self._h, ticket, timeout_ms, ctypes.byref(r), ctypes.byref(st)),
               "pm_server_wait")
        return r.to_dict(), st.to_dict()

    def cancel(self, ticket: int):
        _check(lib().pm_server_cancel(self._h, ticket), "pm_server_cancel")

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().pm_server_get_stats(self._h, ctypes.byref(st)), "pm_server_get_stats")
        return st.to_dict()

    def destroy(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().pm_server_destroy(self._h), "pm_server_destroy")
            self._h = ctypes.c_void_p()
            self._keep = []

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def count_motifs(off, col, k: int, seed: int = 1) -> dict:
    """pm_count_motifs: prepare, sample k + k, finalize (99% bars)."""
    view, keep = _csr_view(off, col)
    r = Result()
    _check(lib().pm_count_motifs(ctypes.byref(view), k, seed, ctypes.byref(r)), "pm_count_motifs")
    del keep
    return r.to_dict()


def finalize(tally_path, tally_cent, W: int, Lambda: int, N1: int, k_path: int, k_cent: int,
             delta: float = 0.01) -> dict:
    tp = np.ascontiguousarray(tally_path, dtype=np.uint64)
    tc = np.ascontiguousarray(tally_cent, dtype=np.uint64)
    r = Result()
    _check(lib().pm_finalize(tp.ctypes.data, tc.ctypes.data, W, Lambda, N1, k_path, k_cent, delta, ctypes.byref(r)),
           "pm_finalize")
    return r.to_dict()


def chernoff_interval(count: int, k: int, delta: float):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(lib().pm_chernoff_interval(count, k, delta, ctypes.byref(lo), ctypes.byref(hi)), "pm_chernoff_interval")
    return lo.value, hi.value


def samples_for_error(rel_err: float, delta: float, alpha: float) -> int:
    k = ctypes.c_uint64()
    _check(lib().pm_samples_for_error(rel_err, delta, alpha, ctypes.byref(k)), "pm_samples_for_error")
    return int(k.value)


def set_draw_order(enabled: bool, min_samples: int = 0):
    """pm_set_draw_order: sort sample batches of at least min_samples (0: the
    default) by their draws first."""
    _check(lib().pm_set_draw_order(1 if enabled else 0, min_samples), "pm_set_draw_order")


SEARCH_LANE, SEARCH_WAVE, SEARCH_HASH = 0, 1, 2


def set_search_mode(mode: int):
    """pm_set_search_mode: adjacency tests through the sorted rows per lane (0)
    or by the whole wave (1), or through the row hash (2, the default)."""
    _check(lib().pm_set_search_mode(mode), "pm_set_search_mode")


def set_sampler_shape(samples_per_lane: int, blocks_per_cu: int):
    """Launch shape of the sampling kernels (tallies do not depend on it)."""
    _check(lib().pm_set_sampler_shape(samples_per_lane, blocks_per_cu), "pm_set_sampler_shape")


def static_scratch_bytes() -> int:
    """pm_static_scratch_bytes: size of pm_count_noalloc's per-device array."""
    return int(lib().pm_static_scratch_bytes())


def release_cached_memory():
    """Return the library's cached device blocks of the current device."""
    _check(lib().pm_release_cached_memory(), "pm_release_cached_memory")


def philox_device(inputs) -> np.ndarray:
    """Device Philox4x32-10 on rows (c0 c1 c2 c3 k0 k1); returns rows of 4 words."""
    a = np.ascontiguousarray(inputs, dtype=np.uint32).reshape(-1, 6)
    out = np.zeros((a.shape[0], 4), np.uint32)
    _check(lib().pm_philox_device(a.ctypes.data, out.ctypes.data, a.shape[0]), "pm_philox_device")
    return out


def device_copy(dst, src, stream=None):
    """pm_device_copy between two same-sized CUDA tensors (asynchronous)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("tensors differ in size")
    _check(lib().pm_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, _stream_ptr(stream)), "pm_device_copy")


def device_gather(table, count: int, seed: int = 1, stream=None):
    """pm_device_gather over a CUDA tensor (asynchronous)."""
    _check(lib().pm_device_gather(table.data_ptr(), table.numel() * table.element_size(), count, seed,
                                  _stream_ptr(stream)), "pm_device_gather")


def profile_enable(on: bool = True):
    """Clear per-kernel totals and switch HIP-event timing on or off."""
    _check(lib().pm_profile_enable(1 if on else 0), "pm_profile_enable")


def profile_select(names=None):
    """Record only the named scopes (an iterable of kernel names as
    profile_read reports them); None or empty records every scope."""
    joined = ",".join(names) if names else ""
    _check(lib().pm_profile_select(joined.encode()), "pm_profile_select")


def profile_read() -> dict:
    """{kernel name: (launches, total ms)} since the last profile_enable."""
    cnt = ctypes.c_int32()
    _check(lib().pm_profile_read(None, 0, ctypes.byref(cnt)), "pm_profile_read")
    arr = (ProfileEntry * max(cnt.value, 1))()
    _check(lib().pm_profile_read(ctypes.cast(arr, ctypes.c_void_p), cnt.value, ctypes.byref(cnt)), "pm_profile_read")
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(cnt.value)}
