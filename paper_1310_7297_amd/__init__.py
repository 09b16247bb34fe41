"""MI355X visibility color maps: thin ctypes binding of libvcm (include/vcm.h).

The functions named like the C entry points (vcm_build_index, vcm_compute,
...) only marshal arguments: every step of the computation runs in the HIP
kernels of libvcm.so.  torch supplies device memory and streams.  There is no
fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, Optional

import numpy as np

from . import scenes

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvcm.so")

VCM_OK, VCM_E_INVALID, VCM_E_NOMEM, VCM_E_DEVICE, VCM_E_AGAIN, VCM_E_NOTFOUND, \
    VCM_E_PENDING, VCM_E_INTERNAL = range(8)
STATUS_NAMES = {0: "VCM_OK", 1: "VCM_E_INVALID", 2: "VCM_E_NOMEM", 3: "VCM_E_DEVICE",
                4: "VCM_E_AGAIN", 5: "VCM_E_NOTFOUND", 6: "VCM_E_PENDING", 7: "VCM_E_INTERNAL"}
VCM_FP32_RECHECK, VCM_FP64 = 0, 1

# Every symbol include/vcm.h declares.
EXPORTS = ("vcm_last_error", "vcm_version", "vcm_build_index", "vcm_free_index",
           "vcm_index_get_info", "vcm_compute", "vcm_compute_noalloc", "vcm_compute_batch",
           "vcm_batch_create",
           "vcm_batch_run", "vcm_batch_get_info", "vcm_batch_destroy", "vcm_server_create",
           "vcm_submit", "vcm_poll", "vcm_wait", "vcm_server_drain", "vcm_server_hold",
           "vcm_server_get_stats", "vcm_server_reset_stats", "vcm_server_destroy", "vcm_tune_cell_size", "vcm_map_error",
           "vcm_error_bounds", "vcm_view_create", "vcm_view_render", "vcm_view_get_info",
           "vcm_view_destroy")


class VcmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class vcm_obstacles(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int64),
                ("lo", ctypes.c_void_p * 3), ("hi", ctypes.c_void_p * 3)]


class vcm_index_opts(ctypes.Structure):
    _fields_ = [("cell_size", ctypes.c_double), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class vcm_index_info(ctypes.Structure):
    _fields_ = [("n_boxes", ctypes.c_int64), ("n_refs", ctypes.c_int64),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("cell_size", ctypes.c_double),
                ("origin", ctypes.c_double * 2), ("device_bytes", ctypes.c_size_t),
                ("build_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("longest_list", ctypes.c_int32)]


class vcm_target(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("normal_axis", ctypes.c_int32),
                ("normal_sign", ctypes.c_int32), ("samples_u", ctypes.c_int32),
                ("samples_v", ctypes.c_int32), ("center", ctypes.c_double * 3),
                ("size", ctypes.c_double * 2)]


class vcm_grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("extent", ctypes.c_double * 3),
                ("n", ctypes.c_int32 * 3)]


class vcm_params(ctypes.Structure):
    _fields_ = [("mu_arcmin", ctypes.c_double), ("near_d0", ctypes.c_double),
                ("fov_deg", ctypes.c_double), ("n_bins", ctypes.c_int32),
                ("bin_scale", ctypes.c_int32), ("method", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("theta_blocks", ctypes.c_int32),
                ("recheck_eps", ctypes.c_double), ("precision", ctypes.c_int32),
                ("gaze", ctypes.c_int32)]


class vcm_query(ctypes.Structure):
    _fields_ = [("target", vcm_target), ("grid", vcm_grid), ("params", vcm_params)]


class vcm_stats(ctypes.Structure):
    _fields_ = [("viewpoints", ctypes.c_uint64), ("rays", ctypes.c_uint64),
                ("box_tests", ctypes.c_uint64), ("rechecks", ctypes.c_uint64),
                ("fp32_disagree", ctypes.c_uint64), ("columns", ctypes.c_uint64),
                ("slot_tests", ctypes.c_uint64), ("inside_box", ctypes.c_uint64),
                ("t_fallbacks", ctypes.c_uint64), ("records", ctypes.c_uint64),
                ("narrow_tests", ctypes.c_uint64), ("kernel_ms", ctypes.c_double),
                ("err_signed", ctypes.c_double), ("err_abs", ctypes.c_double),
                ("bound", ctypes.c_double), ("bound_measured", ctypes.c_double),
                ("blocks", ctypes.c_uint64), ("blocks_decided", ctypes.c_uint64),
                ("leaves", ctypes.c_uint64)]


class vcm_result(ctypes.Structure):
    _fields_ = [("bin", ctypes.c_void_p), ("c", ctypes.c_void_p), ("count", ctypes.c_void_p),
                ("host", ctypes.c_int32)]


class vcm_batch_opts(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


class vcm_tune_opts(ctypes.Structure):
    _fields_ = [("cell_min", ctypes.c_double), ("cell_max", ctypes.c_double),
                ("device", ctypes.c_int32), ("reps", ctypes.c_int32)]


class vcm_tune_result(ctypes.Structure):
    _fields_ = [("best_cell", ctypes.c_double), ("n", ctypes.c_int32),
                ("cell", ctypes.c_double * 16), ("ms", ctypes.c_double * 16)]


class vcm_server_opts(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32)]


class vcm_request_info(ctypes.Structure):
    _fields_ = [("latency_ms", ctypes.c_double), ("queue_ms", ctypes.c_double),
                ("viewpoints", ctypes.c_uint64)]


class vcm_server_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("viewpoints", ctypes.c_uint64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("requests_per_s", ctypes.c_double), ("viewpoints_per_s", ctypes.c_double),
                ("mem_in_use", ctypes.c_size_t), ("mem_peak", ctypes.c_size_t),
                ("mem_budget", ctypes.c_size_t)]


class vcm_view_info(ctypes.Structure):
    _fields_ = [("viewpoints", ctypes.c_uint64), ("device_bytes", ctypes.c_size_t),
                ("create_ms", ctypes.c_double)]


class vcm_batch_info(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("launches", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("viewpoints", ctypes.c_uint64), ("work_items", ctypes.c_uint64),
                ("device_bytes", ctypes.c_size_t), ("tune_ms", ctypes.c_double)]


_lib = None


def load_library(path: Optional[str] = None):
    """Load libvcm.so (after torch, so both share one HIP runtime).

    VCM_LIB overrides the path (to compare two builds of the library)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("VCM_LIB") or LIB_PATH
    try:
        import torch  # noqa: F401  (loads the HIP runtime libvcm links against)
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(path)
    L.vcm_last_error.restype = ctypes.c_char_p
    L.vcm_version.restype = ctypes.c_char_p
    L.vcm_build_index.argtypes = [ctypes.POINTER(vcm_obstacles), ctypes.POINTER(vcm_index_opts),
                                  ctypes.POINTER(ctypes.c_void_p)]
    L.vcm_free_index.argtypes = [ctypes.c_void_p]
    L.vcm_index_get_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(vcm_index_info)]
    L.vcm_compute.argtypes = [ctypes.c_void_p, ctypes.POINTER(vcm_query),
                              ctypes.POINTER(vcm_result), ctypes.c_void_p,
                              ctypes.POINTER(vcm_stats)]
    L.vcm_compute_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(vcm_query),
                                      ctypes.POINTER(vcm_result), ctypes.c_void_p]
    L.vcm_map_error.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                ctypes.c_void_p, ctypes.POINTER(ctypes.c_double * 2)]
    L.vcm_error_bounds.argtypes = [ctypes.POINTER(vcm_query), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_double * 2)]
    L.vcm_compute_batch.argtypes = [ctypes.c_void_p, ctypes.POINTER(vcm_query), ctypes.c_int32,
                                    ctypes.POINTER(vcm_result), ctypes.c_void_p,
                                    ctypes.POINTER(vcm_stats)]
    L.vcm_batch_create.argtypes = [ctypes.c_void_p, ctypes.POINTER(vcm_query), ctypes.c_int32,
                                   ctypes.POINTER(vcm_result), ctypes.POINTER(vcm_batch_opts),
                                   ctypes.POINTER(ctypes.c_void_p)]
    L.vcm_batch_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    L.vcm_batch_get_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(vcm_batch_info)]
    L.vcm_batch_destroy.argtypes = [ctypes.c_void_p]
    L.vcm_server_create.argtypes = [ctypes.c_void_p, ctypes.POINTER(vcm_server_opts),
                                    ctypes.POINTER(ctypes.c_void_p)]
    L.vcm_submit.argtypes = [ctypes.c_void_p, ctypes.POINTER(vcm_query), ctypes.POINTER(vcm_result),
                             ctypes.POINTER(ctypes.c_uint64)]
    L.vcm_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(vcm_request_info)]
    L.vcm_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32,
                           ctypes.POINTER(vcm_request_info)]
    L.vcm_server_drain.argtypes = [ctypes.c_void_p]
    L.vcm_server_get_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(vcm_server_stats)]
    L.vcm_server_reset_stats.argtypes = [ctypes.c_void_p]
    L.vcm_server_destroy.argtypes = [ctypes.c_void_p]
    L.vcm_tune_cell_size.argtypes = [ctypes.POINTER(vcm_obstacles), ctypes.POINTER(vcm_query),
                                     ctypes.c_int32, ctypes.POINTER(vcm_tune_opts),
                                     ctypes.POINTER(vcm_tune_result)]
    L.vcm_view_create.argtypes = [ctypes.c_void_p, ctypes.POINTER(vcm_query), ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_void_p)]
    L.vcm_view_render.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32,
                                  ctypes.POINTER(vcm_result), ctypes.c_void_p]
    L.vcm_view_get_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(vcm_view_info)]
    L.vcm_view_destroy.argtypes = [ctypes.c_void_p]
    L.vcm_server_hold.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    for name in ("vcm_view_create", "vcm_view_render", "vcm_view_get_info", "vcm_view_destroy",
                 "vcm_build_index", "vcm_free_index", "vcm_index_get_info", "vcm_compute",
                 "vcm_compute_noalloc",
                 "vcm_compute_batch", "vcm_batch_create", "vcm_batch_run", "vcm_batch_get_info",
                 "vcm_batch_destroy", "vcm_server_create", "vcm_submit", "vcm_poll", "vcm_wait",
                 "vcm_server_drain", "vcm_server_hold", "vcm_server_get_stats", "vcm_server_reset_stats",
                 "vcm_server_destroy", "vcm_tune_cell_size", "vcm_map_error", "vcm_error_bounds"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != VCM_OK:
        raise VcmError(status, vcm_last_error())


def vcm_last_error() -> str:
    return load_library().vcm_last_error().decode()


def vcm_version() -> str:
    return load_library().vcm_version().decode()


# ------------------------------------------------------------ conversions ---

def make_target(t: scenes.Target) -> vcm_target:
    T = vcm_target()
    T.kind, T.normal_axis, T.normal_sign = int(t.kind), int(t.normal_axis), int(t.normal_sign)
    T.samples_u, T.samples_v = int(t.samples_u), int(t.samples_v)
    for k in range(3):
        T.center[k] = float(t.center[k])
    T.size[0], T.size[1] = float(t.size[0]), float(t.size[1])
    return T


def make_query(q: scenes.Query, precision: int = VCM_FP32_RECHECK) -> vcm_query:
    Q = vcm_query()
    Q.target = make_target(q.target)
    for k in range(3):
        Q.grid.origin[k] = float(q.grid.origin[k])
        Q.grid.extent[k] = float(q.grid.extent[k])
        Q.grid.n[k] = int(q.grid.n[k])
    p = q.params
    P = Q.params
    P.mu_arcmin, P.near_d0, P.fov_deg = float(p.mu_arcmin), float(p.near_d0), float(p.fov_deg)
    P.n_bins, P.bin_scale, P.method = int(p.n_bins), int(p.bin_scale), int(p.method)
    P.mode, P.theta_blocks = int(p.mode), int(p.theta_blocks)
    P.recheck_eps = float(p.recheck_eps)
    P.precision = int(precision)
    P.gaze = int(getattr(p, "gaze", 0))
    return Q


# ------------------------------------------------------------ entry points ---

class Index:
    """Owns a vcm_index handle."""

    def __init__(self, handle: int, dim: int):
        self.handle = ctypes.c_void_p(handle)
        self.dim = dim

    def info(self) -> Dict[str, float]:
        return vcm_index_get_info(self)

    def free(self):
        if self.handle:
            vcm_free_index(self)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _obstacles(scene: scenes.Scene):
    """vcm_obstacles over the scene's arrays (returned with them: keep alive)."""
    lo = np.ascontiguousarray(scene.lo, dtype=np.float64)
    hi = np.ascontiguousarray(scene.hi, dtype=np.float64)
    O = vcm_obstacles()
    O.dim = int(scene.dim)
    O.n = int(lo.shape[1])
    for k in range(3):
        O.lo[k] = lo[k].ctypes.data if O.n else None
        O.hi[k] = hi[k].ctypes.data if O.n else None
    return O, (lo, hi)


def vcm_build_index(scene: scenes.Scene, cell_size: float = 0.0, device: int = 0,
                    stream: Optional[int] = None) -> Index:
    L = load_library()
    O, _keep = _obstacles(scene)
    opts = vcm_index_opts(float(cell_size), int(device), stream)
    h = ctypes.c_void_p()
    _check(L.vcm_build_index(ctypes.byref(O), ctypes.byref(opts), ctypes.byref(h)))
    return Index(h.value, int(scene.dim))


def vcm_free_index(index: Index):
    _check(load_library().vcm_free_index(index.handle))
    index.handle = ctypes.c_void_p()


def vcm_index_get_info(index: Index) -> Dict[str, float]:
    info = vcm_index_info()
    _check(load_library().vcm_index_get_info(index.handle, ctypes.byref(info)))
    return {"n_boxes": info.n_boxes, "n_refs": info.n_refs, "nx": info.nx, "ny": info.ny,
            "cell_size": info.cell_size, "origin": (info.origin[0], info.origin[1]),
            "device_bytes": info.device_bytes, "build_ms": info.build_ms,
            "kernel_ms": info.kernel_ms, "longest_list": info.longest_list}


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def vcm_compute(index: Index, query: scenes.Query, bin_out, c_out=None, count_out=None,
                stream=None, stats: bool = False, precision: int = VCM_FP32_RECHECK):
    """Enqueue one VCM on `stream` (default: torch's current stream).

    bin_out (uint8), c_out (float32), count_out (int16 storage of uint16) are
    torch tensors with one entry per viewpoint, all on the device, or all in
    host memory (then the call returns once they are filled)."""
    L = load_library()
    Q = make_query(query, precision)
    n = query.grid.count
    bufs = [t for t in (bin_out, c_out, count_out) if t is not None]
    host = bool(bufs) and not bufs[0].is_cuda
    for t, name in ((bin_out, "bin"), (c_out, "c"), (count_out, "count")):
        if t is not None:
            if t.is_cuda == host or t.numel() < n or not t.is_contiguous():
                raise ValueError(f"{name}: need contiguous tensors of >= {n} entries, all on the device "
                                 "or all in host memory")
    R = vcm_result(bin_out.data_ptr(), c_out.data_ptr() if c_out is not None else None,
                   count_out.data_ptr() if count_out is not None else None, int(host))
    st = vcm_stats()
    _check(L.vcm_compute(index.handle, ctypes.byref(Q), ctypes.byref(R), _stream_ptr(stream),
                         ctypes.byref(st) if stats else None))
    if stats:
        return {f: getattr(st, f) for f, _ in vcm_stats._fields_}
    return None


def vcm_compute_noalloc(index: Index, query: scenes.Query, bin_out, c_out=None, count_out=None,
                        stream=None, precision: int = VCM_FP32_RECHECK):
    """vcm_compute_noalloc: as vcm_compute, with the library's static scratch
    memory instead of allocations (no statistics)."""
    Q = make_query(query, precision)
    R = _make_result(query.grid.count, bin_out, c_out, count_out)
    _check(load_library().vcm_compute_noalloc(index.handle, ctypes.byref(Q), ctypes.byref(R),
                                              _stream_ptr(stream)))


def _make_result(n, bin_out, c_out=None, count_out=None) -> vcm_result:
    for t, name in ((bin_out, "bin"), (c_out, "c"), (count_out, "count")):
        if t is not None:
            if not t.is_cuda or t.numel() < n or not t.is_contiguous():
                raise ValueError(f"{name}: need a contiguous device tensor of >= {n} entries")
    return vcm_result(bin_out.data_ptr(), c_out.data_ptr() if c_out is not None else None,
                      count_out.data_ptr() if count_out is not None else None)


def _batch_arrays(queries, results, precision):
    nq = len(queries)
    if len(results) != nq:
        raise ValueError("one result triple per query")
    if isinstance(precision, int):
        precision = [precision] * nq
    Qs = (vcm_query * max(nq, 1))()
    Rs = (vcm_result * max(nq, 1))()
    for i, (q, r) in enumerate(zip(queries, results)):
        Qs[i] = make_query(q, precision[i])
        Rs[i] = _make_result(q.grid.count, *r)
    return Qs, Rs


def _stats_dict(st: vcm_stats):
    return {f: getattr(st, f) for f, _ in vcm_stats._fields_}


def vcm_compute_batch(index: Index, queries, results, stream=None, stats: bool = False,
                      precision=VCM_FP32_RECHECK):
    """Enqueue many VCMs over one index; results[i] = (bin, c, count) tensors."""
    L = load_library()
    Qs, Rs = _batch_arrays(queries, results, precision)
    st = vcm_stats()
    _check(L.vcm_compute_batch(index.handle, Qs, len(queries), Rs, _stream_ptr(stream),
                               ctypes.byref(st) if stats else None))
    return _stats_dict(st) if stats else None


class Batch:
    """A prepared batch (vcm_batch_create); run() enqueues one replay."""

    def __init__(self, index: Index, queries, results, chunk: int = 0, blocks_per_cu: int = 0,
                 autotune: bool = False, use_graph: bool = True, precision=VCM_FP32_RECHECK):
        L = load_library()
        self._keep = (index, results)  # buffers must outlive the batch
        Qs, Rs = _batch_arrays(queries, results, precision)
        opts = vcm_batch_opts(int(chunk), int(blocks_per_cu), int(bool(autotune)), int(bool(use_graph)))
        h = ctypes.c_void_p()
        _check(L.vcm_batch_create(index.handle, Qs, len(queries), Rs, ctypes.byref(opts),
                                  ctypes.byref(h)))
        self.handle = h

    def run(self, stream=None):
        _check(load_library().vcm_batch_run(self.handle, _stream_ptr(stream)))

    def info(self):
        i = vcm_batch_info()
        _check(load_library().vcm_batch_get_info(self.handle, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in vcm_batch_info._fields_}

    def close(self):
        if self.handle:
            _check(load_library().vcm_batch_destroy(self.handle))
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A serving loop over one resident index (vcm_server_*).

    submit() returns a ticket, or None when the memory budget is in use
    (VCM_E_AGAIN: retry later); poll() returns None while the request runs,
    else its info dict (raising VcmError if the request failed)."""

    def __init__(self, index: Index, mem_budget_bytes: int = 0, max_inflight: int = 0,
                 max_batch: int = 0, chunk: int = 0, blocks_per_cu: int = 0):
        L = load_library()
        opts = vcm_server_opts(int(mem_budget_bytes), int(max_inflight), int(max_batch), int(chunk),
                               int(blocks_per_cu))
        h = ctypes.c_void_p()
        _check(L.vcm_server_create(index.handle, ctypes.byref(opts), ctypes.byref(h)))
        self.handle = h
        self._index = index
        self._held = {}  # ticket -> result tensors, kept alive until finished

    def submit(self, query: scenes.Query, result, precision: int = VCM_FP32_RECHECK):
        Q = make_query(query, precision)
        R = _make_result(query.grid.count, *result)
        t = ctypes.c_uint64()
        st = load_library().vcm_submit(self.handle, ctypes.byref(Q), ctypes.byref(R), ctypes.byref(t))
        if st == VCM_E_AGAIN:
            return None
        _check(st)
        self._held[t.value] = result
        return t.value

    def _finish(self, st, ticket, info):
        if st == VCM_E_PENDING:
            return None
        self._held.pop(ticket, None)
        _check(st)
        return {"latency_ms": info.latency_ms, "queue_ms": info.queue_ms,
                "viewpoints": info.viewpoints}

    def poll(self, ticket: int):
        info = vcm_request_info()
        st = load_library().vcm_poll(self.handle, ticket, ctypes.byref(info))
        return self._finish(st, ticket, info)

    def wait(self, ticket: int, timeout_ms: int = -1):
        info = vcm_request_info()
        st = load_library().vcm_wait(self.handle, ticket, int(timeout_ms), ctypes.byref(info))
        return self._finish(st, ticket, info)

    def drain(self):
        _check(load_library().vcm_server_drain(self.handle))

    def hold(self, on: bool = True):
        """Hold launches (admitted requests queue) or release them."""
        _check(load_library().vcm_server_hold(self.handle, int(bool(on))))

    def stats(self):
        s = vcm_server_stats()
        _check(load_library().vcm_server_get_stats(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in vcm_server_stats._fields_}

    def reset_stats(self):
        _check(load_library().vcm_server_reset_stats(self.handle))

    def close(self):
        if self.handle:
            _check(load_library().vcm_server_destroy(self.handle))
            self.handle = ctypes.c_void_p()
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class View:
    """Incremental processing (vcm_view_*): the query's visibility kept at a
    360-degree field of view; render() colours it for any field of view and
    gaze without tracing again."""

    def __init__(self, index: Index, query: scenes.Query, stream=None, precision: int = VCM_FP32_RECHECK):
        L = load_library()
        self._index = index
        self.query = query
        Q = make_query(query, precision)
        h = ctypes.c_void_p()
        _check(L.vcm_view_create(index.handle, ctypes.byref(Q), _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    def render(self, fov_deg: float, gaze: int, bin_out, c_out=None, count_out=None, stream=None):
        R = _make_result(self.query.grid.count, bin_out, c_out, count_out)
        _check(load_library().vcm_view_render(self.handle, float(fov_deg), int(gaze), ctypes.byref(R),
                                              _stream_ptr(stream)))

    def info(self):
        i = vcm_view_info()
        _check(load_library().vcm_view_get_info(self.handle, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in vcm_view_info._fields_}

    def close(self):
        if self.handle:
            _check(load_library().vcm_view_destroy(self.handle))
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vcm_tune_cell_size(scene: scenes.Scene, queries, cell_min: float = 0.0, cell_max: float = 0.0,
                       reps: int = 0, device: int = 0, precision=VCM_FP32_RECHECK):
    """Fastest index column width for these queries (vcm_tune_cell_size)."""
    L = load_library()
    O, _keep = _obstacles(scene)
    if isinstance(precision, int):
        precision = [precision] * len(queries)
    Qs = (vcm_query * max(len(queries), 1))()
    for i, q in enumerate(queries):
        Qs[i] = make_query(q, precision[i])
    opts = vcm_tune_opts(float(cell_min), float(cell_max), int(device), int(reps))
    r = vcm_tune_result()
    _check(L.vcm_tune_cell_size(ctypes.byref(O), Qs, len(queries), ctypes.byref(opts), ctypes.byref(r)))
    return {"best_cell": r.best_cell, "cells": [r.cell[i] for i in range(r.n)],
            "ms": [r.ms[i] for i in range(r.n)]}


def vcm_map_error(c_exact, c_approx, stream=None):
    """Signed and absolute approximation error (Sec. V-A) of two device maps."""
    out = (ctypes.c_double * 2)()
    n = c_exact.numel()
    if c_approx.numel() != n:
        raise ValueError("maps differ in size")
    _check(load_library().vcm_map_error(c_exact.data_ptr(), c_approx.data_ptr(), n,
                                        c_exact.device.index or 0, _stream_ptr(stream),
                                        ctypes.byref(out)))
    return out[0], out[1]


def vcm_error_bounds(query: scenes.Query, dim: int):
    out = (ctypes.c_double * 2)()
    Q = make_query(query)
    _check(load_library().vcm_error_bounds(ctypes.byref(Q), int(dim), ctypes.byref(out)))
    return {"mbr": out[0], "tangent": out[1]}


def alloc_result(n: int, device="cuda"):
    import torch
    return (torch.empty(n, dtype=torch.uint8, device=device),
            torch.empty(n, dtype=torch.float32, device=device),
            torch.empty(n, dtype=torch.int16, device=device))


def compute_map(index: Index, query: scenes.Query, stats: bool = False,
                precision: int = VCM_FP32_RECHECK):
    """Convenience: allocate, compute, synchronise, return numpy arrays."""
    import torch
    n = query.grid.count
    b, c, cnt = alloc_result(n)
    st = vcm_compute(index, query, b, c, cnt, stats=stats, precision=precision)
    torch.cuda.synchronize()
    out = {"bin": b.cpu().numpy(), "c": c.cpu().numpy(),
           "count": cnt.cpu().numpy().view(np.uint16)}
    if stats:
        out["stats"] = st
    return out
