"""Python access to the exact CPU oracle (oracle/vcm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The library's compute path never imports it.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# VCM_ORACLE_LIB names another build of the same source (the mutation tests
# load copies of the oracle with a planted slip this way).
_LIB_PATH = os.environ.get("VCM_ORACLE_LIB") or os.path.join(_HERE, "libvcm_oracle.so")
_lib = None


class VoTarget(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("normal_axis", ctypes.c_int),
                ("normal_sign", ctypes.c_int), ("su", ctypes.c_int), ("sv", ctypes.c_int),
                ("center", ctypes.c_double * 3), ("size", ctypes.c_double * 2)]


class VoGrid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("extent", ctypes.c_double * 3),
                ("n", ctypes.c_int64 * 3)]


class VoParams(ctypes.Structure):
    _fields_ = [("mu_arcmin", ctypes.c_double), ("d0", ctypes.c_double),
                ("fov_deg", ctypes.c_double), ("n_bins", ctypes.c_int),
                ("bin_scale", ctypes.c_int), ("mode", ctypes.c_int), ("gaze", ctypes.c_int)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.vo_segment_meets_box.argtypes = [ctypes.c_int, dp, dp, dp, dp]
        L.vo_segment_meets_box.restype = ctypes.c_int
        L.vo_live_samples.argtypes = [ctypes.POINTER(VoTarget), dp, dp]
        L.vo_live_samples.restype = ctypes.c_int
        L.vo_measure.argtypes = [ctypes.POINTER(VoTarget), ctypes.POINTER(VoParams), dp, dp]
        L.vo_measure.restype = None
        L.vo_in_fov.argtypes = [ctypes.POINTER(VoTarget), ctypes.POINTER(VoParams), dp]
        L.vo_in_fov.restype = ctypes.c_int
        L.vo_eval.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp,
                              ctypes.POINTER(VoTarget), ctypes.POINTER(VoGrid),
                              ctypes.POINTER(VoParams), ctypes.POINTER(ctypes.c_int64),
                              ctypes.c_int64, ctypes.c_int,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.vo_eval.restype = ctypes.c_int
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec3(x):
    a = np.zeros(3, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).ravel()
    a[: len(x)] = x
    return a


def make_target(t) -> VoTarget:
    T = VoTarget()
    T.kind = int(t.kind)
    T.normal_axis = int(t.normal_axis)
    T.normal_sign = int(t.normal_sign)
    T.su = int(t.samples_u)
    T.sv = int(t.samples_v)
    for k in range(3):
        T.center[k] = float(t.center[k])
    T.size[0] = float(t.size[0])
    T.size[1] = float(t.size[1])
    return T


def make_grid(g) -> VoGrid:
    G = VoGrid()
    for k in range(3):
        G.origin[k] = float(g.origin[k])
        G.extent[k] = float(g.extent[k])
        G.n[k] = int(g.n[k])
    return G


def make_params(p) -> VoParams:
    P = VoParams()
    P.mu_arcmin = float(p.mu_arcmin)
    P.d0 = float(p.near_d0)
    P.fov_deg = float(p.fov_deg)
    P.n_bins = int(p.n_bins)
    P.bin_scale = int(p.bin_scale)
    P.mode = int(p.mode)
    P.gaze = int(getattr(p, "gaze", 0))
    return P


def segment_meets_box(q, s, lo, hi, dim=3) -> int:
    q, s, lo, hi = (_vec3(v) for v in (q, s, lo, hi))
    r = lib().vo_segment_meets_box(int(dim), _dptr(q), _dptr(s), _dptr(lo), _dptr(hi))
    if r < 0:
        raise ValueError("inputs must be multiples of 2^-8 with lo <= hi")
    return r


def live_samples(target, q) -> np.ndarray:
    T = make_target(target)
    q = _vec3(q)
    out = np.zeros((6 * target.samples_u * target.samples_v, 3), dtype=np.float64)
    n = lib().vo_live_samples(ctypes.byref(T), _dptr(q), _dptr(out))
    return out[:n].copy()


def measure(target, params, q) -> Dict[str, float]:
    T, P = make_target(target), make_params(params)
    q = _vec3(q)
    out = np.zeros(4, dtype=np.float64)
    lib().vo_measure(ctypes.byref(T), ctypes.byref(P), _dptr(q), _dptr(out))
    return {"D": out[0], "alpha": out[1], "V": out[2], "V0": out[3]}


def in_fov(target, params, q) -> bool:
    T, P = make_target(target), make_params(params)
    q = _vec3(q)
    return bool(lib().vo_in_fov(ctypes.byref(T), ctypes.byref(P), _dptr(q)))


def vcm_eval(scene, query, vp_index: Optional[np.ndarray] = None, nthreads: int = 1,
             mode: Optional[int] = None) -> Dict[str, np.ndarray]:
    """Oracle VCM at the listed viewpoint indices (default: the whole grid)."""
    g = query.grid
    if vp_index is None:
        vp_index = np.arange(g.count, dtype=np.int64)
    vp = np.ascontiguousarray(vp_index, dtype=np.int64)
    n = len(vp)
    lo = np.ascontiguousarray(scene.lo, dtype=np.float64)
    hi = np.ascontiguousarray(scene.hi, dtype=np.float64)
    T, G, P = make_target(query.target), make_grid(g), make_params(query.params)
    if mode is not None:
        P.mode = int(mode)
    out = {
        "count": np.zeros(n, dtype=np.uint16),
        "nlive": np.zeros(n, dtype=np.uint16),
        "infov": np.zeros(n, dtype=np.uint8),
        "c": np.zeros(n, dtype=np.float64),
        "cb": np.zeros(n, dtype=np.float64),
        "bin": np.zeros(n, dtype=np.uint8),
    }
    r = lib().vo_eval(int(scene.dim), int(scene.n), _dptr(lo), _dptr(hi),
                      ctypes.byref(T), ctypes.byref(G), ctypes.byref(P),
                      vp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n, int(nthreads),
                      out["count"].ctypes.data, out["nlive"].ctypes.data,
                      out["infov"].ctypes.data, out["c"].ctypes.data,
                      out["cb"].ctypes.data, out["bin"].ctypes.data)
    if r != 0:
        raise ValueError("oracle rejected the query (non-dyadic or invalid input)")
    return out


def viewpoint_coords(grid, vp_index) -> np.ndarray:
    """Cell-centred viewpoint coordinates (x fastest), as the oracle forms them."""
    vp = np.asarray(vp_index, dtype=np.int64)
    nx, ny, nz = (int(v) for v in grid.n)
    ii = np.stack([vp % nx, (vp // nx) % ny, vp // (nx * ny)])
    out = np.zeros((len(vp), 3))
    for a in range(3):
        if grid.extent[a] == 0 and grid.n[a] == 1:
            continue
        out[:, a] = grid.origin[a] + (2 * ii[a] + 1) * (grid.extent[a] / (2.0 * grid.n[a]))
    return out


# ------------------------------------------------------------ pruned -------

class VoCells(ctypes.Structure):
    _fields_ = [("nring", ctypes.c_int), ("d", ctypes.POINTER(ctypes.c_double)),
                ("boff", ctypes.POINTER(ctypes.c_int64)), ("gam", ctypes.POINTER(ctypes.c_double)),
                ("S", ctypes.c_double), ("mu", ctypes.c_double), ("d0", ctypes.c_double),
                ("V0", ctypes.c_double), ("rings_only", ctypes.c_int)]


def _plib():
    L = lib()
    if not hasattr(L, "_pruned_ready"):
        L.vo_partition.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.POINTER(VoCells)]
        L.vo_partition.restype = ctypes.c_int
        L.vo_partition_rings.argtypes = L.vo_partition.argtypes
        L.vo_partition_rings.restype = ctypes.c_int
        L.vo_free_cells.argtypes = [ctypes.POINTER(VoCells)]
        L.vo_cells_size.argtypes = [ctypes.POINTER(VoCells), ctypes.POINTER(ctypes.c_int64)]
        L.vo_cells_size.restype = ctypes.c_int
        L.vo_cells_copy.argtypes = [ctypes.POINTER(VoCells), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]
        L.vo_pruned_colours.argtypes = [ctypes.POINTER(VoCells), ctypes.c_double, ctypes.c_double,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.vo_meridian.argtypes = [ctypes.POINTER(VoTarget), ctypes.c_void_p, ctypes.c_void_p]
        L.vo_block_rep.argtypes = [ctypes.POINTER(VoGrid), ctypes.c_int, ctypes.c_int, ctypes.c_int64]
        L.vo_block_rep.restype = ctypes.c_int64
        L.vo_eval_pruned.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.POINTER(VoTarget), ctypes.POINTER(VoGrid),
                                     ctypes.POINTER(VoParams), ctypes.c_int, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]
        L.vo_hull_meets_box.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 5
        L.vo_hull_meets_box.restype = ctypes.c_int
        L.vo_classify_block.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(VoTarget), ctypes.POINTER(VoGrid),
                                        ctypes.POINTER(VoParams), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]
        L.vo_classify_block.restype = ctypes.c_int
        L.vo_eval_pruned.restype = ctypes.c_int
        L.vo_map_error.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_void_p]
        L.vo_error_bounds.argtypes = [ctypes.POINTER(VoCells), ctypes.c_int, ctypes.c_void_p]
        L.vo_bound_measured.argtypes = [ctypes.POINTER(VoCells), ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
        L._pruned_ready = True
    return L


class Cells:
    """Equi-visible cells (rings x bands) of a target of size S."""

    def __init__(self, S: float, mu_rad: float, d0: float, rings_only: bool = False):
        self._c = VoCells()
        part = _plib().vo_partition_rings if rings_only else _plib().vo_partition
        if part(float(S), float(mu_rad), float(d0), ctypes.byref(self._c)):
            raise ValueError("invalid partition parameters")
        nb = ctypes.c_int64()
        nr = _plib().vo_cells_size(ctypes.byref(self._c), ctypes.byref(nb))
        self.d = np.zeros(nr + 1)
        self.boff = np.zeros(nr + 1, dtype=np.int64)
        self.gam = np.zeros(nb.value)
        _plib().vo_cells_copy(ctypes.byref(self._c), self.d.ctypes.data, self.boff.ctypes.data,
                              self.gam.ctypes.data)
        self.S, self.mu, self.d0, self.V0 = self._c.S, self._c.mu, self._c.d0, self._c.V0

    @property
    def nring(self):
        return len(self.d) - 1

    def bands(self, i):
        return self.gam[self.boff[i]:self.boff[i + 1]]

    def colours(self, D: float, alpha: float):
        out = np.zeros(3)
        cell = np.zeros(2, dtype=np.int32)
        tf = ctypes.c_int()
        _plib().vo_pruned_colours(ctypes.byref(self._c), float(D), float(alpha), out.ctypes.data,
                                  cell.ctypes.data, ctypes.addressof(tf))
        return {"E": out[0], "M": out[1], "T": out[2], "ring": int(cell[0]), "band": int(cell[1]),
                "t_fallback": bool(tf.value)}

    def error_bounds(self, dim: int):
        out = np.zeros(2)
        _plib().vo_error_bounds(ctypes.byref(self._c), int(dim), out.ctypes.data)
        return {"mbr": out[0], "tangent": out[1]}

    def bound_measured(self, D, alpha, A: float):
        """Sums of |V_M - V_E| A and |V_T - V_E| A (radians times size) over
        viewpoints with meridian coordinates (D, alpha), each of size A."""
        D = np.ascontiguousarray(D, dtype=np.float64)
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        out = np.zeros(2)
        _plib().vo_bound_measured(ctypes.byref(self._c), len(D), D.ctypes.data, alpha.ctypes.data,
                                  float(A), out.ctypes.data)
        return {"mbr": out[0], "tangent": out[1]}

    def __del__(self):
        try:
            _plib().vo_free_cells(ctypes.byref(self._c))
        except Exception:
            pass


def meridian(target, q):
    T = make_target(target)
    q = _vec3(q)
    out = np.zeros(2)
    _plib().vo_meridian(ctypes.byref(T), q.ctypes.data, out.ctypes.data)
    return out[0], out[1]


def block_rep(grid, dim, theta, idx):
    G = make_grid(grid)
    return int(_plib().vo_block_rep(ctypes.byref(G), int(dim), int(theta), int(idx)))


def vcm_eval_pruned(scene, query, method: int, theta: int = 1,
                    vp_index: Optional[np.ndarray] = None, nthreads: int = 1):
    g = query.grid
    if vp_index is None:
        vp_index = np.arange(g.count, dtype=np.int64)
    vp = np.ascontiguousarray(vp_index, dtype=np.int64)
    n = len(vp)
    lo = np.ascontiguousarray(scene.lo, dtype=np.float64)
    hi = np.ascontiguousarray(scene.hi, dtype=np.float64)
    T, G, P = make_target(query.target), make_grid(g), make_params(query.params)
    out = {"count": np.zeros(n, dtype=np.uint16), "c": np.zeros(n), "cb": np.zeros(n),
           "bin": np.zeros(n, dtype=np.uint8), "cell": np.zeros((n, 2), dtype=np.int32),
           "t_fallback": np.zeros(n, dtype=np.uint8), "decided": np.zeros(n, dtype=np.uint8)}
    r = _plib().vo_eval_pruned(int(scene.dim), int(scene.n), lo.ctypes.data, hi.ctypes.data,
                               ctypes.byref(T), ctypes.byref(G), ctypes.byref(P), int(method),
                               int(theta), vp.ctypes.data, n, int(nthreads),
                               out["count"].ctypes.data, out["c"].ctypes.data,
                               out["cb"].ctypes.data, out["bin"].ctypes.data,
                               out["cell"].ctypes.data, out["t_fallback"].ctypes.data,
                               out["decided"].ctypes.data)
    if r != 0:
        raise ValueError("oracle rejected the pruned query")
    return out


def map_error(c_exact, c_approx):
    ce = np.ascontiguousarray(c_exact, dtype=np.float64)
    ca = np.ascontiguousarray(c_approx, dtype=np.float64)
    s, a = ctypes.c_double(), ctypes.c_double()
    _plib().vo_map_error(ce.ctypes.data, ca.ctypes.data, len(ce), ctypes.addressof(s),
                         ctypes.addressof(a))
    return s.value, a.value


# ------------------------------------------------------------ blocks -------

def hull_meets_box(L, H, s, a, c, dim=3) -> bool:
    """Does the closed box [a, c] meet the convex hull of the box [L, H] and
    the point s?"""
    L, H, s, a, c = (_vec3(v) for v in (L, H, s, a, c))
    r = _plib().vo_hull_meets_box(int(dim), L.ctypes.data, H.ctypes.data, s.ctypes.data,
                                  a.ctypes.data, c.ctypes.data)
    if r < 0:
        raise ValueError("inputs must be multiples of 2^-8 with lo <= hi")
    return bool(r)


def classify_block(scene, query, lo_idx, hi_idx):
    """Whole-block classification of the viewpoints with grid indices
    lo_idx .. hi_idx (inclusive): None if undecided, else (count, N, in_fov)
    shared by every viewpoint of the block."""
    lo = np.ascontiguousarray(scene.lo, dtype=np.float64)
    hi = np.ascontiguousarray(scene.hi, dtype=np.float64)
    T, G, P = make_target(query.target), make_grid(query.grid), make_params(query.params)
    il = np.zeros(3, dtype=np.int64)
    ih = np.zeros(3, dtype=np.int64)
    il[:len(lo_idx)] = lo_idx
    ih[:len(hi_idx)] = hi_idx
    out = np.zeros(3, dtype=np.int32)
    r = _plib().vo_classify_block(int(scene.dim), int(scene.n), lo.ctypes.data, hi.ctypes.data,
                                  ctypes.byref(T), ctypes.byref(G), ctypes.byref(P), il.ctypes.data,
                                  ih.ctypes.data, out.ctypes.data)
    if r < 0:
        raise ValueError("invalid block or query")
    return (int(out[0]), int(out[1]), int(out[2])) if r else None
