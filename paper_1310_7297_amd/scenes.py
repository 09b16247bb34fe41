"""Seeded synthetic inputs: obstacle cities, targets, viewpoint grids, parameters.

This module only draws random numbers and quantizes them; it holds none of the
visibility arithmetic.  Both the HIP path and the CPU oracle consume its output.

Every coordinate it emits is a multiple of 2**-8 with magnitude below 2**14, so
the values, and every difference of two of them, are exact in float32.

The paper's experiments use two proprietary city models normalised to a
10,000 x 10,000 space (Sec. V-A); they are not available, so axis-aligned box
cities drawn here stand in for them, with the shapes and densities of the
workloads this library is measured on.  The parameter defaults follow the
paper's parameter table (Table 2): angular resolution 4 arcmin, minimum block
size 1, field of view 120 degrees.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

QUANTUM = 1.0 / 256.0
COORD_LIMIT = float(2 ** 14)

# Target kinds (match the C-ABI enum values).  VIEWER: the viewer of a
# viewer-centric map, size[0] = the radius d_max of the region it covers.
SEGMENT = 0
BILLBOARD = 1
CUBE = 2
VIEWER = 3

# Modes, methods, bin scales (match the C-ABI enum values).
FULL = 0
FRACTION = 1
BRUTE = 0
PRUNED_E = 1
PRUNED_M = 2
PRUNED_T = 3
BIN_LINEAR = 0
BIN_LOG = 1

# Lognormal building heights with mean 30 m and standard deviation 15 m.
_H_MEAN, _H_SD = 30.0, 15.0
_SIGMA_LN = math.sqrt(math.log(1.0 + (_H_SD / _H_MEAN) ** 2))
_MU_LN = math.log(_H_MEAN) - 0.5 * _SIGMA_LN ** 2


def quantize(x):
    """Round to the nearest multiple of 2**-8 (ties to even)."""
    return np.round(np.asarray(x, dtype=np.float64) * 256.0) / 256.0


@dataclasses.dataclass
class Scene:
    dim: int
    lo: np.ndarray  # (3, n) float64
    hi: np.ndarray  # (3, n) float64

    @property
    def n(self) -> int:
        return int(self.lo.shape[1])

    def sha(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.dim).tobytes())
        h.update(np.ascontiguousarray(self.lo).tobytes())
        h.update(np.ascontiguousarray(self.hi).tobytes())
        return h.hexdigest()


@dataclasses.dataclass
class Target:
    kind: int
    center: Tuple[float, float, float]
    size: Tuple[float, float]          # segment: (length, 0); billboard: (width, height); cube: (edge, 0)
    normal_axis: int = 1               # segment/billboard only
    normal_sign: int = 1
    samples_u: int = 8
    samples_v: int = 8

    def aabb(self):
        c = np.asarray(self.center, dtype=np.float64)
        lo = c.copy()
        hi = c.copy()
        if self.kind == VIEWER:
            return lo, hi
        if self.kind == CUBE:
            e = self.size[0] / 2.0
            return c - e, c + e
        if self.kind == SEGMENT:
            ax = 1 - self.normal_axis
            lo[ax] -= self.size[0] / 2.0
            hi[ax] += self.size[0] / 2.0
            return lo, hi
        ax = 1 - self.normal_axis
        lo[ax] -= self.size[0] / 2.0
        hi[ax] += self.size[0] / 2.0
        lo[2] -= self.size[1] / 2.0
        hi[2] += self.size[1] / 2.0
        return lo, hi


@dataclasses.dataclass
class Grid:
    origin: Tuple[float, float, float]
    extent: Tuple[float, float, float]
    n: Tuple[int, int, int]

    @property
    def count(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


@dataclasses.dataclass
class Params:
    mu_arcmin: float = 4.0
    near_d0: float = 0.25
    fov_deg: float = 360.0
    n_bins: int = 16
    bin_scale: int = BIN_LINEAR
    method: int = BRUTE
    mode: int = FULL
    theta_blocks: int = 1
    recheck_eps: float = 2.0 ** -20
    gaze: int = 0              # field-of-view axis: 0 = the target's normal, +-(1 + k) = +-axis k


@dataclasses.dataclass
class Query:
    target: Target
    grid: Grid
    params: Params


# ---------------------------------------------------------------- cities ----

def _drop_near_target(lo, hi, targets: Sequence[Target], clearance: float):
    keep = np.ones(lo.shape[1], dtype=bool)
    for t in targets:
        tlo, thi = t.aabb()
        tlo = tlo - clearance
        thi = thi + clearance
        ov = np.ones_like(keep)
        for k in range(3):
            ov &= (lo[k] <= thi[k]) & (hi[k] >= tlo[k])
        keep &= ~ov
    return lo[:, keep].copy(), hi[:, keep].copy()


def city(extent: float, n_boxes: int, seed: int, side=(20.0, 80.0),
         targets: Sequence[Target] = (), clearance: float = 5.0) -> Scene:
    """Axis-aligned box city on the ground plane.

    Per box, in this order: centre x, centre y, footprint width, footprint
    depth (all uniform), then a lognormal height with mean 30 m and sd 15 m.
    Overlap is allowed.  Boxes within `clearance` of any target are dropped.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((n_boxes, 4))
    z = rng.standard_normal(n_boxes)
    cx = quantize(u[:, 0] * extent)
    cy = quantize(u[:, 1] * extent)
    w = quantize(side[0] + u[:, 2] * (side[1] - side[0]))
    d = quantize(side[0] + u[:, 3] * (side[1] - side[0]))
    h = quantize(np.exp(_MU_LN + _SIGMA_LN * z))
    h = np.maximum(h, QUANTUM)
    lo = np.stack([quantize(cx - w / 2), quantize(cy - d / 2), np.zeros(n_boxes)])
    hi = np.stack([quantize(cx + w / 2), quantize(cy + d / 2), h])
    lo, hi = _drop_near_target(lo, hi, targets, clearance)
    return Scene(3, lo, hi)


def city_zipf(extent: float, n_boxes: int, seed: int, side=(20.0, 80.0), districts: int = 32,
              s: float = 1.0, targets: Sequence[Target] = (), clearance: float = 5.0) -> Scene:
    """Box city whose density follows a Zipf law over districts: the space is
    cut into districts x districts squares, ranked in a seeded random order,
    and each box falls in the district of rank r with probability
    proportional to 1 / r**s, uniformly inside it.  Per box, in this order:
    district, offset x, offset y, width, depth, then the lognormal height (as
    in `city`).  Boxes within `clearance` of any target are dropped."""
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(districts * districts)
    w_rank = 1.0 / np.arange(1, districts * districts + 1, dtype=np.float64) ** s
    prob = np.empty_like(w_rank)
    prob[order] = w_rank / w_rank.sum()
    d = rng.choice(districts * districts, size=n_boxes, p=prob)
    u = rng.random((n_boxes, 4))
    z = rng.standard_normal(n_boxes)
    step = extent / districts
    cx = quantize((d % districts + u[:, 0]) * step)
    cy = quantize((d // districts + u[:, 1]) * step)
    w = quantize(side[0] + u[:, 2] * (side[1] - side[0]))
    dd = quantize(side[0] + u[:, 3] * (side[1] - side[0]))
    h = np.maximum(quantize(np.exp(_MU_LN + _SIGMA_LN * z)), QUANTUM)
    lo = np.stack([quantize(cx - w / 2), quantize(cy - dd / 2), np.zeros(n_boxes)])
    hi = np.stack([quantize(cx + w / 2), quantize(cy + dd / 2), h])
    lo, hi = _drop_near_target(lo, hi, targets, clearance)
    return Scene(3, lo, hi)


def sweep_billboard(n_boxes: int = 20000, dist: str = "uniform", seed: int = 3):
    """Workload of the parameter sweeps (Table 2's parameters on a 3-D city):
    a 4 km city of `n_boxes` boxes (uniform or Zipf-clustered), a 30 m x 15 m
    billboard facing +y at the centre, 256 x 256 x 64 viewpoints over
    0-150 m, field of view 120 degrees (the paper's default), 16 bins."""
    t = Target(BILLBOARD, (2000.0, 2000.0, 10.0), (30.0, 15.0), normal_axis=1, normal_sign=1,
               samples_u=16, samples_v=8)
    if dist == "uniform":
        scene = city(4000.0, n_boxes, seed=seed, targets=[t])
    else:
        scene = city_zipf(4000.0, n_boxes, seed=seed, targets=[t])
    g = Grid((0.0, 0.0, 0.0), (4000.0, 4000.0, 150.0), (256, 256, 64))
    return scene, Query(t, g, Params(n_bins=16, fov_deg=120.0))


def plain_2d(extent: float, n_rects: int, seed: int, side=(10.0, 50.0),
             targets: Sequence[Target] = (), clearance: float = 5.0,
             max_tries: int = 100000) -> Scene:
    """Non-overlapping, non-touching rectangles, rejection-sampled in order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rects: List[Tuple[float, float, float, float]] = []
    forbid = []
    for t in targets:
        tlo, thi = t.aabb()
        forbid.append((tlo[0] - clearance, tlo[1] - clearance,
                       thi[0] + clearance, thi[1] + clearance))
    tries = 0
    while len(rects) < n_rects:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("rejection sampling did not converge")
        u = rng.random(4)
        cx = float(quantize(u[0] * extent))
        cy = float(quantize(u[1] * extent))
        w = float(quantize(side[0] + u[2] * (side[1] - side[0])))
        d = float(quantize(side[0] + u[3] * (side[1] - side[0])))
        r = (float(quantize(cx - w / 2)), float(quantize(cy - d / 2)),
             float(quantize(cx + w / 2)), float(quantize(cy + d / 2)))
        bad = False
        for o in rects + forbid:
            if r[0] <= o[2] and o[0] <= r[2] and r[1] <= o[3] and o[1] <= r[3]:
                bad = True
                break
        if not bad:
            rects.append(r)
    a = np.asarray(rects, dtype=np.float64).reshape(-1, 4)
    lo = np.stack([a[:, 0], a[:, 1], np.zeros(len(a))])
    hi = np.stack([a[:, 2], a[:, 3], np.zeros(len(a))])
    return Scene(2, lo, hi)


def random_boxes(n: int, seed: int, extent=64.0, max_side=16.0, dim=3,
                 grid_step: float = 1.0) -> Scene:
    """Small boxes on a coarse lattice (many coincident faces: grazing-heavy)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    steps = int(extent / grid_step)
    lo = np.zeros((3, n))
    hi = np.zeros((3, n))
    for k in range(dim):
        a = rng.integers(0, steps, n) * grid_step
        s = rng.integers(0, int(max_side / grid_step) + 1, n) * grid_step
        lo[k] = a
        hi[k] = np.minimum(a + s, extent)
    return Scene(dim, quantize(lo), quantize(hi))


# -------------------------------------------------------------- workloads ---

def plain2d_50rects():
    """2-D plain: 1000 x 1000, 50 rectangles, segment target, 64 x 64 grid."""
    t = Target(SEGMENT, (500.0, 500.0, 0.0), (40.0, 0.0), normal_axis=1,
               normal_sign=1, samples_u=32, samples_v=1)
    scene = plain_2d(1000.0, 50, seed=1, targets=[t])
    g = Grid((0.0, 0.0, 0.0), (1000.0, 1000.0, 0.0), (64, 64, 1))
    p = Params(n_bins=8, fov_deg=360.0)
    return scene, Query(t, g, p)


def city2km_billboard():
    """3-D plain: 2 km city, 5,000 boxes, 10 x 5 m billboard, 128x128x32."""
    t = Target(BILLBOARD, (1000.0, 1000.0, 12.5), (10.0, 5.0), normal_axis=1,
               normal_sign=1, samples_u=16, samples_v=8)
    scene = city(2000.0, 5000, seed=2, targets=[t])
    g = Grid((0.0, 0.0, 0.0), (2000.0, 2000.0, 150.0), (128, 128, 32))
    p = Params(n_bins=16, fov_deg=360.0)
    return scene, Query(t, g, p)


def city4km_cube():
    """3-D pruned vs brute: 4 km city, 20,000 boxes, 30 m cube, 256x256x64."""
    t = Target(CUBE, (2000.0, 2000.0, 15.0), (30.0, 0.0), samples_u=8, samples_v=8)
    scene = city(4000.0, 20000, seed=3, targets=[t])
    g = Grid((0.0, 0.0, 0.0), (4000.0, 4000.0, 150.0), (256, 256, 64))
    p = Params(n_bins=16, fov_deg=360.0)
    return scene, Query(t, g, p)


def _batch_targets(rng, n, city_extent, window):
    queries = []
    grids_xy = (32, 64, 128, 256)
    grids_z = (16, 32, 64)
    for _ in range(n):
        u = rng.random(8)
        size = float(np.round((5.0 + 35.0 * u[1]) * 8.0) / 8.0)
        cx = float(quantize(size + u[2] * (city_extent - 2 * size)))
        cy = float(quantize(size + u[3] * (city_extent - 2 * size)))
        if u[0] < 0.5:
            axis = 0 if u[4] < 0.5 else 1
            sign = 1 if u[5] < 0.5 else -1
            t = Target(BILLBOARD, (cx, cy, float(quantize(10.0 + size / 4.0))),
                       (size, size / 2.0), normal_axis=axis, normal_sign=sign,
                       samples_u=16, samples_v=8)
        else:
            t = Target(CUBE, (cx, cy, size / 2.0), (size, 0.0), samples_u=8, samples_v=8)
        nxy = grids_xy[min(3, int(u[6] * 4))]
        nz = grids_z[min(2, int(u[7] * 3))]
        ox = min(max(cx - window / 2.0, 0.0), city_extent - window)
        oy = min(max(cy - window / 2.0, 0.0), city_extent - window)
        g = Grid((float(quantize(ox)), float(quantize(oy)), 0.0), (window, window, 150.0),
                 (nxy, nxy, nz))
        queries.append(Query(t, g, Params(n_bins=16, fov_deg=360.0)))
    return queries


def city6km_batch256(n_targets: int = 256):
    """Batched: 50,000-box 6.4 km city shared by 256 targets of mixed kind and size."""
    rng = np.random.Generator(np.random.PCG64(4))
    queries = _batch_targets(rng, n_targets, 6400.0, 2560.0)
    scene = city(6400.0, 50000, seed=4, targets=[q.target for q in queries])
    return scene, queries


def city8km_serving(n_requests: int = 2000):
    """Serving: 100,000-box 8 km city; queries with grids 64^2x16/128^2x32/256^2x64."""
    rng = np.random.Generator(np.random.PCG64(55))
    queries = _batch_targets(rng, n_requests, 8000.0, 3072.0)
    w = rng.random(n_requests)
    for q, x in zip(queries, w):
        if x < 0.6:
            q.grid.n = (64, 64, 16)
        elif x < 0.9:
            q.grid.n = (128, 128, 32)
        else:
            q.grid.n = (256, 256, 64)
    scene = city(8000.0, 100000, seed=5, targets=[q.target for q in queries])
    return scene, queries


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, n))


def viewpoint_sample(grid: Grid, k: int, seed: int) -> np.ndarray:
    """Seeded sorted sample of k distinct viewpoint indices (x fastest)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = grid.count
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
