"""Pins of the oracle's whole-map semantics: the obstructed-region gate
(Def. 2.3), field of view (Sec. III-B), live samples, and symmetries."""
import math

import numpy as np
import pytest

import oracle
from independent import visible_count
from paper_1310_7297_amd import scenes
from paper_1310_7297_amd.scenes import (BILLBOARD, CUBE, FRACTION, FULL, SEGMENT, Grid,
                                         Params, Query, Scene, Target)


def _empty(dim):
    return Scene(dim, np.zeros((3, 0)), np.zeros((3, 0)))


def _samples_independent(t, q):
    """Facet-lattice sample centres, enumerated from the facet definitions."""
    c = np.asarray(t.center, dtype=float)
    out = []
    if t.kind in (SEGMENT, BILLBOARD):
        w = 1 - t.normal_axis
        us = c[w] - t.size[0] / 2 + (np.arange(t.samples_u) + 0.5) * t.size[0] / t.samples_u
        if t.kind == SEGMENT:
            vs = [0.0]
        else:
            vs = c[2] - t.size[1] / 2 + (np.arange(t.samples_v) + 0.5) * t.size[1] / t.samples_v
        for v in vs:
            for u in us:
                p = c.copy()
                p[w] = u
                p[2] = v
                out.append(p)
        return np.array(out)
    E = t.size[0]
    for k in range(3):
        for sgn in (-1, 1):
            plane = c[k] + sgn * E / 2
            if sgn * (q[k] - plane) <= 0:
                continue
            a, b = [x for x in range(3) if x != k]
            for v in c[b] - E / 2 + (np.arange(t.samples_v) + 0.5) * E / t.samples_v:
                for u in c[a] - E / 2 + (np.arange(t.samples_u) + 0.5) * E / t.samples_u:
                    p = np.zeros(3)
                    p[k], p[a], p[b] = plane, u, v
                    out.append(p)
    return np.array(out).reshape(-1, 3)


def test_empty_scene_all_visible():
    s, q = scenes.plain2d_50rects()
    o = oracle.vcm_eval(_empty(2), q)
    assert np.all(o["count"] == 32) and np.all(o["nlive"] == 32)
    pts = oracle.viewpoint_coords(q.grid, np.arange(q.grid.count))
    for i in range(0, q.grid.count, 97):
        m = oracle.measure(q.target, q.params, pts[i])
        assert o["c"][i] == pytest.approx(m["V"] / m["V0"], rel=1e-15)


def test_cube_live_counts():
    t = Target(CUBE, (0.0, 0.0, 15.0), (30.0, 0.0), samples_u=8, samples_v=8)
    assert len(oracle.live_samples(t, (100.0, 100.0, 100.0))) == 192   # three faces
    assert len(oracle.live_samples(t, (0.0, 0.0, 100.0))) == 64        # only the top
    assert len(oracle.live_samples(t, (100.0, 0.0, 15.0))) == 64       # only +x
    assert len(oracle.live_samples(t, (100.0, 100.0, 15.0))) == 128    # +x and +y
    assert len(oracle.live_samples(t, (0.0, 0.0, 15.0))) == 0          # inside
    assert len(oracle.live_samples(t, (15.0, 0.0, 100.0))) == 64       # on the +x plane: not facing
    assert len(oracle.live_samples(t, (15.00390625, 0.0, 100.0))) == 128


def test_fov_wedge():
    """FOV wedge about the target normal, apex at the target centre."""
    t = Target(SEGMENT, (0.0, 0.0, 0.0), (4.0, 0.0), normal_axis=1, normal_sign=1,
               samples_u=4, samples_v=1)
    deg = lambda a, r=100.0: (r * math.sin(math.radians(a)), r * math.cos(math.radians(a)), 0.0)
    # angle from the normal; 120-degree FOV admits up to 60 degrees either side
    for fov, inside, outside in ((120, [0, 30, 59, -59], [61, 90, 180, -61]),
                                 (60, [0, 29, -29], [31, -31, 90]),
                                 (180, [0, 89, -89], [91, 180]),
                                 (240, [0, 119, 180 - 61 + 1], [121, 150, 180]),
                                 (300, [149, -149, 0], [151, 180]),
                                 (360, [0, 90, 180], [])):
        p = Params(fov_deg=fov)
        for a in inside:
            assert oracle.in_fov(t, p, deg(a)), (fov, a)
        for a in outside:
            assert not oracle.in_fov(t, p, deg(a)), (fov, a)
    # closed wedges: viewpoints exactly on the boundary are inside (45 and 135
    # degrees from the normal for FOVs of 90 and 270 degrees), one lattice
    # step further out they are not
    for fov, on, off in ((90, (50.0, 50.0, 0.0), (50.00390625, 50.0, 0.0)),
                         (270, (50.0, -50.0, 0.0), (49.99609375, -50.0, 0.0))):
        assert oracle.in_fov(t, Params(fov_deg=fov), on), fov
        assert not oracle.in_fov(t, Params(fov_deg=fov), off), fov
    # closed at 90 degrees for a 180-degree FOV: points on the target line are inside
    assert oracle.in_fov(t, Params(fov_deg=180), (50.0, 0.0, 0.0))
    assert not oracle.in_fov(t, Params(fov_deg=180), (50.0, -0.00390625, 0.0))
    # the normal sign flips the wedge
    t2 = Target(SEGMENT, (0.0, 0.0, 0.0), (4.0, 0.0), normal_axis=1, normal_sign=-1,
                samples_u=4, samples_v=1)
    assert not oracle.in_fov(t2, Params(fov_deg=120), deg(0))
    assert oracle.in_fov(t2, Params(fov_deg=120), deg(180))


def test_behind_wall_and_inside_box():
    t = Target(BILLBOARD, (0.0, 0.0, 5.0), (8.0, 4.0), normal_axis=1, samples_u=8, samples_v=4)
    wall = Scene(3, np.array([[-50.0], [20.0], [0.0]]), np.array([[50.0], [22.0], [60.0]]))
    g = Grid((-8.0, 40.0, 0.0), (16.0, 16.0, 16.0), (4, 4, 4))   # behind the wall
    o = oracle.vcm_eval(wall, Query(t, g, Params(mode=FRACTION)))
    assert np.all(o["count"] == 0) and np.all(o["c"] == 0.0) and np.all(o["nlive"] == 32)
    g = Grid((-8.0, 20.0, 0.0), (16.0, 2.0, 16.0), (4, 1, 4))    # inside the wall
    o = oracle.vcm_eval(wall, Query(t, g, Params(mode=FRACTION)))
    assert np.all(o["count"] == 0)
    g = Grid((-8.0, -40.0, 0.0), (16.0, 16.0, 16.0), (4, 4, 4))  # in front: clear
    o = oracle.vcm_eval(wall, Query(t, g, Params(mode=FRACTION)))
    assert np.all(o["count"] == 32)


def test_one_blocked_sample_full_vs_fraction():
    """Complete visibility is required (Def. 2.3): one blocked sample zeroes the
    colour in FULL mode; FRACTION mode keeps (N-1)/N of it."""
    t = Target(SEGMENT, (500.0, 500.0, 0.0), (40.0, 0.0), normal_axis=1, samples_u=32, samples_v=1)
    # a tiny box just in front of the first sample (x = 480.625)
    lo = np.array([[480.5], [500.5], [0.0]])
    hi = np.array([[480.75], [500.75], [0.0]])
    sc = Scene(2, lo, hi)
    g = Grid((496.0, 596.0, 0.0), (8.0, 8.0, 0.0), (1, 1, 1))   # viewpoint (500, 600)
    qpt = np.array([500.0, 600.0, 0.0])
    n_vis = visible_count(2, lo, hi, qpt, _samples_independent(t, qpt))
    assert n_vis == 31
    full = oracle.vcm_eval(sc, Query(t, g, Params(mode=FULL)))
    frac = oracle.vcm_eval(sc, Query(t, g, Params(mode=FRACTION)))
    m = oracle.measure(t, Params(), qpt)
    assert full["count"][0] == 0 and full["c"][0] == 0.0
    assert frac["count"][0] == 31
    assert frac["c"][0] == pytest.approx(31 / 32 * m["V"] / m["V0"], rel=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_exhaustive_tiny_scenes_against_independent_counts(seed):
    """<= 8 boxes, all viewpoints of a small grid, lattice-aligned (grazing)."""
    rng = np.random.default_rng(100 + seed)
    dim = 2 if seed % 3 == 0 else 3
    sc = scenes.random_boxes(8, seed, extent=32.0, max_side=8.0, dim=dim, grid_step=2.0)
    if dim == 2:
        t = Target(SEGMENT, (16.0, 16.0, 0.0), (4.0, 0.0), normal_axis=seed % 2, samples_u=8, samples_v=1)
        g = Grid((0.0, 0.0, 0.0), (32.0, 32.0, 0.0), (16, 16, 1))
    elif seed % 3 == 1:
        t = Target(BILLBOARD, (16.0, 16.0, 4.0), (4.0, 2.0), normal_axis=seed % 2, samples_u=4, samples_v=2)
        g = Grid((0.0, 0.0, 0.0), (32.0, 32.0, 16.0), (8, 8, 4))
    else:
        t = Target(CUBE, (16.0, 16.0, 4.0), (4.0, 0.0), samples_u=2, samples_v=2)
        g = Grid((0.0, 0.0, 0.0), (32.0, 32.0, 16.0), (8, 8, 4))
    # drop boxes touching the target
    tlo, thi = t.aabb()
    ov = np.ones(sc.n, bool)
    for k in range(dim):
        ov &= (sc.lo[k] <= thi[k]) & (sc.hi[k] >= tlo[k])
    sc = Scene(dim, sc.lo[:, ~ov], sc.hi[:, ~ov])
    o = oracle.vcm_eval(sc, Query(t, g, Params(mode=FRACTION)))
    pts = oracle.viewpoint_coords(g, np.arange(g.count))
    partial = blocked = clear = 0
    for i, p in enumerate(pts):
        smp = _samples_independent(t, p)
        assert o["nlive"][i] == len(smp)
        n_vis = visible_count(dim, sc.lo, sc.hi, p, smp)
        assert o["count"][i] == n_vis, (i, p)
        partial += 0 < n_vis < len(smp)
        blocked += n_vis == 0 and len(smp) > 0
        clear += n_vis == len(smp) and len(smp) > 0
    assert blocked > 0 and clear > 0 and (partial > 0 or seed >= 4)


def test_mirror_symmetry_plain2d():
    """Mirroring scene, target and grid about x = 500 mirrors the map."""
    s, q = scenes.plain2d_50rects()
    q.params.mode = FRACTION
    o = oracle.vcm_eval(s, q)
    lo = s.lo.copy()
    hi = s.hi.copy()
    lo[0], hi[0] = 1000.0 - s.hi[0], 1000.0 - s.lo[0]
    om = oracle.vcm_eval(Scene(2, lo, hi), q)
    a = o["count"].reshape(64, 64)
    b = om["count"].reshape(64, 64)[:, ::-1]
    assert np.array_equal(a, b)
    assert np.array_equal(o["bin"].reshape(64, 64), om["bin"].reshape(64, 64)[:, ::-1])
    ca = o["c"].reshape(64, 64)
    cb = om["c"].reshape(64, 64)[:, ::-1]
    assert np.allclose(ca, cb, rtol=1e-13, atol=0)


def test_translation_invariance():
    s, q = scenes.plain2d_50rects()
    q.params.mode = FRACTION
    o = oracle.vcm_eval(s, q)
    off = np.array([[1234.5], [-640.25], [0.0]])
    s2 = Scene(2, s.lo + off, s.hi + off)
    t = q.target
    t2 = Target(t.kind, (t.center[0] + 1234.5, t.center[1] - 640.25, 0.0), t.size,
                t.normal_axis, t.normal_sign, t.samples_u, t.samples_v)
    g2 = Grid((1234.5, -640.25, 0.0), q.grid.extent, q.grid.n)
    o2 = oracle.vcm_eval(s2, Query(t2, g2, q.params))
    assert np.array_equal(o["count"], o2["count"])
    assert np.allclose(o["c"], o2["c"], rtol=1e-12, atol=0)


def test_rejects_invalid():
    s, q = scenes.plain2d_50rects()
    q.grid.origin = (0.1, 0.0, 0.0)
    with pytest.raises(ValueError):
        oracle.vcm_eval(s, q)
    s, q = scenes.plain2d_50rects()
    q.params.n_bins = 1
    with pytest.raises(ValueError):
        oracle.vcm_eval(s, q)


def test_rejects_target_meeting_an_obstacle():
    """The target is not an obstacle (Def. 2.1): a box that touches or enters
    the target's box makes the query invalid; one lattice step away is fine."""
    t = Target(BILLBOARD, (0.0, 0.0, 5.0), (8.0, 4.0), normal_axis=1, samples_u=8, samples_v=4)
    g = Grid((-8.0, -40.0, 0.0), (16.0, 16.0, 16.0), (2, 2, 2))
    q = Query(t, g, Params())
    # the billboard spans x in [-4, 4], y = 0, z in [3, 7]
    for lo, hi, bad in (((4.0, -1.0, 0.0), (6.0, 1.0, 9.0), True),          # touches the edge x = 4
                        ((-1.0, 0.0, 0.0), (1.0, 2.0, 3.0), True),          # touches the bottom corner line
                        ((-1.0, -1.0, 4.0), (1.0, 1.0, 5.0), True),         # goes through it
                        ((4.00390625, -1.0, 0.0), (6.0, 1.0, 9.0), False),  # one step beside it
                        ((-1.0, 0.0, 0.0), (1.0, 2.0, 2.99609375), False)):  # one step below
        sc = Scene(3, np.array(lo, dtype=float).reshape(3, 1), np.array(hi, dtype=float).reshape(3, 1))
        if bad:
            with pytest.raises(ValueError):
                oracle.vcm_eval(sc, q)
        else:
            oracle.vcm_eval(sc, q)


def test_fov_gaze_direction():
    """The wedge can turn with a gaze direction instead of the target's normal
    (incremental processing, Sec. IV-C): gaze 0 is the normal itself; a cube
    takes a field of view below 360 degrees only with a gaze."""
    t = Target(BILLBOARD, (0.0, 0.0, 5.0), (8.0, 4.0), normal_axis=1, normal_sign=-1, samples_u=8, samples_v=4)
    rng = np.random.default_rng(7)
    pts = np.round(rng.uniform(-50, 50, size=(300, 3)) * 4) / 4
    for fov in (60.0, 120.0, 180.0, 240.0, 300.0):
        for q in pts:
            assert oracle.in_fov(t, Params(fov_deg=fov), q) == oracle.in_fov(t, Params(fov_deg=fov, gaze=-2), q)
    # gaze +z on a cube: within 60 degrees of straight up
    c = Target(CUBE, (0.0, 0.0, 4.0), (4.0, 0.0), samples_u=2, samples_v=2)
    p = Params(fov_deg=120.0, gaze=3)
    assert oracle.in_fov(c, p, (0.0, 0.0, 40.0)) and oracle.in_fov(c, p, (10.0, 0.0, 24.0))
    assert not oracle.in_fov(c, p, (40.0, 0.0, 4.0)) and not oracle.in_fov(c, p, (0.0, 0.0, -20.0))
    # tan(60 deg) = sqrt(3): the edge of the wedge has no lattice point; just inside and outside
    assert oracle.in_fov(c, p, (17.0, 0.0, 14.0)) and not oracle.in_fov(c, p, (18.0, 0.0, 14.0))
    g = Grid((-16.0, -16.0, 0.0), (32.0, 32.0, 32.0), (4, 4, 4))
    with pytest.raises(ValueError):
        oracle.vcm_eval(Scene(3, np.zeros((3, 0)), np.zeros((3, 0))), Query(c, g, Params(fov_deg=120.0)))
    o = oracle.vcm_eval(Scene(3, np.zeros((3, 0)), np.zeros((3, 0))), Query(c, g, p))
    assert 0 < o["infov"].sum() < g.count
