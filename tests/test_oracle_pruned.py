"""Pins of the oracle's pruned construction: equi-visible cells (Sec. III-A),
MBR and tangential approximations (Sec. IV-A), error metric (Sec. V-A)."""
import math

import numpy as np
import pytest

import oracle
from paper_1310_7297_amd import scenes
from paper_1310_7297_amd.scenes import (BILLBOARD, CUBE, FRACTION, FULL, SEGMENT, Grid, Params,
                                         Query, Scene, Target)

MU = 4.0 / 60.0 * math.pi / 180.0


def V(S, D, alpha=math.pi / 2):
    return 2 * math.atan((alpha / (math.pi / 2)) * S / (2 * D))


@pytest.fixture(scope="module")
def cells30():
    return oracle.Cells(30.0, MU, 0.25)


def test_rings_step_the_facing_angle_by_mu(cells30):
    """Sec. III-A-1: consecutive ring boundaries differ by mu in visual angle
    at the facing angle, starting at the near point, ending where V = mu."""
    c = cells30
    assert c.d[0] == 0.25
    for i in range(c.nring):
        assert abs(V(30.0, c.d[i]) - (c.V0 - i * MU)) < 1e-12
    # last boundary: the distance at which the target subtends mu (Sec. IV-B)
    assert abs(V(30.0, c.d[-1]) - MU) < 1e-15
    assert abs(c.d[-1] - 30.0 / (2 * math.tan(MU / 2))) < 1e-6
    assert np.all(np.diff(c.d) > 0)
    # the last full step still has V >= mu, one more would not
    K = c.nring - 1
    assert c.V0 - K * MU >= MU > c.V0 - (K + 1) * MU


def test_bands_step_the_angle_by_mu_at_mid_distance(cells30):
    """Sec. III-A-2: within a ring, band boundaries are the viewing angles at
    which the visual angle at the ring's middle distance drops by mu."""
    c = cells30
    for i in (0, 1, 10, 500, 1500, c.nring - 2, c.nring - 1):
        g = c.bands(i)
        dp = 0.5 * (c.d[i] + c.d[i + 1])
        W0 = V(30.0, dp)
        assert g[0] == math.pi / 2 and g[-1] == 0.0
        assert np.all(np.diff(g) < 0)
        for j in range(1, len(g) - 1):
            assert abs(V(30.0, dp, g[j]) - (W0 - j * MU)) < 1e-10
        # the last interior boundary keeps W >= mu
        L = len(g) - 2
        assert W0 - L * MU >= MU > W0 - (L + 1) * MU


def test_cell_colour_is_within_mu_far_from_the_target(cells30):
    """Eq. 3 requires points of a cell to look alike within mu.  The cell's
    centre colour stays within 1.5 mu of every point of the cell once the
    viewpoint is at least S/4 away (near the target at oblique angles the
    paper's rings, computed facing the target, are too wide for that)."""
    c = cells30
    rng = np.random.default_rng(3)
    worst = 0.0
    for _ in range(1500):
        D = math.exp(rng.uniform(math.log(7.5), math.log(c.d[-1] * 0.999)))
        a = rng.uniform(0, math.pi / 2)
        r = c.colours(D, a)
        worst = max(worst, abs(r["E"] * c.V0 - V(30.0, D, a)) / MU)
    assert worst <= 1.5, worst


def test_own_cell_lookup(cells30):
    c = cells30
    rng = np.random.default_rng(4)
    for _ in range(300):
        D = math.exp(rng.uniform(math.log(0.3), math.log(c.d[-1] * 0.99)))
        a = rng.uniform(0, math.pi / 2)
        r = c.colours(D, a)
        i, j = r["ring"], r["band"]
        assert c.d[i] <= D < c.d[i + 1]
        g = c.bands(i)
        assert g[j + 1] < a <= g[j] or (a <= g[j] and j == len(g) - 2)
    assert c.colours(c.d[-1] * 1.001, 0.5)["E"] == 0.0


def test_mbr_contains_its_cell_and_m_tracks_e(cells30):
    """Every MBR contains its cell, so VCM_M finds a cell for every viewpoint;
    as mu shrinks the approximations approach the exact colours."""
    c = cells30
    rng = np.random.default_rng(5)
    for _ in range(200):
        i = int(rng.integers(0, c.nring))
        g = c.bands(i)
        j = int(rng.integers(0, len(g) - 1))
        d = rng.uniform(c.d[i], c.d[i + 1])
        a = rng.uniform(g[j + 1], g[j])
        rho, h = d * math.cos(a), d * math.sin(a)
        assert c.d[i] * math.cos(g[j]) <= rho + 1e-9 <= c.d[i + 1] * math.cos(g[j + 1]) + 2e-9
        assert c.d[i] * math.sin(g[j + 1]) <= h + 1e-9 <= c.d[i + 1] * math.sin(g[j]) + 2e-9
    diffs = []
    for mu_arc in (16.0, 4.0, 1.0):
        cc = oracle.Cells(12.0, mu_arc / 60 * math.pi / 180, 0.25)
        rng = np.random.default_rng(6)
        tot_m = tot_t = 0.0
        for _ in range(300):
            D = math.exp(rng.uniform(math.log(3.0), math.log(2000.0)))
            a = rng.uniform(0, math.pi / 2)
            r = cc.colours(D, a)
            tot_m += abs(r["M"] - r["E"])
            tot_t += abs(r["T"] - r["E"])
        diffs.append((tot_m, tot_t))
    assert diffs[0][0] > diffs[1][0] > diffs[2][0]
    assert diffs[0][1] >= diffs[1][1] >= diffs[2][1]


def test_colours_symmetric_in_quadrants():
    """The partition is computed for the first quadrant and reflected
    (Sec. III-A-2): mirrored viewpoints get the same colours."""
    t = Target(SEGMENT, (0.0, 0.0, 0.0), (12.0, 0.0), normal_axis=1, samples_u=4, samples_v=1)
    c = oracle.Cells(12.0, MU, 0.25)
    for q in ((30.0, 40.0), (3.0, 70.0), (200.0, 5.0)):
        outs = []
        for sx in (1, -1):
            for sy in (1, -1):
                D, a = oracle.meridian(t, (sx * q[0], sy * q[1], 0.0))
                outs.append(c.colours(D, a))
        for k in ("E", "M", "T"):
            assert len({o[k] for o in outs}) == 1


def test_error_metric():
    ce = np.array([0.5, 0.25, 0.0, 0.25])
    assert oracle.map_error(ce, ce) == (0.0, 0.0)
    s, a = oracle.map_error(ce, np.zeros(4))
    assert s == 1.0 and a == 1.0
    s, a = oracle.map_error(ce, ce * 0.9)
    assert abs(s - 0.1) < 1e-15 and abs(a - 0.1) < 1e-15
    s, a = oracle.map_error(ce, np.array([0.6, 0.15, 0.0, 0.25]))
    assert abs(s - 0.0) < 1e-15 and abs(a - 0.2) < 1e-15


def test_error_bounds_order(cells30):
    """The MBR's far corner is farther than the tangent rectangle's, and it
    counts bands up to a wider angle, so its bound is the larger."""
    b2 = cells30.error_bounds(2)
    b3 = cells30.error_bounds(3)
    for b in (b2, b3):
        assert 0 < b["tangent"] < b["mbr"] < math.inf


def test_block_representative():
    """Smallest blocks have the largest power-of-two side not above theta
    (blocks are halved), are aligned, are cut by the grid's end, and are
    represented by their lowest-index centre viewpoint."""
    g = Grid((0.0, 0.0, 0.0), (10.0, 10.0, 10.0), (5, 5, 5))
    idx = lambda i, j, k: i + 5 * (j + 5 * k)
    for i in range(5):
        assert oracle.block_rep(g, 3, 1, idx(i, 2, 3)) == idx(i, 2, 3)
    assert oracle.block_rep(g, 3, 2, idx(1, 2, 3)) == idx(0, 2, 2)
    assert oracle.block_rep(g, 3, 3, idx(1, 2, 3)) == idx(0, 2, 2)   # side 2
    assert oracle.block_rep(g, 3, 4, idx(4, 4, 4)) == idx(4, 4, 4)   # ragged block
    assert oracle.block_rep(g, 3, 4, idx(3, 0, 2)) == idx(1, 1, 1)
    assert oracle.block_rep(g, 3, 7, idx(3, 0, 2)) == idx(1, 1, 1)   # side 4


def test_pruned_gate_equals_brute_at_theta_one():
    scene, q = scenes.plain2d_50rects()
    for mode in (FULL, FRACTION):
        q.params.mode = mode
        b = oracle.vcm_eval(scene, q, nthreads=8)
        for m in (1, 2, 3):
            p = oracle.vcm_eval_pruned(scene, q, m, 1, nthreads=8)
            assert np.array_equal(p["count"], b["count"])
            assert np.all((p["c"] > 0) == (b["c"] > 0))


# ---------------------------------------------------------------------------
# Selection rules of VCM_M and VCM_T and the cell colour, checked on tiny
# partitions (large mu, so that rings are few and wide and the approximated
# cells overlap a lot) against the geometry of the cells themselves.

TINY = [(10.0, 5.0), (4.0, 3.0), (10.0, 12.0), (30.0, 2.0)]   # (S in m, mu in degrees)


def _tiny(S, mu_deg):
    return oracle.Cells(S, math.radians(mu_deg), 0.25)


def _centre_colour(c, i, j):
    """Visual angle (Eq. 1 with the oblique size of Eq. 2) at the centre of
    cell (i, j) in parameter space -- the middle distance of the ring and the
    middle angle of the band -- over V0."""
    g = c.bands(i)
    return V(c.S, 0.5 * (c.d[i] + c.d[i + 1]), 0.5 * (g[j] + g[j + 1])) / c.V0


def _sector_mbr(r0, r1, g_lo, g_hi, n=257):
    """Bounding box, in the (rho, h) quadrant, of the annular sector
    {r in [r0, r1], angle in [g_lo, g_hi]}, from points of its boundary (the
    arcs and the two radial edges, their end points included)."""
    ang = np.linspace(g_lo, g_hi, n)
    rr = np.linspace(r0, r1, n)
    xs = np.concatenate([r0 * np.cos(ang), r1 * np.cos(ang), rr * math.cos(g_lo), rr * math.cos(g_hi)])
    ys = np.concatenate([r0 * np.sin(ang), r1 * np.sin(ang), rr * math.sin(g_lo), rr * math.sin(g_hi)])
    return xs.min(), xs.max(), ys.min(), ys.max()


def _trapezoid(r0, r1, g_lo, g_hi):
    """Corners, counter-clockwise, of the quadrilateral bounded by the band's
    two radial edges and the tangents of the arcs r0 and r1 at the band's
    middle angle."""
    gm = 0.5 * (g_lo + g_hi)
    out = []
    for r, gs in ((r0, (g_hi, g_lo)), (r1, (g_lo, g_hi))):
        for g in gs:
            L = r / math.cos(g - gm)   # where the tangent line meets the edge ray
            out.append((L * math.cos(g), L * math.sin(g)))
    return out


def _points(c, n, seed):
    rng = np.random.default_rng(seed)
    D = np.exp(rng.uniform(math.log(0.3), math.log(c.d[-1] * 0.999), n))
    a = rng.uniform(0.0, math.pi / 2, n)
    return D, a


@pytest.mark.parametrize("S,mu_deg", TINY)
def test_m_takes_the_lowest_cell_whose_mbr_holds_q(S, mu_deg):
    """VCM_M (Sec. IV-A, MBR approximation): the colour of the first cell, in
    (ring, band) order, whose bounding box holds q; the boxes here come from
    points of the cells' boundaries, not from a closed form."""
    c = _tiny(S, mu_deg)
    cells = []
    for i in range(c.nring):
        g = c.bands(i)
        for j in range(len(g) - 1):
            cells.append((i, j, _sector_mbr(c.d[i], c.d[i + 1], g[j + 1], g[j])))
    D, a = _points(c, 2500, int(S * 100 + mu_deg))
    checked = other = 0
    for Dk, ak in zip(D, a):
        rho, h = Dk * math.cos(ak), Dk * math.sin(ak)
        eps = 1e-9 * Dk
        strict = [(i, j) for i, j, (x0, x1, y0, y1) in cells
                  if x0 + eps <= rho <= x1 - eps and y0 + eps <= h <= y1 - eps]
        loose = [(i, j) for i, j, (x0, x1, y0, y1) in cells
                 if x0 - eps <= rho <= x1 + eps and y0 - eps <= h <= y1 + eps]
        if not strict or strict[0] != loose[0]:
            continue   # within rounding of some box's edge: either answer is right
        i, j = strict[0]
        r = c.colours(Dk, ak)
        assert r["M"] == pytest.approx(_centre_colour(c, i, j), rel=1e-12, abs=1e-15), (Dk, ak)
        checked += 1
        other += (i, j) != (r["ring"], r["band"])
    assert checked > 2000
    assert other > 100, "too few viewpoints take another cell's colour to exercise the rule"


@pytest.mark.parametrize("S,mu_deg", TINY)
def test_t_takes_the_lowest_ring_whose_tangent_trapezoid_holds_q(S, mu_deg):
    """VCM_T (Sec. IV-A, tangential approximation): the colour of the first
    ring whose cell, cut by the tangents of its arcs at the middle of the
    band, holds q; the quadrilaterals here are built from their corners and
    tested with a generic point-in-convex-polygon rule.  No quadrilateral
    holds q: q's own cell."""
    c = _tiny(S, mu_deg)
    order, polys = [], []
    for i in range(c.nring):
        g = c.bands(i)
        for j in range(len(g) - 1):
            order.append((i, j))
            polys.append(_trapezoid(c.d[i], c.d[i + 1], g[j + 1], g[j]))
    P = np.array(polys)                      # (cells, 4 corners, 2)
    E0 = P                                   # edge starts
    E1 = np.roll(P, -1, axis=1)              # edge ends
    ex, ey = E1[..., 0] - E0[..., 0], E1[..., 1] - E0[..., 1]
    el = np.hypot(ex, ey)
    D, a = _points(c, 2500, int(S * 10 + mu_deg))
    checked = other = 0
    for Dk, ak in zip(D, a):
        x, y = Dk * math.cos(ak), Dk * math.sin(ak)
        side = (ex * (y - E0[..., 1]) - ey * (x - E0[..., 0])) / el   # left of every edge: inside
        slack = 1e-9 * Dk
        inside = np.all(side >= -slack, axis=1)
        near = inside & np.any(np.abs(side) <= slack, axis=1)
        hits = np.nonzero(inside)[0]
        if len(hits) and near[hits[0]]:
            continue   # within rounding of the first candidate's edge
        r = c.colours(Dk, ak)
        if len(hits) == 0:
            assert r["t_fallback"] and r["T"] == r["E"]
        else:
            hit = order[hits[0]]
            assert not r["t_fallback"]
            assert r["T"] == pytest.approx(_centre_colour(c, *hit), rel=1e-12, abs=1e-15), (Dk, ak)
            other += hit != (r["ring"], r["band"])
        checked += 1
    assert checked > 2000 and other > 20


def test_t_single_band_rings_project_on_the_diagonal():
    """A ring whose visual angle at its middle distance is below 2 mu has one
    band, from 90 degrees down to 0; its tangents touch the arcs at 45
    degrees, so the ring holds q under VCM_T exactly when the projection of q
    on the diagonal, D cos(alpha - 45 deg), lies in the ring."""
    c = _tiny(10.0, 12.0)
    single = [i for i in range(c.nring) if len(c.bands(i)) == 2]
    assert single
    i = single[-1]
    rng = np.random.default_rng(9)
    n = 0
    for _ in range(400):
        a = rng.uniform(0.02, math.pi / 2 - 0.02)
        p = rng.uniform(c.d[i] * 1.001, c.d[i + 1] * 0.999)
        D = p / math.cos(a - math.pi / 4)
        if D >= c.d[-1]:
            continue
        r = c.colours(D, a)
        # lower rings cannot hold q: their trapezoids end below d_i in every direction
        assert r["T"] == pytest.approx(_centre_colour(c, i, 0), rel=1e-12)
        n += 1
    assert n > 200


@pytest.mark.parametrize("S,mu_deg", [(30.0, 4.0 / 60.0)] + TINY)
def test_cell_colour_is_the_visual_angle_at_the_parameter_midpoint(S, mu_deg):
    """A cell's colour is the visibility at its centre (Sec. III-A): here the
    middle of the ring's distances and of the band's angles, through Eq. 1
    and Eq. 2 (a colour taken at d_i, d_{i+1}, gamma_j or gamma_{j+1}
    differs by at least one mu step)."""
    c = _tiny(S, mu_deg)
    rng = np.random.default_rng(int(S + 10 * mu_deg))
    for _ in range(400):
        i = int(rng.integers(0, c.nring))
        g = c.bands(i)
        j = int(rng.integers(0, len(g) - 1))
        D = rng.uniform(c.d[i], c.d[i + 1]) if i > 0 else rng.uniform(0.01, c.d[1])
        a = rng.uniform(g[j + 1], g[j])
        r = c.colours(D, a)
        if (r["ring"], r["band"]) != (i, j):
            continue   # on a boundary after rounding
        assert r["E"] == pytest.approx(_centre_colour(c, i, j), rel=1e-13)


@pytest.mark.parametrize("dim,S,mu_deg", [(2, 10.0, 5.0), (2, 4.0, 3.0), (3, 10.0, 5.0), (3, 4.0, 3.0)])
def test_measured_error_within_the_printed_bounds(dim, S, mu_deg):
    """Sec. IV-A: the colouring error of the MBR and tangential
    approximations, summed over the whole region of distinguishable
    visibility as |V_approx - V_E| times the size each viewpoint stands for,
    stays below E_MBR and E_Tangent.  The bounds are sums over the cells of
    one meridian quadrant (2-D; the plane holds four) or of the half-space on
    one side of the target plane (3-D; the space holds two).  Measured
    ratios are small (about 0.02-0.3): the printed bounds are far from tight."""
    c = _tiny(S, mu_deg)
    m = 600 if dim == 2 else 90
    step = c.d[-1] / m
    xs = (np.arange(-m, m) + 0.5) * step
    if dim == 2:
        X, Y = np.meshgrid(xs, xs, indexing="ij")
        rho, h, A, copies = np.abs(X).ravel(), np.abs(Y).ravel(), step ** 2, 4
    else:
        X, Y, Z = np.meshgrid(xs, xs, xs, indexing="ij")
        rho, h, A, copies = np.hypot(X, Y).ravel(), np.abs(Z).ravel(), step ** 3, 2
    got = c.bound_measured(np.hypot(rho, h), np.arctan2(h, rho), A)
    bound = c.error_bounds(dim)
    for k in ("mbr", "tangent"):
        ratio = got[k] / (copies * bound[k])
        assert 0.0 < ratio < 1.0, (k, ratio)
