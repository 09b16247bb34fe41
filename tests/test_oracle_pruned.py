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
    g = Grid((0.0, 0.0, 0.0), (10.0, 10.0, 10.0), (5, 5, 5))
    idx = lambda i, j, k: i + 5 * (j + 5 * k)
    for i in range(5):
        assert oracle.block_rep(g, 3, 1, idx(i, 2, 3)) == idx(i, 2, 3)
    assert oracle.block_rep(g, 3, 2, idx(1, 2, 3)) == idx(0, 2, 2)
    assert oracle.block_rep(g, 3, 3, idx(1, 2, 3)) == idx(1, 1, 4)
    assert oracle.block_rep(g, 3, 4, idx(4, 4, 4)) == idx(4, 4, 4)   # ragged block
    assert oracle.block_rep(g, 3, 4, idx(3, 0, 2)) == idx(1, 1, 1)


def test_pruned_gate_equals_brute_at_theta_one():
    scene, q = scenes.plain2d_50rects()
    for mode in (FULL, FRACTION):
        q.params.mode = mode
        b = oracle.vcm_eval(scene, q)
        for m in (1, 2, 3):
            p = oracle.vcm_eval_pruned(scene, q, m, 1)
            assert np.array_equal(p["count"], b["count"])
            assert np.all((p["c"] > 0) == (b["c"] > 0))
