"""Trend checks of the paper's parameter sweeps (Table 2; Sec. V-C and V-D)
on synthetic cities: the paper's datasets are not available, so only the
directions of its findings are checked, at the ends of each range.

* angular resolution mu: the errors of VCM_M and VCM_T against VCM_E grow
  from mu = 1' to 16', and VCM_T is the more accurate of the two;
* minimum block size theta: fewer viewpoints are traced as theta grows
  (the misjudged share stays small: decided blocks are exact);
* field of view: more rays are traced (more viewpoints are in view) as the
  field of view widens from 60 to 360 degrees;
* obstacles: with more obstacles (5k to 25k, uniform and Zipf-clustered) the
  space is more obstructed (fewer viewpoints see the target)."""
import numpy as np
import pytest

import paper_1310_7297_amd as vcm
from paper_1310_7297_amd import scenes
from paper_1310_7297_amd.scenes import FULL, PRUNED_E, PRUNED_M, PRUNED_T, BRUTE, Grid, Params, Query

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    vcm.load_library()


def _small(q):
    """The sweep grid at a quarter of the viewpoints per axis (same extent)."""
    return Query(q.target, Grid(q.grid.origin, q.grid.extent, (128, 128, 32)), q.params)


def _with(q, **kw):
    return Query(q.target, q.grid, Params(**{**q.params.__dict__, **kw}))


@pytest.fixture(scope="module")
def city():
    scene, q = scenes.sweep_billboard()
    idx = vcm.vcm_build_index(scene, cell_size=64.0)
    yield scene, _small(q), idx
    idx.free()


def _errors(idx, q):
    out = {}
    for name, m in (("M", PRUNED_M), ("T", PRUNED_T)):
        st = vcm.compute_map(idx, _with(q, method=m, mode=FULL), stats=True)["stats"]
        out[name] = st["err_abs"]
    return out


def test_mu_sweep(city):
    _, q, idx = city
    e = {mu: _errors(idx, _with(q, mu_arcmin=mu)) for mu in (1.0, 4.0, 16.0)}
    print({mu: {k: round(v, 5) for k, v in d.items()} for mu, d in e.items()})
    assert e[16.0]["M"] > e[1.0]["M"] and e[16.0]["T"] > e[1.0]["T"]
    assert sum(d["T"] for d in e.values()) < sum(d["M"] for d in e.values())


def test_theta_sweep(city):
    """Larger minimum blocks trace fewer viewpoints.  The paper finds the
    error growing with theta; with blocks decided exactly before any
    representative is used, the viewpoints misjudged against theta = 1 stay
    few at every theta here (a finding, not the paper's trend), and the
    test bounds them."""
    _, q, idx = city
    base = vcm.compute_map(idx, _with(q, method=PRUNED_E, mode=FULL))
    wrong, traced = [], []
    for th in (2, 4, 16):
        g = vcm.compute_map(idx, _with(q, method=PRUNED_E, mode=FULL, theta_blocks=th), stats=True)
        wrong.append(float(((g["count"] > 0) != (base["count"] > 0)).mean()))
        traced.append(g["stats"]["leaves"])
    print(wrong, traced)
    assert traced[0] > traced[1] > traced[2]
    assert all(0.0 <= w < 0.01 for w in wrong)


def test_fov_sweep(city):
    _, q, idx = city
    rays = []
    for fov in (60.0, 120.0, 360.0):
        g = vcm.compute_map(idx, _with(q, method=BRUTE, mode=FULL, fov_deg=fov), stats=True)
        rays.append(g["stats"]["rays"])
    print(rays)
    assert rays[0] < rays[1] < rays[2]


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_obstacle_sweep(dist):
    seen = []
    for n in (5000, 25000):
        sc, q = scenes.sweep_billboard(n, dist)
        q = _with(_small(q), method=BRUTE, mode=FULL)
        idx = vcm.vcm_build_index(sc, cell_size=64.0)
        g = vcm.compute_map(idx, q)
        seen.append(float((g["count"] > 0).mean()))
        idx.free()
    print(dist, seen)
    assert seen[1] < seen[0]
