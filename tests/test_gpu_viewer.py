"""Parity of the viewer-centric VCM (Sec. IV-B) on the GPU with the oracle:
brute force and the pruned constructions, 2-D and 3-D, through the C-ABI."""
import numpy as np
import pytest

import oracle
import paper_1310_7297_amd as vcm
from paper_1310_7297_amd import scenes
from paper_1310_7297_amd.scenes import (BIN_LOG, FRACTION, FULL, VIEWER, Grid, Params, Query, Scene,
                                         Target)
from parity import compare, compare_pruned

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    vcm.load_library()


def _viewer(center, dmax, axis=1, sign=1):
    return Target(VIEWER, center, (dmax, 0.0), normal_axis=axis, normal_sign=sign, samples_u=1,
                  samples_v=1)


def _map(scene, q, stats=False, precision=vcm.VCM_FP32_RECHECK):
    idx = vcm.vcm_build_index(scene)
    out = vcm.compute_map(idx, q, stats=stats, precision=precision)
    idx.free()
    return out


def _without_viewer(sc, v):
    keep = ~np.all((sc.lo[:sc.dim] <= np.array(v[:sc.dim])[:, None]) &
                   (sc.hi[:sc.dim] >= np.array(v[:sc.dim])[:, None]), axis=0)
    return Scene(sc.dim, sc.lo[:, keep], sc.hi[:, keep])


@pytest.mark.parametrize("fov", [360.0, 120.0, 240.0])
@pytest.mark.parametrize("precision", [vcm.VCM_FP32_RECHECK, vcm.VCM_FP64])
def test_viewer_2d_whole_map(fov, precision):
    scene, _ = scenes.plain2d_50rects()
    v = (500.0, 500.0, 0.0)
    t = _viewer(v, 400.0)
    q = Query(t, Grid((0.0, 0.0, 0.0), (1000.0, 1000.0, 0.0), (64, 64, 1)),
              Params(n_bins=8, fov_deg=fov, bin_scale=BIN_LOG))
    g = _map(scene, q, precision=precision)
    o = oracle.vcm_eval(scene, q)
    compare(g, o, 8, label=f"viewer 2d fov {fov}")
    assert 200 < (o["count"] > 0).sum() < q.grid.count - 200


@pytest.mark.parametrize("mode", [FULL, FRACTION])
def test_viewer_3d_city_sampled(mode):
    """A street-level viewer in the 4 km city, the ball of 600 m about it."""
    scene, _ = scenes.city4km_cube()
    v = (1800.0, 2200.0, 1.5)
    scene = _without_viewer(scene, v)
    t = _viewer(v, 600.0)
    q = Query(t, Grid((1152.0, 1552.0, 0.0), (1280.0, 1280.0, 120.0), (128, 128, 24)),
              Params(n_bins=16, mode=mode, bin_scale=BIN_LOG))
    g = _map(scene, q)
    vp = np.unique(np.concatenate([scenes.viewpoint_sample(q.grid, 3000, 1),
                                   np.arange(60 + 128 * 64, 68 + 128 * 64)]))
    o = oracle.vcm_eval(scene, q, vp, nthreads=16)
    compare(g, o, 16, idx=vp, label=f"viewer city mode {mode}")
    assert (o["count"] > 0).sum() > 20
    # outside the ball: nothing
    pts = oracle.viewpoint_coords(q.grid, np.arange(q.grid.count))
    out = np.linalg.norm(pts - np.array(v), axis=1) > 600.0
    assert np.all(g["count"][out] == 0) and np.all(g["c"][out] == 0.0)


@pytest.mark.parametrize("method", [1, 2, 3])
@pytest.mark.parametrize("theta", [1, 2])
def test_viewer_pruned_whole_map(method, theta):
    sc = scenes.city(256.0, 60, seed=9, side=(6.0, 24.0))
    v = (128.0, 128.0, 40.0)
    sc = _without_viewer(sc, v)
    t = _viewer(v, 96.0)
    q = Query(t, Grid((32.0, 32.0, 0.0), (192.0, 192.0, 64.0), (24, 24, 8)),
              Params(n_bins=16, method=method, theta_blocks=theta, mode=FULL, bin_scale=BIN_LOG))
    g = _map(scene=sc, q=q, stats=True)
    vp = np.arange(q.grid.count, dtype=np.int64)
    o = oracle.vcm_eval_pruned(sc, q, method, theta, vp, nthreads=8)
    compare_pruned(g, o, sc, q, vp, method)
    assert (o["count"] > 0).sum() > 100
    if theta == 1:
        b = _map(sc, Query(t, q.grid, Params(n_bins=16, mode=FULL)))
        assert np.array_equal(g["count"], b["count"])


def test_viewer_validation():
    scene, _ = scenes.plain2d_50rects()
    idx = vcm.vcm_build_index(scene)
    b, c, n = vcm.alloc_result(16)
    g = Grid((0.0, 0.0, 0.0), (1000.0, 1000.0, 0.0), (4, 4, 1))
    bad = [Target(VIEWER, (500.0, 500.0, 0.0), (400.0, 0.0), samples_u=2, samples_v=1),
           Target(VIEWER, (500.0, 500.0, 0.0), (400.1, 0.0), samples_u=1, samples_v=1),
           Target(VIEWER, (500.0, 500.0, 3.0), (400.0, 0.0), samples_u=1, samples_v=1)]
    # a viewer inside an obstacle
    bad.append(Target(VIEWER, tuple(float(x) for x in scene.lo[:, 0]) , (400.0, 0.0), samples_u=1,
                      samples_v=1))
    for t in bad:
        with pytest.raises(vcm.VcmError) as e:
            vcm.vcm_compute(idx, Query(t, g, Params()), b, c, n)
        assert e.value.status == vcm.VCM_E_INVALID
    idx.free()
