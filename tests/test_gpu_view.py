"""Incremental processing (Sec. IV-C) on the GPU: a view keeps every
viewpoint's visibility at a 360-degree field of view and renders maps for
other fields of view and gaze directions without tracing again."""
import numpy as np
import pytest

import oracle
import paper_1310_7297_amd as vcm
from paper_1310_7297_amd import scenes
from paper_1310_7297_amd.scenes import (BILLBOARD, BIN_LOG, CUBE, FRACTION, FULL, SEGMENT, Grid, Params,
                                         Query, Scene, Target)
from parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    vcm.load_library()


def _with(q, **kw):
    return Query(q.target, q.grid, Params(**{**q.params.__dict__, **kw}))


def _host(r):
    import torch
    torch.cuda.synchronize()
    return {"bin": r[0].cpu().numpy(), "c": r[1].cpu().numpy(), "count": r[2].cpu().numpy().view(np.uint16)}


def _scene(kind):
    if kind == SEGMENT:
        scene, q = scenes.plain2d_50rects()
        return scene, q.target, q.grid
    if kind == CUBE:
        t = Target(CUBE, (128.0, 128.0, 6.0), (12.0, 0.0), samples_u=8, samples_v=8)
    else:
        t = Target(BILLBOARD, (128.0, 128.0, 8.0), (12.0, 6.0), normal_axis=0, normal_sign=-1,
                   samples_u=16, samples_v=8)
    scene = scenes.city(256.0, 80, seed=13, side=(6.0, 24.0), targets=[t], clearance=2.0)
    # ragged against the blocks in y and z; on the 2^-8 lattice
    return scene, t, Grid((0.0, 0.0, 0.0), (256.0, 288.0, 48.0), (64, 36, 12))


GAZES = {SEGMENT: [(120.0, 0), (90.0, 1), (240.0, -2), (60.0, -1), (360.0, 2)],
         BILLBOARD: [(120.0, 0), (60.0, 2), (240.0, -1), (180.0, 3), (300.0, -3)],
         CUBE: [(120.0, 3), (90.0, 1), (240.0, -2), (360.0, 0), (60.0, -3)]}


@pytest.mark.parametrize("kind", [SEGMENT, BILLBOARD, CUBE])
@pytest.mark.parametrize("method,theta", [(0, 1), (1, 1), (3, 1)])
@pytest.mark.parametrize("mode", [FULL, FRACTION])
def test_render_equals_compute(kind, method, theta, mode):
    """Renders of one view, for several fields of view and gaze directions in
    a row, equal vcm_compute of the query with that field of view, bit for
    bit (brute force, and pruned maps with theta = 1)."""
    scene, t, g = _scene(kind)
    q = Query(t, g, Params(n_bins=16, mode=mode, method=method, theta_blocks=theta, bin_scale=BIN_LOG))
    idx = vcm.vcm_build_index(scene)
    view = vcm.View(idx, q)
    assert view.info()["viewpoints"] == g.count
    for fov, gaze in GAZES[kind]:
        r = vcm.alloc_result(g.count)
        view.render(fov, gaze, *r)
        got = _host(r)
        want = vcm.compute_map(idx, _with(q, fov_deg=fov, gaze=gaze))
        for k in ("bin", "c", "count"):
            assert np.array_equal(got[k], want[k]), (fov, gaze, k)
        if method == 0:
            o = oracle.vcm_eval(scene, _with(q, fov_deg=fov, gaze=gaze),
                                scenes.viewpoint_sample(g, 600, 3), nthreads=8)
            compare(got, o, 16, idx=scenes.viewpoint_sample(g, 600, 3), label=f"view {kind} {fov} {gaze}")
    view.close()
    idx.free()


@pytest.mark.parametrize("theta", [2, 4])
def test_render_of_blocks_masks_each_viewpoint(theta):
    """A pruned map with larger blocks: the gates of the 360-degree map,
    each viewpoint masked by its own position (against the oracle)."""
    scene, t, g = _scene(BILLBOARD)
    q = Query(t, g, Params(n_bins=16, mode=FULL, method=1, theta_blocks=theta, bin_scale=BIN_LOG))
    idx = vcm.vcm_build_index(scene)
    view = vcm.View(idx, q)
    vp = np.arange(g.count, dtype=np.int64)
    o360 = oracle.vcm_eval_pruned(scene, q, 1, theta, vp, nthreads=8)
    pts = oracle.viewpoint_coords(g, vp)
    for fov, gaze in ((120.0, 0), (240.0, 2)):
        r = vcm.alloc_result(g.count)
        view.render(fov, gaze, *r)
        got = _host(r)
        p = _with(q, fov_deg=fov, gaze=gaze).params
        inside = np.array([oracle.in_fov(t, p, x) for x in pts])
        assert np.array_equal(got["count"], np.where(inside, o360["count"], 0))
        want_c = np.where(inside, o360["c"], 0.0)
        assert np.all(np.abs(got["c"] - want_c) <= 1e-5 * want_c + 1e-9)
        assert 0 < inside.sum() < g.count
    view.close()
    idx.free()


def test_view_arguments():
    scene, t, g = _scene(CUBE)
    idx = vcm.vcm_build_index(scene)
    q = Query(t, g, Params(n_bins=16, mode=FULL))
    view = vcm.View(idx, q)
    r = vcm.alloc_result(g.count)
    for fov, gaze in ((120.0, 0), (120.0, 4), (0.0, 1)):   # a cube needs a gaze; axis 3; fov 0
        with pytest.raises(vcm.VcmError) as e:
            view.render(fov, gaze, *r)
        assert e.value.status == vcm.VCM_E_INVALID
    view.close()
    idx.free()
