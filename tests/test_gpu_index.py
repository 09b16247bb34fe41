"""The obstacle index at scale: the 100,000-box 8 km city at every column
width from 16 to 256 m.  The column lists hold exactly the boxes whose grown
footprint overlaps the column (counted here on the host from the same rule),
and maps do not depend on the column width: the index only decides which
boxes a ray is tested against, never the outcome."""
import math

import numpy as np
import pytest

import oracle
import paper_1310_7297_amd as vcm
from paper_1310_7297_amd import scenes
from paper_1310_7297_amd.scenes import FRACTION, FULL, Grid, Query
from parity import compare

pytestmark = pytest.mark.gpu

FAT = 2.0 ** -6     # footprint growth of the index (absorbs the walk's rounding)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    vcm.load_library()


@pytest.fixture(scope="module")
def city8km():
    scene, qs = scenes.city8km_serving(n_requests=8)
    return scene, qs


def _host_lists(scene, cs):
    """Per-column reference counts of the grown footprints, on the host."""
    lo, hi = scene.lo.astype(np.float64), scene.hi.astype(np.float64)
    x0 = math.floor((lo[0].min() - FAT) / cs) * cs
    y0 = math.floor((lo[1].min() - FAT) / cs) * cs
    nx = int(math.floor((hi[0].max() + FAT - x0) / cs)) + 1
    ny = int(math.floor((hi[1].max() + FAT - y0) / cs)) + 1
    ax = np.clip(np.floor((lo[0] - x0 - FAT) / cs), 0, nx - 1).astype(np.int64)
    bx = np.clip(np.floor((hi[0] - x0 + FAT) / cs), 0, nx - 1).astype(np.int64)
    ay = np.clip(np.floor((lo[1] - y0 - FAT) / cs), 0, ny - 1).astype(np.int64)
    by = np.clip(np.floor((hi[1] - y0 + FAT) / cs), 0, ny - 1).astype(np.int64)
    counts = np.zeros((ny, nx), np.int64)
    for dy in range(int((by - ay).max()) + 1):
        for dx in range(int((bx - ax).max()) + 1):
            m = (ay + dy <= by) & (ax + dx <= bx)
            np.add.at(counts, (ay[m] + dy, ax[m] + dx), 1)
    return nx, ny, counts


@pytest.mark.parametrize("cs", [16.0, 32.0, 64.0, 128.0, 256.0])
def test_index_lists_at_scale(city8km, cs):
    scene, _ = city8km
    idx = vcm.vcm_build_index(scene, cell_size=cs)
    info = vcm.vcm_index_get_info(idx)
    nx, ny, counts = _host_lists(scene, cs)
    print(f"cell {cs:5.0f} m: {info['nx']}x{info['ny']} columns, {info['n_refs']} refs, longest "
          f"{info['longest_list']}, kernels {info['kernel_ms']:.3f} ms, build {info['build_ms']:.1f} ms")
    assert (info["nx"], info["ny"]) == (nx, ny)
    assert info["n_boxes"] == scene.n
    assert info["n_refs"] == counts.sum()
    assert info["longest_list"] == counts.max()
    assert info["kernel_ms"] > 0.0
    idx.free()


def test_maps_do_not_depend_on_the_column_width(city8km):
    """The same queries on indexes of 16 to 256 m columns give bit-identical
    maps (the 256 m lists are the longest the sort has to order), and a
    sample of the 256 m map agrees with the oracle."""
    scene, qs = city8km
    ref = {}
    for cs in (16.0, 64.0, 256.0):
        idx = vcm.vcm_build_index(scene, cell_size=cs)
        for i, q in enumerate(qs[:3]):
            for mode in (FRACTION, FULL):
                qq = Query(q.target, q.grid, scenes.Params(**{**q.params.__dict__, "mode": mode}))
                g = vcm.compute_map(idx, qq)
                key = (i, mode)
                if key not in ref:
                    ref[key] = g
                else:
                    for f in ("count", "bin", "c"):
                        assert np.array_equal(g[f], ref[key][f]), (cs, key, f)
                if cs == 256.0 and i == 0:
                    vp = scenes.viewpoint_sample(qq.grid, 2048, 31)
                    compare(g, oracle.vcm_eval(scene, qq, vp, nthreads=16), 16, idx=vp,
                            label=f"city8km 256 m mode {mode}")
        idx.free()


def test_small_and_empty_indexes():
    """Empty scenes, one box, 2-D scenes: the column lists end with their
    sentinel and the maps equal the oracle's."""
    for sc in (scenes.Scene(3, np.zeros((3, 0)), np.zeros((3, 0))),
               scenes.Scene(3, np.array([[10.0], [10.0], [0.0]]), np.array([[20.0], [30.0], [5.0]])),
               scenes.plain2d_50rects()[0]):
        if sc.dim == 3:
            t = scenes.Target(scenes.CUBE, (40.0, 40.0, 4.0), (4.0, 0.0), samples_u=2, samples_v=2)
            q = Query(t, Grid((0.0, 0.0, 0.0), (64.0, 64.0, 16.0), (16, 16, 4)), scenes.Params(n_bins=8))
        else:
            q = scenes.plain2d_50rects()[1]
        for cs in (1.0, 8.0, 256.0):
            idx = vcm.vcm_build_index(sc, cell_size=cs)
            info = vcm.vcm_index_get_info(idx)
            assert info["n_refs"] >= sc.n
            compare(vcm.compute_map(idx, q), oracle.vcm_eval(sc, q), 8, label=f"cs {cs} n {sc.n}")
            idx.free()
