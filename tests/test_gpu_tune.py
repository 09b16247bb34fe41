"""Index autotuning: the map does not depend on the index's column width, and
the tuner returns the fastest width it timed."""
import numpy as np
import pytest

import paper_1310_7297_amd as vcm
from mixed import mixed_queries, mixed_scene
from paper_1310_7297_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    vcm.load_library()


@pytest.mark.parametrize("mode", [scenes.FULL, scenes.FRACTION])
def test_map_independent_of_cell_size(mode):
    scene, q = scenes.city2km_billboard()
    q = scenes.Query(q.target, q.grid, scenes.Params(**{**q.params.__dict__, "mode": mode}))
    maps = []
    for cs in (8.0, 32.0, 128.0, 512.0):
        idx = vcm.vcm_build_index(scene, cell_size=cs)
        assert idx.info()["cell_size"] == cs
        maps.append(vcm.compute_map(idx, q))
        idx.free()
    for m in maps[1:]:
        for k in ("bin", "c", "count"):
            assert np.array_equal(m[k], maps[0][k]), k


def test_tuner_returns_fastest_width():
    scene, targets = mixed_scene()
    qs, _ = mixed_queries(targets)
    qs = [q for q in qs if q.params.method == scenes.BRUTE]
    r = vcm.vcm_tune_cell_size(scene, qs, cell_min=8.0, cell_max=64.0, reps=1)
    assert r["cells"] == [8.0, 16.0, 32.0, 64.0]
    assert r["best_cell"] == r["cells"][int(np.argmin(r["ms"]))]
    assert all(t > 0 for t in r["ms"])
    with pytest.raises(vcm.VcmError):
        vcm.vcm_tune_cell_size(scene, qs, cell_min=24.0)
