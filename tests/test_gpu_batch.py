"""Batched queries (one persistent launch over many maps on one index).

Batching changes the schedule only: every result must be bit-identical to the
same query computed alone by vcm_compute, which the brute-force and pruned
parity tests tie to the oracle.  A few batched results are also compared with
the oracle directly."""
import numpy as np
import pytest

import oracle
import paper_1310_7297_amd as vcm
from paper_1310_7297_amd import scenes
from paper_1310_7297_amd.scenes import BRUTE, FRACTION, FULL, Params, Query
from mixed import mixed_queries, mixed_scene
from parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    vcm.load_library()


def _solo(idx, q, precision=vcm.VCM_FP32_RECHECK):
    r = vcm.alloc_result(q.grid.count)
    vcm.vcm_compute(idx, q, *r, precision=precision)
    return r


def _same(a, b, what):
    import torch
    torch.cuda.synchronize()
    for x, y, name in zip(a, b, ("bin", "c", "count")):
        n = min(x.numel(), y.numel())
        assert torch.equal(x[:n], y[:n]), f"{what}: {name} differs"


def test_batch_equals_solo_mixed():
    """Billboards and cubes, FULL and FRACTION, float32 and float64, brute and
    pruned (theta 1 and 2), ragged and single-viewpoint grids."""
    scene, targets = mixed_scene()
    qs, prec = mixed_queries(targets)
    idx = vcm.vcm_build_index(scene)
    solo = [_solo(idx, q, p) for q, p in zip(qs, prec)]
    res = [vcm.alloc_result(q.grid.count) for q in qs]
    vcm.vcm_compute_batch(idx, qs, res, precision=prec)
    for i, (a, b) in enumerate(zip(solo, res)):
        _same(a, b, f"query {i}")
    idx.free()


def test_batch_stats_add_up():
    """A batch does the work of its queries run one by one.  FRACTION mode:
    every counter adds up.  FULL mode: rays and viewpoints; its slab tests
    and columns depend on the work-item length (the blocker cache carries
    from one viewpoint of an item to the next), which a single small map
    shortens to keep the device busy."""
    scene, targets = mixed_scene()
    qs, _ = mixed_queries(targets)
    qs = [q for q in qs if q.params.method == BRUTE]
    assert any(q.params.mode == FULL for q in qs) and any(q.params.mode == FRACTION for q in qs)
    idx = vcm.vcm_build_index(scene)
    for sub, keys in ((qs, ("rays", "viewpoints")),
                      ([q for q in qs if q.params.mode == FRACTION],
                       ("rays", "box_tests", "rechecks", "columns", "viewpoints"))):
        tot = dict.fromkeys(keys, 0)
        for q in sub:
            r = vcm.alloc_result(q.grid.count)
            st = vcm.vcm_compute(idx, q, *r, stats=True)
            for k in tot:
                tot[k] += st[k]
        res = [vcm.alloc_result(q.grid.count) for q in sub]
        st = vcm.vcm_compute_batch(idx, sub, res, stats=True)
        for k in tot:
            assert st[k] == tot[k], k
        assert st["fp32_disagree"] == 0
    idx.free()


def test_batch_against_oracle():
    scene, targets = mixed_scene()
    qs, _ = mixed_queries(targets)
    qs = [q for q in qs if q.params.method == BRUTE][:4]
    idx = vcm.vcm_build_index(scene)
    res = [vcm.alloc_result(q.grid.count) for q in qs]
    vcm.vcm_compute_batch(idx, qs, res)
    import torch
    torch.cuda.synchronize()
    for q, (b, c, cnt) in zip(qs, res):
        vp = scenes.viewpoint_sample(q.grid, 300, 3)
        o = oracle.vcm_eval(scene, q, vp)
        g = {"bin": b.cpu().numpy(), "c": c.cpu().numpy(), "count": cnt.cpu().numpy().view(np.uint16)}
        compare(g, o, q.params.n_bins, idx=vp)
    idx.free()


@pytest.mark.parametrize("use_graph", [False, True])
def test_prepared_batch_replays(use_graph):
    """A prepared batch (autotuned, optionally a HIP graph) gives the solo
    results on every replay, with other work on the stream in between."""
    import torch
    scene, targets = mixed_scene()
    qs, prec = mixed_queries(targets)
    idx = vcm.vcm_build_index(scene)
    solo = [_solo(idx, q, p) for q, p in zip(qs, prec)]
    res = [vcm.alloc_result(q.grid.count) for q in qs]
    b = vcm.Batch(idx, qs, res, autotune=True, use_graph=use_graph, precision=prec)
    info = b.info()
    assert info["graph"] == int(use_graph)
    assert info["chunk"] in (4, 8, 16, 32, 64) and info["blocks_per_cu"] in (4, 8)
    assert info["viewpoints"] == sum(q.grid.count for q in qs)
    for rep in range(3):
        for r in res:
            for t in r:
                t.fill_(7 + rep)
        b.run()
        torch.cuda.synchronize()
        for i, (x, y) in enumerate(zip(solo, res)):
            _same(x, y, f"replay {rep} query {i}")
        scratch = torch.randn(1 << 20, device="cuda")
        (scratch * 2).sum().item()  # eager work between replays
    b.close()
    idx.free()


@pytest.mark.parametrize("chunk", [1, 3, 64])
def test_batch_chunk_shapes(chunk):
    """Any chunk in 1..64 gives the same maps (items never straddle rows)."""
    import torch
    scene, targets = mixed_scene()
    qs, prec = mixed_queries(targets)
    idx = vcm.vcm_build_index(scene)
    ref = [vcm.alloc_result(q.grid.count) for q in qs]
    vcm.vcm_compute_batch(idx, qs, ref, precision=prec)
    res = [vcm.alloc_result(q.grid.count) for q in qs]
    b = vcm.Batch(idx, qs, res, chunk=chunk, blocks_per_cu=2, use_graph=False, precision=prec)
    b.run()
    torch.cuda.synchronize()
    for i, (x, y) in enumerate(zip(ref, res)):
        _same(x, y, f"chunk {chunk} query {i}")
    b.close()
    idx.free()


def test_empty_batch_and_rejects():
    scene, targets = mixed_scene()
    idx = vcm.vcm_build_index(scene)
    assert vcm.vcm_compute_batch(idx, [], []) is None
    st = vcm.vcm_compute_batch(idx, [], [], stats=True)
    assert st["viewpoints"] == 0
    qs, _ = mixed_queries(targets)
    bad = Query(qs[0].target, qs[0].grid, Params(n_bins=1))
    res = [vcm.alloc_result(q.grid.count) for q in (qs[0], bad)]
    with pytest.raises(vcm.VcmError) as e:
        vcm.vcm_compute_batch(idx, [qs[0], bad], res)
    assert "query 1" in str(e.value)
    with pytest.raises(vcm.VcmError):
        vcm.Batch(idx, [qs[0]], res[:1], chunk=65)
    idx.free()


def test_city6km_batch256_equals_solo_and_oracle():
    """256 targets of mixed kind and size on a shared 50,000-box city, grids
    from 32x32x16 to 256x256x64, in one batched launch."""
    import torch
    scene, qs = scenes.city6km_batch256()
    idx = vcm.vcm_build_index(scene)
    res = [vcm.alloc_result(q.grid.count) for q in qs]
    b = vcm.Batch(idx, qs, res, autotune=True, use_graph=True)
    b.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    for i in range(len(qs)):
        one = _solo(idx, qs[i])
        _same(one, res[i], f"city6km_batch256 query {i}")
        del one
    for i in rng.choice(len(qs), 6, replace=False):
        q = qs[i]
        vp = scenes.viewpoint_sample(q.grid, 48, int(i))
        o = oracle.vcm_eval(scene, q, vp, nthreads=8)
        bb, c, cnt = res[i]
        g = {"bin": bb.cpu().numpy(), "c": c.cpu().numpy(), "count": cnt.cpu().numpy().view(np.uint16)}
        compare(g, o, q.params.n_bins, idx=vp)
    b.close()
    idx.free()
