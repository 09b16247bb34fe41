"""Serving loop: admission by device memory, continuous batching, latency.

Every served result must be bit-identical to the same query computed alone
(vcm_compute), whatever else was batched with it."""
import threading
import time

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


def _solo(idx, q, precision=vcm.VCM_FP32_RECHECK):
    r = vcm.alloc_result(q.grid.count)
    vcm.vcm_compute(idx, q, *r, precision=precision)
    return r


def _same(a, b, what):
    import torch
    torch.cuda.synchronize()
    for x, y, name in zip(a, b, ("bin", "c", "count")):
        assert torch.equal(x, y), f"{what}: {name} differs"


def _serve(server, qs, results, prec, arrivals):
    """Submit on a thread at the given arrival times (retrying on VCM_E_AGAIN);
    return the tickets in query order."""
    tickets = [None] * len(qs)
    t0 = time.perf_counter()

    def run():
        for i, q in enumerate(qs):
            while time.perf_counter() - t0 < arrivals[i]:
                time.sleep(0.0002)
            while True:
                t = server.submit(q, results[i], precision=prec[i])
                if t is not None:
                    tickets[i] = t
                    break
                time.sleep(0.0005)

    th = threading.Thread(target=run)
    th.start()
    th.join(timeout=120)
    assert not th.is_alive()
    return tickets


def test_served_results_equal_solo():
    scene, targets = mixed_scene()
    qs, prec = mixed_queries(targets)
    qs, prec = qs * 4, prec * 4
    idx = vcm.vcm_build_index(scene)
    solo = [_solo(idx, q, p) for q, p in zip(qs, prec)]
    res = [vcm.alloc_result(q.grid.count) for q in qs]
    srv = vcm.Server(idx, max_inflight=2, max_batch=8)
    arrivals = scenes.poisson_arrivals(2000.0, len(qs), 9)
    tickets = _serve(srv, qs, res, prec, arrivals)
    infos = [srv.wait(t, 60000) for t in tickets]
    assert all(i is not None for i in infos)
    for i, (a, b) in enumerate(zip(solo, res)):
        _same(a, b, f"request {i}")
    st = srv.stats()
    assert st["completed"] == len(qs) and st["failed"] == 0
    assert st["launches"] <= len(qs)
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert st["mem_in_use"] == 0
    srv.close()
    idx.free()


def test_waiting_requests_share_one_launch():
    """Requests admitted while launches are held go out together when
    released: one launch for eight requests with max_batch 64, three with
    max_batch 3 (submission order, a launch per slot at a time); every
    result equals the request computed alone."""
    scene, targets = mixed_scene()
    qs, prec = mixed_queries(targets)
    small, sp = qs[:8], prec[:8]
    idx = vcm.vcm_build_index(scene)
    solo = [_solo(idx, q, p) for q, p in zip(small, sp)]
    for max_batch, launches in ((64, 1), (3, 3)):
        srv = vcm.Server(idx, max_inflight=1, max_batch=max_batch)
        srv.hold(True)
        res = [vcm.alloc_result(q.grid.count) for q in small]
        tickets = [srv.submit(q, r, precision=p) for q, r, p in zip(small, res, sp)]
        assert all(t is not None for t in tickets)
        time.sleep(0.01)
        assert srv.stats()["launches"] == 0
        srv.hold(False)
        for t in tickets:
            assert srv.wait(t, 60000) is not None
        st = srv.stats()
        assert st["completed"] == 8 and st["failed"] == 0
        assert st["launches"] == launches, st
        for i, (a, b) in enumerate(zip(solo, res)):
            _same(a, b, f"request {i} (max_batch {max_batch})")
        srv.close()
    idx.free()


def test_admission_by_memory():
    """A budget for about two requests: later submits are refused with
    VCM_E_AGAIN until earlier ones finish; the budget is never exceeded."""
    scene, targets = mixed_scene()
    qs, prec = mixed_queries(targets)
    q = qs[0]  # a 32x32x8 billboard map
    n = q.grid.count
    budget = 2 * (7 * n + 1024)
    idx = vcm.vcm_build_index(scene)
    ref = _solo(idx, q)
    srv = vcm.Server(idx, mem_budget_bytes=budget, max_inflight=1)
    res = [vcm.alloc_result(n) for _ in range(12)]
    done, refused = 0, 0
    pending = []
    for r in res:
        while True:
            t = srv.submit(q, r)
            if t is not None:
                pending.append(t)
                break
            refused += 1
            srv.wait(pending.pop(0), 60000)
            done += 1
    for t in pending:
        srv.wait(t, 60000)
    assert refused > 0
    st = srv.stats()
    assert st["mem_peak"] <= budget and st["rejected"] == refused
    for i, r in enumerate(res):
        _same(ref, r, f"request {i}")
    big = scenes.Query(q.target, scenes.Grid(q.grid.origin, q.grid.extent, (64, 64, 16)), q.params)
    with pytest.raises(vcm.VcmError) as e:
        srv.submit(big, vcm.alloc_result(big.grid.count))
    assert e.value.status == vcm.VCM_E_INVALID
    srv.close()
    idx.free()


def test_poll_semantics_and_errors():
    scene, targets = mixed_scene()
    qs, _ = mixed_queries(targets)
    idx = vcm.vcm_build_index(scene)
    srv = vcm.Server(idx)
    with pytest.raises(vcm.VcmError) as e:
        srv.poll(12345)
    assert e.value.status == vcm.VCM_E_NOTFOUND
    r = vcm.alloc_result(qs[0].grid.count)
    t = srv.submit(qs[0], r)
    info = srv.wait(t, 60000)
    assert info["viewpoints"] == qs[0].grid.count and info["latency_ms"] >= info["queue_ms"] >= 0
    with pytest.raises(vcm.VcmError):
        srv.poll(t)  # a finished ticket is reported once
    bad = scenes.Query(qs[0].target, qs[0].grid, scenes.Params(n_bins=300))
    with pytest.raises(vcm.VcmError) as e:
        srv.submit(bad, r)
    assert e.value.status == vcm.VCM_E_INVALID
    srv.drain()
    assert srv.stats()["mem_in_use"] == 0
    srv.close()
    idx.free()


def test_destroy_with_requests_in_flight():
    """Shutting down with requests waiting and running neither hangs nor
    faults; launched work completes before the streams go away."""
    scene, targets = mixed_scene()
    qs, prec = mixed_queries(targets)
    idx = vcm.vcm_build_index(scene)
    srv = vcm.Server(idx, max_inflight=1, max_batch=2)
    res = [vcm.alloc_result(q.grid.count) for q in qs]
    for q, r, p in zip(qs, res, prec):
        assert srv.submit(q, r, precision=p) is not None
    srv.close()
    import torch
    torch.cuda.synchronize()
    idx.free()


def test_city8km_serving_sample():
    """Requests of the serving workload (100,000-box 8 km city, grids
    64x64x16 / 128x128x32 / 256x256x64) arriving at 500 per second."""
    scene, qs = scenes.city8km_serving(n_requests=120)
    idx = vcm.vcm_build_index(scene)
    res = [vcm.alloc_result(q.grid.count) for q in qs]
    srv = vcm.Server(idx, max_inflight=2, max_batch=32)
    arrivals = scenes.poisson_arrivals(500.0, len(qs), 55)
    prec = [vcm.VCM_FP32_RECHECK] * len(qs)
    tickets = _serve(srv, qs, res, prec, arrivals)
    for t in tickets:
        assert srv.wait(t, 120000) is not None
    st = srv.stats()
    assert st["completed"] == len(qs)
    rng = np.random.default_rng(5)
    for i in rng.choice(len(qs), 12, replace=False):
        _same(_solo(idx, qs[i]), res[i], f"city8km_serving request {i}")
    srv.close()
    idx.free()
