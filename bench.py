#!/usr/bin/env python3
"""Benchmark: brute-force VCM throughput on one MI355X.

Workload (default): 4 km x 4 km synthetic city with 20,000 boxes, a 30 m cube
target sampled 8 x 8 per face, 256 x 256 x 64 viewpoints, 16 colour bins,
float32 ray tests with exact float64 recheck, FRACTION mode (every live ray
resolved).  One step = one vcm_compute over the whole grid with the obstacle
index already resident in HBM.  Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic lane-operations per unit of work: one float32 slab test of a ray
# against a box; one corridor column visit; one box record examined by a
# column scan (its top against the floor, its extent across the walk and its
# bottom against the slice: four differences, two ors, two compares); one
# candidate record checked against the corridor over its own extent along the
# walk (clip, two parameter bounds with margins, four extents, four compares).
OPS_PER_BOX_TEST = 20
OPS_PER_COLUMN = 12
OPS_PER_RECORD = 8
OPS_PER_NARROW_TEST = 30
# MI355X: 256 CUs x 4 SIMD x 16 lanes per clock x 2.4 GHz (non-packed lane ops).
PEAK_LANE_OPS = 256 * 64 * 2.4e9
PEAK_HBM = 8.0e12

# HBM bytes per launch of the timed kernel, from the committed rocprofv3
# FETCH_SIZE / WRITE_SIZE summary (copy-kernel calibrated), valid only for the
# kernel sources it was taken on.
PROFILE = os.path.join(ROOT, "profiles", "k_brute_city20k_cube_fraction.md")
TRAFFIC_BYTES = 87600525
TRAFFIC_CELL = 128.0
KERNEL_SOURCES = ("brute.hip", "index.hip", "vcm_internal.h")


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1310_7297_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, mode: str, cell: float):
    """The profiled HBM bytes, or None if the workload or the kernel differs."""
    if workload != "cube" or mode != "fraction" or cell != TRAFFIC_CELL:
        return None
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    return TRAFFIC_BYTES if kernel_sources_hash() in text else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cube", choices=("cube", "billboard"),
                    help="cube: 4 km city, 20,000 boxes, 30 m cube; billboard: 2 km city, 5,000 boxes")
    ap.add_argument("--mode", default="fraction", choices=("fraction", "full"))
    ap.add_argument("--cell", type=float, default=-1.0,
                    help="index column width; -1 (default): autotuned over 32/64/128 m for this "
                         "workload; 0: the library's automatic width")
    ap.add_argument("--cpu-sample", type=int, default=16384)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="time the headline map only (no other mode, batch or serving legs)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched leg (256 targets, 6.4 km city)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg (8 km city, Poisson arrivals)")
    ap.add_argument("--no-pruned", action="store_true", help="skip the pruned-construction leg")
    ap.add_argument("--serve-requests", type=int, default=240)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    return ap.parse_args()


def copy_probe(mib: int):
    """A plain copy kernel of known size: reads and writes `mib` MiB once."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy probe: {mib} MiB read and written per copy, 3 copies", flush=True)


def timed_steps(vcm, idx, q, bufs, steps, warmup):
    import torch
    b, c, cnt = bufs
    for _ in range(warmup):
        vcm.vcm_compute(idx, q, b, c, cnt)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        vcm.vcm_compute(idx, q, b, c, cnt)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = [e0.elapsed_time(e1) for e0, e1 in evs]
    return wall, kms


def bench_pruned(vcm, idx, q):
    """4 km cube map: the pruned construction (VCM_E, VCM_M, VCM_T) beside the
    brute-force map, FULL mode (the paper's rule): time per map, the Sec. V-A
    error of VCM_E against the brute force and of VCM_M / VCM_T against
    VCM_E, the Sec. IV-A bounds, and VCM_E over minimum block sizes."""
    import torch
    from paper_1310_7297_amd import scenes
    n = q.grid.count

    def with_(**kw):
        return scenes.Query(q.target, q.grid, scenes.Params(**{**q.params.__dict__, **kw}))

    def run(qq, reps=3):
        r = vcm.alloc_result(n)
        vcm.vcm_compute(idx, qq, *r)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            vcm.vcm_compute(idx, qq, *r)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return r, min(ms)

    brute, t_b = run(with_(mode=scenes.FULL, method=scenes.BRUTE))
    out = {"mode": "full", "brute_ms": t_b, "methods": {}, "theta": {}}
    maps = {}
    for name, m in (("E", scenes.PRUNED_E), ("M", scenes.PRUNED_M), ("T", scenes.PRUNED_T)):
        r, t = run(with_(mode=scenes.FULL, method=m))
        maps[name] = r
        ref = brute if name == "E" else maps["E"]
        err = vcm.vcm_map_error(ref[1], r[1])
        out["methods"][name] = {"ms": t, "error_vs": "brute" if name == "E" else "E",
                                "error_signed": err[0], "error_abs": err[1]}
    out["bounds"] = vcm.vcm_error_bounds(q, 3)
    for th in (2, 4, 8, 16):
        r, t = run(with_(mode=scenes.FULL, method=scenes.PRUNED_E, theta_blocks=th))
        err = vcm.vcm_map_error(maps["E"][1], r[1])
        out["theta"][str(th)] = {"ms": t, "error_signed_vs_theta1": err[0], "error_abs_vs_theta1": err[1]}
    return out


def bench_batch():
    """Batched: 256 targets on a shared 50,000-box city, grids 32x32x16 to
    256x256x64.  One prepared batch (autotuned launch shape, HIP graph) against
    the same 256 queries as sequential vcm_compute calls; results identical."""
    import torch
    import paper_1310_7297_amd as vcm
    from paper_1310_7297_amd import scenes
    scene, qs = scenes.city6km_batch256()
    tuning = vcm.vcm_tune_cell_size(scene, qs[::8], cell_min=16.0, cell_max=128.0, reps=1)
    idx = vcm.vcm_build_index(scene, cell_size=tuning["best_cell"])
    n_vp = sum(q.grid.count for q in qs)
    seq = [vcm.alloc_result(q.grid.count) for q in qs]
    res = [vcm.alloc_result(q.grid.count) for q in qs]
    t0 = time.perf_counter()
    b = vcm.Batch(idx, qs, res, autotune=True, use_graph=True)
    create_s = time.perf_counter() - t0
    info = b.info()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    def sequential():
        for q, r in zip(qs, seq):
            vcm.vcm_compute(idx, q, *r)

    t_seq = timed(sequential, 2)
    t_batch = timed(b.run, 3)
    t_once = timed(lambda: vcm.vcm_compute_batch(idx, qs, res), 2)
    torch.cuda.synchronize()
    same = all(torch.equal(x, y) for a, r in zip(seq, res) for x, y in zip(a, r))
    b.close()
    idx.free()
    return {"workload": "city6km_batch256: 256 billboards/cubes (5-40 m), 50,000-box 6.4 km city, "
                        "grids 32x32x16..256x256x64",
            "viewpoints": n_vp, "sequential_viewpoints_per_s": n_vp / t_seq,
            "batched_viewpoints_per_s": n_vp / t_batch,
            "batched_unprepared_viewpoints_per_s": n_vp / t_once,
            "speedup_vs_sequential": t_seq / t_batch, "identical_to_sequential": bool(same),
            "chunk": info["chunk"], "blocks_per_cu": info["blocks_per_cu"],
            "launches": info["launches"], "graph": bool(info["graph"]),
            "create_s": create_s, "autotune_ms": info["tune_ms"], "index_cell_tuning": tuning}


def bench_serve(n_req: int):
    """Serving: Poisson arrivals over a resident 100,000-box 8 km city; grids
    64x64x16 / 128x128x32 / 256x256x64 (0.6/0.3/0.1).  p50/p99 latency and
    throughput per arrival rate, and the same requests as sequential calls."""
    import threading
    import torch
    import paper_1310_7297_amd as vcm
    from paper_1310_7297_amd import scenes
    scene, qs = scenes.city8km_serving(n_requests=n_req)
    tuning = vcm.vcm_tune_cell_size(scene, qs[:32], cell_min=16.0, cell_max=128.0, reps=1)
    idx = vcm.vcm_build_index(scene, cell_size=tuning["best_cell"])
    res = [vcm.alloc_result(q.grid.count) for q in qs]
    n_vp = sum(q.grid.count for q in qs)
    # sequential plain calls, back to back
    for q, r in zip(qs[:8], res[:8]):
        vcm.vcm_compute(idx, q, *r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q, r in zip(qs, res):
        vcm.vcm_compute(idx, q, *r)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    out = {"workload": "city8km_serving: 100,000-box 8 km city, Poisson arrivals, grids 64x64x16 / "
                       "128x128x32 / 256x256x64 (0.6/0.3/0.1)",
           "requests": n_req, "mean_viewpoints": n_vp / n_req,
           "sequential_requests_per_s": n_req / t_seq, "index_cell_tuning": tuning, "rates": []}
    srv = vcm.Server(idx, max_inflight=2, max_batch=64)
    for rate in (100.0, 250.0, 500.0, 1000.0, 4000.0, 16000.0):
        srv.reset_stats()
        arr = scenes.poisson_arrivals(rate, n_req, 55)
        tickets = []
        t0 = time.perf_counter()

        def submit():
            for i, q in enumerate(qs):
                while time.perf_counter() - t0 < arr[i]:
                    time.sleep(0.0001)
                while True:
                    t = srv.submit(q, res[i])
                    if t is not None:
                        tickets.append(t)
                        break
                    time.sleep(0.0002)

        th = threading.Thread(target=submit)
        th.start()
        th.join()
        srv.drain()
        for t in tickets:
            srv.poll(t)
        st = srv.stats()
        out["rates"].append({"offered_req_per_s": rate, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                             "max_ms": st["max_ms"], "requests_per_s": st["requests_per_s"],
                             "viewpoints_per_s": st["viewpoints_per_s"], "launches": st["launches"],
                             "rejected_submits": st["rejected"], "mem_peak": st["mem_peak"]})
        print(f"serve: offered {rate:.0f} req/s -> {st['requests_per_s']:.0f} req/s, "
              f"p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
    srv.close()
    idx.free()
    return out


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the maps "
              "would shard by viewpoint ranges with no exchange between GPUs)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1310_7297_amd as vcm
    from paper_1310_7297_amd import scenes

    cfg = scenes.city4km_cube if args.workload == "cube" else scenes.city2km_billboard
    scene, q = cfg()
    mode = scenes.FRACTION if args.mode == "fraction" else scenes.FULL
    q.params.mode = mode
    n_vp = q.grid.count

    tuning = None
    cell = args.cell
    if cell < 0:
        # index autotuner (untimed set-up): fastest column width for this map
        tuning = vcm.vcm_tune_cell_size(scene, [q], cell_min=32.0, cell_max=256.0, reps=1)
        cell = tuning["best_cell"]
    t0 = time.perf_counter()
    idx = vcm.vcm_build_index(scene, cell_size=cell)
    info = idx.info()
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    bufs = vcm.alloc_result(n_vp)

    # Counters for the algorithmic work (untimed run with statistics).
    st = vcm.vcm_compute(idx, q, *bufs, stats=True)
    torch.cuda.synchronize()

    wall, kms = timed_steps(vcm, idx, q, bufs, args.steps, args.warmup)
    ms_step = wall / args.steps * 1e3
    kernel_ms = float(np.mean(kms))
    vps = n_vp * args.steps / wall
    rays_ps = st["rays"] * args.steps / wall

    ops = (OPS_PER_BOX_TEST * st["box_tests"] + OPS_PER_COLUMN * st["columns"]
           + OPS_PER_RECORD * st["records"] + OPS_PER_NARROW_TEST * st["narrow_tests"])
    achieved = ops / (kernel_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                "unit": "Tlane-op/s", "frac": achieved / PEAK_LANE_OPS,
                "traffic": measured_traffic(args.workload, args.mode, info["cell_size"]),
                "kernel": "k_brute", "kernel_ms": kernel_ms,
                "box_tests_per_launch": st["box_tests"], "columns_per_launch": st["columns"],
                "rechecks_per_launch": st["rechecks"],
                "records_per_launch": st["records"], "narrow_tests_per_launch": st["narrow_tests"],
                "slot_tests_per_launch": st.get("slot_tests"),
                "inside_box_viewpoints": st.get("inside_box"),
                "hbm_bytes_algorithmic": 7 * n_vp,
                "hbm_frac": 7 * n_vp / (kernel_ms * 1e-3) / PEAK_HBM}

    extra = {}
    if not args.no_extra:
        # FULL-mode (the paper's complete-visibility rule) throughput beside it.
        qf = scenes.Query(q.target, q.grid, scenes.Params(**{**q.params.__dict__, "mode":
                                                              scenes.FULL if mode == scenes.FRACTION
                                                              else scenes.FRACTION}))
        w2, k2 = timed_steps(vcm, idx, qf, bufs, max(2, args.steps // 2), 1)
        extra["other_mode"] = {"mode": "full" if mode == scenes.FRACTION else "fraction",
                               "viewpoints_per_s": n_vp * max(2, args.steps // 2) / w2,
                               "kernel_ms": float(np.mean(k2))}

    if not (args.no_pruned or args.no_extra) and args.workload == "cube":
        extra["pruned"] = bench_pruned(vcm, idx, q)
        print("pruned: " + ", ".join(f"{k} {v['ms']:.2f} ms" for k, v in extra["pruned"]["methods"].items()),
              file=sys.stderr, flush=True)
    if not (args.no_batch or args.no_extra):
        extra["batch"] = bench_batch()
        print(f"batch: {extra['batch']['speedup_vs_sequential']:.2f}x sequential", file=sys.stderr,
              flush=True)
    if not (args.no_serve or args.no_extra):
        extra["serving"] = bench_serve(args.serve_requests)

    cpu = None
    if not args.no_cpu:
        import oracle
        vp = scenes.viewpoint_sample(q.grid, args.cpu_sample, 12345)
        t0 = time.perf_counter()
        o = oracle.vcm_eval(scene, q, vp, nthreads=1)
        dt = time.perf_counter() - t0
        cpu = {"value": len(vp) / dt, "unit": "viewpoints/s", "cores": 1, "kind": "oracle",
               "sample": f"{len(vp)} seeded uniform-random viewpoints of the same grid and mode, "
                         f"single thread, {dt:.1f} s",
               "rays_per_s": float(o["nlive"][o["infov"] > 0].astype(np.int64).sum()) / dt}
        # the same oracle split over the host's cores (reported beside it)
        ncores = min(16, len(os.sched_getaffinity(0)))
        t0 = time.perf_counter()
        oracle.vcm_eval(scene, q, vp, nthreads=ncores)
        dt_all = time.perf_counter() - t0
        extra["cpu_baseline_all_cores"] = {"value": len(vp) / dt_all, "unit": "viewpoints/s",
                                           "cores": ncores, "kind": "oracle",
                                           "sample": f"the same {len(vp)} viewpoints, {ncores} threads"}

    line = {
        "metric": "VCM viewpoints/s (brute-force map, 3D city)",
        "value": vps,
        "unit": "viewpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64recheck",
        "data": "synthetic",
        "config": {"workload": ("city4km_cube: 4 km city, 20,000 boxes, 30 m cube 8x8/face, "
                                "256x256x64 viewpoints" if args.workload == "cube" else
                                "city2km_billboard: 2 km city, 5,000 boxes, 10x5 m billboard 16x8, "
                                "128x128x32 viewpoints"),
                   "mode": args.mode, "viewpoints": n_vp, "boxes": scene.n, "n_bins": q.params.n_bins,
                   "cell_size": info["cell_size"], "parallelism": "single-gpu"},
        "rays_per_s": rays_ps,
        "rays_per_step": st["rays"],
        "index": {"build_s": build_s, "device_bytes": info["device_bytes"], "refs": info["n_refs"],
                  "columns": [info["nx"], info["ny"]], "cell_size": info["cell_size"],
                  "cell_tuning": tuning},
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
