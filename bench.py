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

# Algorithmic lane-operations per unit of work (the roofline's useful work):
# one float32 slab test of a ray against a box (6 subtractions or products,
# 3 min, 3 max, max3/min3, clamps and compares: 20); one corridor column
# visited (12).  The headline fraction counts these only.
OPS_PER_BOX_TEST = 20
OPS_PER_COLUMN = 12
# This implementation's own culling, reported beside the headline: one box
# record examined by a column scan (four differences, two ors, two compares)
# and one candidate checked against the corridor over its own extent along
# the walk (clip, two parameter bounds with margins, four extents, four
# compares).
OPS_PER_RECORD = 8
OPS_PER_NARROW_TEST = 30
# MI355X: 256 CUs x 4 SIMD x 16 lanes per clock x 2.4 GHz (non-packed lane ops).
PEAK_LANE_OPS = 256 * 64 * 2.4e9
PEAK_HBM = 8.0e12

# HBM bytes per launch of the timed kernel, from the committed rocprofv3
# FETCH_SIZE / WRITE_SIZE summary (copy-kernel calibrated), valid only for the
# kernel sources it was taken on.
PROFILE = os.path.join(ROOT, "profiles", "k_brute_city20k_cube_fraction.md")
TRAFFIC_BYTES = 139207458
TRAFFIC_CELL = 128.0
KERNEL_SOURCES = ("brute.hip", "trace_common.h", "index.hip", "vcm_internal.h")
# Issue counters of the same profile (per launch), valid under the same hash.
PROFILE_VALU = {"fraction": 2.685e9, "full": 5.313e8}
CUS, CLOCK = 256, 2.4e9


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1310_7297_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_valid(workload: str, cell: float) -> bool:
    """The committed profile covers this workload, index width and kernel sources."""
    if workload != "cube" or cell != TRAFFIC_CELL:
        return False
    try:
        text = open(PROFILE).read()
    except OSError:
        return False
    return kernel_sources_hash() in text


def measured_traffic(workload: str, mode: str, cell: float):
    """The profiled HBM bytes, or None if the workload or the kernel differs."""
    if mode != "fraction" or not profile_valid(workload, cell):
        return None
    return TRAFFIC_BYTES


def roofline_of(st, kernel_ms):
    """Useful-work roofline of one ray-kernel launch from its statistics."""
    ops = OPS_PER_BOX_TEST * st["box_tests"] + OPS_PER_COLUMN * st["columns"]
    cull = OPS_PER_RECORD * st["records"] + OPS_PER_NARROW_TEST * st["narrow_tests"]
    t = kernel_ms * 1e-3
    return {"achieved": ops / t / 1e12, "frac": ops / t / PEAK_LANE_OPS, "lane_ops_per_launch": ops,
            "with_culling": {"lane_ops_per_launch": ops + cull, "achieved": (ops + cull) / t / 1e12,
                             "frac": (ops + cull) / t / PEAK_LANE_OPS}}


def oracle_agreement(gpu, orc, n_bins):
    """The timed map against the float64 oracle on the same viewpoints: counts
    exact; bins exact except where the oracle's colour is within 1e-6 of a bin
    edge; colours within 1e-5 relative (1e-9 absolute floor)."""
    import numpy as np
    cnt = np.count_nonzero(gpu["count"].astype(np.int64) != orc["count"].astype(np.int64))
    x = orc["cb"] * n_bins
    k = np.round(x)
    edge = (np.abs(x - k) < 1e-6 * n_bins) & (k >= 1) & (k <= n_bins - 1)   # interior bin edges
    bins = np.count_nonzero((gpu["bin"] != orc["bin"]) & ~edge)
    err = np.abs(gpu["c"].astype(np.float64) - orc["c"])
    rel = err / np.maximum(np.abs(orc["c"]), 1e-30)
    out = np.count_nonzero(err > 1e-5 * np.abs(orc["c"]) + 1e-9)
    return {"viewpoints": int(len(orc["count"])), "count_mismatches": int(cnt),
            "bin_mismatches_off_edge": int(bins), "edge_viewpoints_skipped": int(edge.sum()),
            "colour_out_of_tolerance": int(out),
            "max_rel_colour_error": float(np.max(np.where(orc["c"] > 0, rel, 0.0), initial=0.0)),
            "tolerance": "count exact; bins exact off 1e-6 of interior edges; colour 1e-5 relative + 1e-9"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cube", choices=("cube", "billboard"),
                    help="cube: 4 km city, 20,000 boxes, 30 m cube; billboard: 2 km city, 5,000 boxes")
    ap.add_argument("--mode", default="fraction", choices=("fraction", "full"))
    ap.add_argument("--cell", type=float, default=128.0,
                    help="index column width (default 128 m: what the index autotuner picks for the "
                         "4 km cube map, within 0.1%% of 256 m); -1: run the autotuner over 32-256 m "
                         "first; 0: the library's automatic width")
    ap.add_argument("--cpu-sample", type=int, default=16384)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="time the headline map only (no other mode, batch or serving legs)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched leg (256 targets, 6.4 km city)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg (8 km city, Poisson arrivals)")
    ap.add_argument("--no-pruned", action="store_true", help="skip the pruned-construction leg")
    ap.add_argument("--no-index", action="store_true", help="skip the index-build leg (100,000 boxes)")
    ap.add_argument("--no-sweeps", action="store_true", help="skip the parameter sweeps (mu, theta, FOV, obstacles)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 2-D plain and 2 km billboard maps timed beside the headline")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests per arrival rate of the serving leg (2,000 as configured)")
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


def bench_configs(steps: int):
    """The two smaller configurations beside the headline, brute force in both
    modes: the 2-D plain map (1000 x 1000, 50 rectangles, segment target of
    32 samples, 64 x 64 viewpoints, float64 throughout) and the 3-D plain map
    (2 km city, 5,000 boxes, 10 x 5 m billboard 16 x 8, 128 x 128 x 32
    viewpoints, float32 + exact recheck).  Returns the figures and, per map,
    its outputs on a sample of viewpoints (all of the 2-D map), which the
    oracle leg compares with the float64 oracle."""
    import numpy as np
    import torch
    import paper_1310_7297_amd as vcm
    from paper_1310_7297_amd import scenes
    out, samples = {}, []
    for name, cfg, prec, n_sample in (("plain2d_50rects", scenes.plain2d_50rects, vcm.VCM_FP64, 4096),
                                      ("city2km_billboard", scenes.city2km_billboard, vcm.VCM_FP32_RECHECK,
                                       16384)):
        scene, q0 = cfg()
        idx = vcm.vcm_build_index(scene)
        n = q0.grid.count
        bufs = vcm.alloc_result(n)
        vp = scenes.viewpoint_sample(q0.grid, n_sample, 777)
        leg = {"viewpoints": n, "boxes": scene.n, "precision": "f64" if prec == vcm.VCM_FP64 else "f32+f64recheck",
               "cell_size": idx.info()["cell_size"]}
        for mname, mode in (("full", scenes.FULL), ("fraction", scenes.FRACTION)):
            q = scenes.Query(q0.target, q0.grid, scenes.Params(**{**q0.params.__dict__, "mode": mode}))
            st = vcm.vcm_compute(idx, q, *bufs, stats=True, precision=prec)
            vcm.vcm_compute(idx, q, *bufs, precision=prec)
            torch.cuda.synchronize()
            stream = torch.cuda.current_stream()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(steps)]
            t0 = time.perf_counter()
            for e0, e1 in evs:
                e0.record(stream)
                vcm.vcm_compute(idx, q, *bufs, precision=prec)
                e1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            kms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
            g = {"bin": bufs[0].cpu().numpy(), "c": bufs[1].cpu().numpy(),
                 "count": bufs[2].cpu().numpy().view(np.uint16)}
            leg[mname] = {"viewpoints_per_s": n * steps / wall, "rays_per_s": st["rays"] * steps / wall,
                          "kernel_ms": kms, "rays_per_map": st["rays"]}
            samples.append((leg[mname], scene, q, vp, {k: v[vp] for k, v in g.items()}))
        idx.free()
        out[name] = leg
    return out, samples


def bench_pruned(vcm, idx, q):
    """4 km cube map: the pruned construction (VCM_E, VCM_M, VCM_T) beside the
    brute-force map, in both modes.  Per method: time per map (visible-region
    blocks, the traced representatives of the undecided smallest blocks, and
    the cell colouring), the blocks decided and traced, the Sec. V-A error of
    VCM_E against the brute force and of VCM_M / VCM_T against VCM_E, and the
    Sec. IV-A bound beside the error it covers measured over the grid; then
    VCM_E over minimum block sizes."""
    import torch
    from paper_1310_7297_amd import scenes
    n = q.grid.count

    def with_(**kw):
        return scenes.Query(q.target, q.grid, scenes.Params(**{**q.params.__dict__, **kw}))

    def run(qq, reps=3):
        r = vcm.alloc_result(n)
        st = vcm.vcm_compute(idx, qq, *r, stats=True)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            vcm.vcm_compute(idx, qq, *r)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return r, min(ms), st

    out = {}
    for mode_name, mode in (("full", scenes.FULL), ("fraction", scenes.FRACTION)):
        _, t_b, _ = run(with_(mode=mode, method=scenes.BRUTE))
        leg = {"brute_ms": t_b, "methods": {}, "theta": {}}
        maps = {}
        for name, m in (("E", scenes.PRUNED_E), ("M", scenes.PRUNED_M), ("T", scenes.PRUNED_T)):
            r, t, st = run(with_(mode=mode, method=m))
            maps[name] = r
            d = {"ms": t, "vs_brute": t_b / t, "blocks": st["blocks"], "blocks_decided": st["blocks_decided"],
                 "traced_viewpoints": st["leaves"], "error_vs": "brute" if name == "E" else "E",
                 "error_signed": st["err_signed"], "error_abs": st["err_abs"]}
            if name != "E":
                d.update({"bound": st["bound"], "bound_measured": st["bound_measured"],
                          "bound_ratio": st["bound_measured"] / st["bound"] if st["bound"] > 0 else None})
            leg["methods"][name] = d
        for th in (2, 4, 8, 16):
            r, t, st = run(with_(mode=mode, method=scenes.PRUNED_E, theta_blocks=th))
            err = vcm.vcm_map_error(maps["E"][1], r[1])
            leg["theta"][str(th)] = {"ms": t, "vs_brute": t_b / t, "blocks": st["blocks"],
                                     "blocks_decided": st["blocks_decided"], "traced_blocks": st["leaves"],
                                     "error_signed_vs_theta1": err[0], "error_abs_vs_theta1": err[1]}
        out[mode_name] = leg
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
    # the configured arrival rates, then higher ones to find where the server
    # stops keeping up (achieved below 95 % of offered)
    for rate in (50.0, 100.0, 200.0, 500.0, 1000.0, 2000.0, 4000.0, 8000.0, 16000.0):
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
    keeps = [r["offered_req_per_s"] for r in out["rates"] if r["requests_per_s"] >= 0.95 * r["offered_req_per_s"]]
    out["saturation_req_per_s"] = max(r["requests_per_s"] for r in out["rates"])
    out["highest_rate_kept_up"] = max(keeps) if keeps else None
    return out


def bench_sweeps(cell: float = 64.0):
    """The paper's parameter sweeps (Table 2) on the synthetic 3-D city, as
    trend checks of VCM_E, VCM_M and VCM_T (FULL mode, the paper's rule):
    angular resolution mu, minimum block size theta, field of view, and the
    number of obstacles with uniform and Zipf-clustered placement.  Per
    setting: time per map of each method and of the brute force, the Sec. V-A
    error of VCM_M / VCM_T against VCM_E and of VCM_E against the brute
    force (theta: against VCM_E at theta = 1), and the visible fraction."""
    import torch
    import paper_1310_7297_amd as vcm
    from paper_1310_7297_amd import scenes

    def timed(idx, q, r):
        st = vcm.vcm_compute(idx, q, *r, stats=True)
        ms = []
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            vcm.vcm_compute(idx, q, *r)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return min(ms), st

    def with_(q, **kw):
        return scenes.Query(q.target, q.grid, scenes.Params(**{**q.params.__dict__, **kw}))

    def methods(idx, q):
        n = q.grid.count
        rb, r = vcm.alloc_result(n), {m: vcm.alloc_result(n) for m in "EMT"}
        tb, _ = timed(idx, with_(q, method=scenes.BRUTE), rb)
        out = {"brute_ms": tb}
        for m, code in (("E", scenes.PRUNED_E), ("M", scenes.PRUNED_M), ("T", scenes.PRUNED_T)):
            t, st = timed(idx, with_(q, method=code), r[m])
            out[m] = {"ms": t, "error_signed": st["err_signed"], "error_abs": st["err_abs"]}
        cnt = rb[2].cpu().numpy().view("uint16")
        out["visible_fraction"] = float((cnt > 0).mean())
        return out, r

    res = {"workload": "sweep_billboard: 4 km city, 30 x 15 m billboard, 256x256x64 viewpoints, "
                       "FOV 120 (defaults: 20,000 uniform boxes, mu 4', theta 1)", "mode": "full"}
    scene, q = scenes.sweep_billboard()
    idx = vcm.vcm_build_index(scene, cell_size=cell)
    res["mu"] = {}
    for mu in (1.0, 2.0, 4.0, 8.0, 16.0):
        res["mu"][str(int(mu))], _ = methods(idx, with_(q, mu_arcmin=mu))
    res["theta"] = {}
    _, base = methods(idx, q)
    for th in (2, 4, 8, 16):
        r = vcm.alloc_result(q.grid.count)
        t, st = timed(idx, with_(q, method=scenes.PRUNED_E, theta_blocks=th), r)
        err = vcm.vcm_map_error(base["E"][1], r[1])
        res["theta"][str(th)] = {"E_ms": t, "error_signed_vs_theta1": err[0], "error_abs_vs_theta1": err[1],
                                 "blocks": st["blocks"], "traced_viewpoints": st["leaves"]}
    res["fov"] = {}
    for fov in (60.0, 120.0, 180.0, 240.0, 300.0, 360.0):
        res["fov"][str(int(fov))], _ = methods(idx, with_(q, fov_deg=fov))
    idx.free()
    res["obstacles"] = {}
    for dist in ("uniform", "zipf"):
        for n in (5000, 10000, 15000, 20000, 25000):
            sc, qq = scenes.sweep_billboard(n, dist)
            idx = vcm.vcm_build_index(sc, cell_size=cell)
            res["obstacles"][f"{dist}_{n // 1000}k"], _ = methods(idx, qq)
            idx.free()
    return res


def bench_index():
    """Index build at scale: the 100,000-box 8 km city at column widths of 16
    to 256 m (device time of the build kernels, wall time of the whole build
    including the host's copies)."""
    import paper_1310_7297_amd as vcm
    from paper_1310_7297_amd import scenes
    scene, _ = scenes.city8km_serving(n_requests=1)
    vcm.vcm_build_index(scene, cell_size=64.0).free()    # first launch of the build kernels
    out = []
    for cs in (16.0, 32.0, 64.0, 128.0, 256.0):
        kms, wall = [], []
        for _ in range(3):
            idx = vcm.vcm_build_index(scene, cell_size=cs)
            info = idx.info()
            kms.append(info["kernel_ms"])
            wall.append(info["build_ms"])
            idx.free()
        out.append({"cell_size": cs, "columns": info["nx"] * info["ny"], "refs": info["n_refs"],
                    "longest_list": info["longest_list"], "kernel_ms": min(kms), "build_ms": min(wall),
                    "device_bytes": info["device_bytes"]})
    return {"workload": "city8km_serving scene: 100,000 boxes, 8 km", "boxes": scene.n, "cells": out}


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

    # index autotuner (untimed set-up): the fastest column width for this map,
    # reported; the timed steps use it with --cell -1, else the width given
    tuning = vcm.vcm_tune_cell_size(scene, [q], cell_min=32.0, cell_max=256.0, reps=1)
    cell = tuning["best_cell"] if args.cell < 0 else args.cell
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

    # the timed map, for the comparison with the oracle below
    gmap = {"bin": bufs[0].cpu().numpy(), "c": bufs[1].cpu().numpy(),
            "count": bufs[2].cpu().numpy().view(np.uint16)}

    rl = roofline_of(st, kernel_ms)
    hw = None
    if profile_valid(args.workload, info["cell_size"]):
        valu = PROFILE_VALU[args.mode]
        hw = {"valu_issue_per_cu_clock": valu / (CUS * kernel_ms * 1e-3 * CLOCK),
              "source": "SQ_INSTS_VALU of the committed profile (same kernel sources)"}
    roofline = {"bound": "alu", "achieved": rl["achieved"], "peak": PEAK_LANE_OPS / 1e12,
                "unit": "Tlane-op/s", "frac": rl["frac"],
                "traffic": measured_traffic(args.workload, args.mode, info["cell_size"]),
                "kernel": "k_brute", "kernel_ms": kernel_ms,
                "work": "20 lane-ops per float32 slab test + 12 per corridor column, per launch",
                "lane_ops_per_launch": rl["lane_ops_per_launch"],
                "with_culling": rl["with_culling"], "hardware": hw,
                "box_tests_per_launch": st["box_tests"], "columns_per_launch": st["columns"],
                "rechecks_per_launch": st["rechecks"],
                "records_per_launch": st["records"], "narrow_tests_per_launch": st["narrow_tests"],
                "slot_tests_per_launch": st.get("slot_tests"),
                "open_lanes_per_slot_test": st["box_tests"] / max(1, st["slot_tests"]),
                "inside_box_viewpoints": st.get("inside_box"),
                "hbm_bytes_algorithmic": 7 * n_vp,
                "hbm_frac": 7 * n_vp / (kernel_ms * 1e-3) / PEAK_HBM}

    extra = {}
    if not args.no_extra:
        # the other mode (FULL: the paper's complete-visibility rule) beside it,
        # with its own useful-work fraction
        qf = scenes.Query(q.target, q.grid, scenes.Params(**{**q.params.__dict__, "mode":
                                                              scenes.FULL if mode == scenes.FRACTION
                                                              else scenes.FRACTION}))
        st2 = vcm.vcm_compute(idx, qf, *bufs, stats=True)
        w2, k2 = timed_steps(vcm, idx, qf, bufs, max(2, args.steps // 2), 1)
        rl2 = roofline_of(st2, float(np.mean(k2)))
        other = "full" if mode == scenes.FRACTION else "fraction"
        hw2 = None
        if profile_valid(args.workload, info["cell_size"]):
            hw2 = PROFILE_VALU[other] / (CUS * float(np.mean(k2)) * 1e-3 * CLOCK)
        extra["other_mode"] = {"mode": other, "valu_issue_per_cu_clock": hw2,
                               "viewpoints_per_s": n_vp * max(2, args.steps // 2) / w2,
                               "kernel_ms": float(np.mean(k2)), "roofline_frac": rl2["frac"],
                               "roofline_frac_with_culling": rl2["with_culling"]["frac"],
                               "box_tests_per_launch": st2["box_tests"], "columns_per_launch": st2["columns"]}

    if not (args.no_pruned or args.no_extra) and args.workload == "cube":
        extra["pruned"] = bench_pruned(vcm, idx, q)
        for mname, leg in extra["pruned"].items():
            print(f"pruned ({mname}): brute {leg['brute_ms']:.2f} ms, " +
                  ", ".join(f"{k} {v['ms']:.2f} ms" for k, v in leg["methods"].items()),
                  file=sys.stderr, flush=True)
    config_samples = []
    if not (args.no_configs or args.no_extra):
        extra["configs"], config_samples = bench_configs(max(2, args.steps // 2))
        print("configs: " + ", ".join(f"{k} {v['full']['viewpoints_per_s'] / 1e6:.0f} M vp/s (full)"
                                      for k, v in extra["configs"].items()), file=sys.stderr, flush=True)
    if not (args.no_index or args.no_extra):
        extra["index_build"] = bench_index()
    if not (args.no_sweeps or args.no_extra):
        extra["sweeps"] = bench_sweeps()
        print("sweeps: done", file=sys.stderr, flush=True)
    if not (args.no_batch or args.no_extra):
        extra["batch"] = bench_batch()
        print(f"batch: {extra['batch']['speedup_vs_sequential']:.2f}x sequential", file=sys.stderr,
              flush=True)
    if not (args.no_serve or args.no_extra):
        extra["serving"] = bench_serve(args.serve_requests)

    cpu = None
    agreement = None
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
        # the timed map's error against the float64 oracle on that sample
        agreement = oracle_agreement({k: v[vp] for k, v in gmap.items()}, o, q.params.n_bins)
        # the same oracle split over all the host's cores (reported beside it)
        ncores = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        oracle.vcm_eval(scene, q, vp, nthreads=ncores)
        dt_all = time.perf_counter() - t0
        extra["cpu_baseline_all_cores"] = {"value": len(vp) / dt_all, "unit": "viewpoints/s",
                                           "cores": ncores, "nproc": os.cpu_count(), "kind": "oracle",
                                           "sample": f"the same {len(vp)} viewpoints, {ncores} threads"}
        # the smaller configurations' maps against the oracle on their samples
        for leg, sc, qc, vpc, gs in config_samples:
            leg["oracle_agreement"] = oracle_agreement(gs, oracle.vcm_eval(sc, qc, vpc, nthreads=ncores),
                                                       qc.params.n_bins)

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
        "oracle_agreement": agreement,
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
