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

# Algorithmic VALU lane-operations per unit of work (see the design notes):
# one float32 slab test of a ray against a box, and one corridor column visit.
OPS_PER_BOX_TEST = 20
OPS_PER_COLUMN = 12
# MI355X: 256 CUs x 4 SIMD x 16 lanes per clock x 2.4 GHz (non-packed lane ops).
PEAK_LANE_OPS = 256 * 64 * 2.4e9
PEAK_HBM = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3, choices=(2, 3))
    ap.add_argument("--mode", default="fraction", choices=("fraction", "full"))
    ap.add_argument("--cell", type=float, default=0.0)
    ap.add_argument("--cpu-sample", type=int, default=16384)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
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


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by viewpoint tiles with no exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1310_7297_amd as vcm
    from paper_1310_7297_amd import scenes

    cfg = scenes.config3 if args.config == 3 else scenes.config2
    scene, q = cfg()
    mode = scenes.FRACTION if args.mode == "fraction" else scenes.FULL
    q.params.mode = mode
    n_vp = q.grid.count

    t0 = time.perf_counter()
    idx = vcm.vcm_build_index(scene, cell_size=args.cell)
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

    ops = OPS_PER_BOX_TEST * st["box_tests"] + OPS_PER_COLUMN * st["columns"]
    achieved = ops / (kernel_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                "unit": "Tlane-op/s", "frac": achieved / PEAK_LANE_OPS, "traffic": None,
                "kernel": "k_brute", "kernel_ms": kernel_ms,
                "box_tests_per_launch": st["box_tests"], "columns_per_launch": st["columns"],
                "rechecks_per_launch": st["rechecks"],
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
        "config": {"workload": f"config{args.config}: "
                   + ("4 km city, 20,000 boxes, 30 m cube 8x8/face, 256x256x64 viewpoints"
                      if args.config == 3 else
                      "2 km city, 5,000 boxes, 10x5 m billboard 16x8, 128x128x32 viewpoints"),
                   "mode": args.mode, "viewpoints": n_vp, "boxes": scene.n, "n_bins": q.params.n_bins,
                   "cell_size": info["cell_size"], "parallelism": "single-gpu"},
        "rays_per_s": rays_ps,
        "rays_per_step": st["rays"],
        "index": {"build_s": build_s, "device_bytes": info["device_bytes"], "refs": info["n_refs"],
                  "columns": [info["nx"], info["ny"]]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
