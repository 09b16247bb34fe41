"""Seeded mixed workload shared by the batch and serving tests: a small city
with billboards and cubes, and queries of every kind, mode, method and
precision over ragged and single-viewpoint grids."""
import numpy as np

import paper_1310_7297_amd as vcm
from paper_1310_7297_amd import scenes
from paper_1310_7297_amd.scenes import (BILLBOARD, BIN_LOG, BRUTE, CUBE, FRACTION, FULL, PRUNED_E,
                                         PRUNED_M, PRUNED_T, Grid, Params, Query, Target)


def mixed_scene():
    targets = [
        Target(BILLBOARD, (96.0, 160.0, 6.0), (8.0, 4.0), normal_axis=0, normal_sign=1,
               samples_u=8, samples_v=4),
        Target(BILLBOARD, (300.0, 220.0, 9.0), (12.0, 6.0), normal_axis=1, normal_sign=-1,
               samples_u=16, samples_v=8),
        Target(CUBE, (256.0, 256.0, 5.0), (10.0, 0.0), samples_u=8, samples_v=8),
        Target(CUBE, (400.0, 96.0, 4.0), (8.0, 0.0), samples_u=4, samples_v=4),
        Target(CUBE, (128.0, 400.0, 8.0), (16.0, 0.0), samples_u=16, samples_v=8),
    ]
    scene = scenes.city(512.0, 160, seed=21, side=(6.0, 30.0), targets=targets, clearance=2.0)
    scene = scenes.Scene(3, scene.lo, np.vstack([scene.hi[:2], np.minimum(scene.hi[2], 16.0)]))
    return scene, targets


def mixed_queries(targets):
    grids = [((0.0, 0.0, 0.0), (512.0, 512.0, 64.0), (32, 32, 8)),
             ((64.0, 64.0, 0.0), (208.0, 112.0, 40.0), (13, 7, 5)),
             ((0.0, 0.0, 0.0), (512.0, 512.0, 128.0), (64, 64, 4)),
             ((200.0, 200.0, 0.0), (128.0, 128.0, 16.0), (1, 1, 1)),
             ((0.0, 128.0, 0.0), (480.0, 288.0, 48.0), (40, 24, 6))]
    qs, prec = [], []
    rng = np.random.default_rng(5)
    methods = [BRUTE, BRUTE, PRUNED_E, PRUNED_M, PRUNED_T]
    for i in range(15):
        t = targets[i % len(targets)]
        o, e, n = grids[(i * 3) % len(grids)]
        m = methods[i % len(methods)]
        p = Params(n_bins=16, mode=FRACTION if i % 2 else FULL, method=m,
                   theta_blocks=1 + (i % 3 == 2), bin_scale=BIN_LOG if i % 4 == 1 else 0,
                   fov_deg=360.0 if t.kind == CUBE or i % 3 else 120.0)
        qs.append(Query(t, Grid(o, e, n), p))
        prec.append(vcm.VCM_FP64 if rng.random() < 0.25 else vcm.VCM_FP32_RECHECK)
    return qs, prec


