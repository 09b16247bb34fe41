"""Pins of the oracle's visible-region blocks (Sec. III-C-1): a block of
viewpoints is decided as a whole when the target is completely seen from all
of it or from none of it, else split down to the minimum block size, whose
undecided blocks take their representative's visibility."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1310_7297_amd import scenes
from paper_1310_7297_amd.scenes import (BILLBOARD, CUBE, FRACTION, FULL, SEGMENT, Grid, Params,
                                         Query, Scene, Target)


def _lattice(rng, n, step, extent):
    return rng.integers(0, int(extent / step) + 1, size=n) * step


def test_hull_of_a_point_block_is_the_segment_test():
    """With the block shrunk to one viewpoint q, the hull of the block and a
    sample s is the segment [q, s]: the test reduces to the exact segment
    predicate (grazing-heavy lattice cases)."""
    rng = np.random.default_rng(1)
    n = 0
    for _ in range(3000):
        dim = 2 if rng.random() < 0.3 else 3
        q = _lattice(rng, 3, 1.0, 8.0)
        s = _lattice(rng, 3, 1.0, 8.0)
        a = _lattice(rng, 3, 1.0, 8.0)
        c = a + _lattice(rng, 3, 1.0, 3.0)
        if dim == 2:
            q[2] = s[2] = a[2] = c[2] = 0.0
        want = oracle.segment_meets_box(q, s, a, c, dim=dim)
        assert oracle.hull_meets_box(q, q, s, a, c, dim=dim) == bool(want)
        n += want
    assert 150 < n < 2850


def _lp_meets(L, H, s, a, c, dim):
    """Feasibility of: lambda in [0, 1], u = lambda p with p in [L, H], and
    s + lambda (p - s) = s (1 - lambda) + u in [a, c]; variables (lambda, u)."""
    from scipy.optimize import linprog
    A, b = [], []
    for k in range(dim):
        row = np.zeros(dim + 1)
        row[0], row[1 + k] = L[k], -1.0          # lambda L_k - u_k <= 0
        A.append(row); b.append(0.0)
        row = np.zeros(dim + 1)
        row[0], row[1 + k] = -H[k], 1.0          # u_k - lambda H_k <= 0
        A.append(row); b.append(0.0)
        row = np.zeros(dim + 1)
        row[0], row[1 + k] = s[k], -1.0          # a_k <= s_k (1 - lambda) + u_k
        A.append(row); b.append(s[k] - a[k])
        row = np.zeros(dim + 1)
        row[0], row[1 + k] = -s[k], 1.0          # s_k (1 - lambda) + u_k <= c_k
        A.append(row); b.append(c[k] - s[k])
    bounds = [(0.0, 1.0)] + [(None, None)] * dim
    r = linprog(np.zeros(dim + 1), A_ub=np.array(A), b_ub=np.array(b), bounds=bounds, method="highs")
    return r.status == 0


def test_hull_test_matches_a_linear_program():
    """The box meets the hull of a block and a point exactly when a linear
    program over (lambda, lambda p) is feasible; cases the program cannot
    settle within its tolerance (the box grown or shrunk by 1e-4 answers
    differently) are skipped."""
    rng = np.random.default_rng(2)
    checked = hits = 0
    for _ in range(1500):
        dim = 2 if rng.random() < 0.3 else 3
        L = _lattice(rng, 3, 0.5, 16.0)
        H = L + _lattice(rng, 3, 0.5, 6.0)
        s = _lattice(rng, 3, 0.5, 16.0)
        if rng.random() < 0.5:
            a = _lattice(rng, 3, 0.5, 16.0)
        else:   # a box around a lattice point near the hull
            x = s + rng.random() * (rng.uniform(L, H) - s)
            a = np.round(x * 2) / 2 - _lattice(rng, 3, 0.5, 1.0)
        c = a + _lattice(rng, 3, 0.5, 4.0)
        if dim == 2:
            for v in (L, H, s, a, c):
                v[2] = 0.0
        grow = _lp_meets(L, H, s, a - 1e-4, c + 1e-4, dim)
        shrink = _lp_meets(L, H, s, a + 1e-4, c - 1e-4, dim) if np.all(c - a > 2e-4) else False
        if grow != shrink:
            continue
        assert oracle.hull_meets_box(L, H, s, a, c, dim=dim) == grow, (L, H, s, a, c, dim)
        checked += 1
        hits += grow
    assert checked > 1000 and 100 < hits < checked - 100


def _tiny_scene(seed):
    """Grazing-heavy boxes on a 2 m lattice around a target at the centre."""
    dim = 2 if seed % 4 == 0 else 3
    sc = scenes.random_boxes(8, seed, extent=32.0, max_side=8.0, dim=dim, grid_step=2.0)
    if dim == 2:
        t = Target(SEGMENT, (16.0, 16.0, 0.0), (4.0, 0.0), normal_axis=seed % 2, samples_u=4, samples_v=1)
        g = Grid((0.0, 0.0, 0.0), (32.0, 32.0, 0.0), (16, 16, 1))
    elif seed % 4 == 1:
        t = Target(BILLBOARD, (16.0, 16.0, 4.0), (4.0, 2.0), normal_axis=seed % 2, samples_u=4,
                   samples_v=2, normal_sign=1 if seed % 8 < 4 else -1)
        g = Grid((0.0, 0.0, 0.0), (32.0, 32.0, 16.0), (16, 16, 8))
    else:
        t = Target(CUBE, (16.0, 16.0, 4.0), (4.0, 0.0), samples_u=2, samples_v=2)
        g = Grid((0.0, 0.0, 0.0), (32.0, 32.0, 16.0), (16, 16, 8))
    tlo, thi = t.aabb()
    ov = np.ones(sc.n, bool)
    for k in range(dim):
        ov &= (sc.lo[k] <= thi[k]) & (sc.hi[k] >= tlo[k])
    return Scene(dim, sc.lo[:, ~ov], sc.hi[:, ~ov]), t, g


@pytest.mark.parametrize("mode", [FULL, FRACTION])
def test_decided_blocks_agree_with_brute_force_everywhere(mode):
    """A decided block gives every one of its viewpoints exactly the count,
    live count and field of view the brute-force oracle gives it; blocks of
    every kind of decision occur."""
    rng = np.random.default_rng(3 + mode)
    kinds = {"seen": 0, "hidden": 0, "outside": 0, "undecided": 0, "partial": 0}
    for seed in range(24):
        sc, t, g = _tiny_scene(seed)
        fov = 360.0 if t.kind == CUBE else [360.0, 120.0, 180.0, 240.0][seed % 4]
        q = Query(t, g, Params(n_bins=16, mode=mode, fov_deg=fov))
        full = oracle.vcm_eval(sc, q, nthreads=4)
        n = np.array(g.n)
        for _ in range(40):
            side = int(rng.choice([1, 2, 4, 8]))
            lo = np.array([rng.integers(0, n[k]) for k in range(3)])
            lo = lo // side * side
            hi = np.minimum(lo + side - 1, n - 1)
            if sc.dim == 2:
                lo[2] = hi[2] = 0
            r = oracle.classify_block(sc, q, lo[:sc.dim], hi[:sc.dim])
            if r is None:
                kinds["undecided"] += 1
                continue
            cnt, N, inf = r
            rng_idx = [np.arange(lo[k], hi[k] + 1) for k in range(3)]
            for i, j, k in itertools.product(*rng_idx):
                v = i + n[0] * (j + n[1] * k)
                assert full["count"][v] == cnt and full["nlive"][v] == N and full["infov"][v] == inf, \
                    (seed, lo, hi, r, v, full["count"][v], full["nlive"][v], full["infov"][v])
            if not inf or N == 0:
                kinds["outside"] += 1
            elif cnt == N:
                kinds["seen"] += 1
            elif cnt == 0:
                kinds["hidden"] += 1
            else:
                kinds["partial"] += 1
    assert kinds["seen"] > 20 and kinds["hidden"] > 20 and kinds["undecided"] > 20, kinds
    if mode == FRACTION:
        assert kinds["partial"] > 5, kinds


def test_block_hand_cases():
    t = Target(BILLBOARD, (0.0, 0.0, 5.0), (8.0, 4.0), normal_axis=1, samples_u=8, samples_v=4)
    g = Grid((-32.0, -64.0, 0.0), (64.0, 128.0, 32.0), (16, 32, 8))   # 4 m steps
    empty = Scene(3, np.zeros((3, 0)), np.zeros((3, 0)))
    wall = Scene(3, np.array([[-50.0], [20.0], [0.0]]), np.array([[50.0], [22.0], [60.0]]))
    pole = Scene(3, np.array([[-0.5], [24.0], [0.0]]), np.array([[0.5], [25.0], [60.0]]))
    behind = Scene(3, np.array([[-50.0], [-30.0], [0.0]]), np.array([[50.0], [-28.0], [60.0]]))
    q = Query(t, g, Params(mode=FULL))
    front = ([4, 24, 0], [7, 27, 3])      # y from 32 to 44: beyond the wall at y = 20..22
    # nothing in the way: every block sees all 32 samples
    assert oracle.classify_block(empty, q, *front) == (32, 32, 1)
    # a wall between the block and the target hides it from all of the block
    assert oracle.classify_block(wall, q, *front) == (0, 32, 1)
    # a thin pole in front of the target hides some samples from some viewpoints
    assert oracle.classify_block(pole, q, *front) is None
    # a wall behind the block (the target on the other side) does not matter
    other = ([4, 24, 0], [7, 27, 3])
    assert oracle.classify_block(behind, q, *other) == (32, 32, 1)
    # a field of view of 180 degrees: blocks fully behind the target plane are
    # out, blocks across it are undecided
    q180 = Query(t, g, Params(mode=FULL, fov_deg=180.0))
    assert oracle.classify_block(empty, q180, [4, 2, 0], [7, 5, 3]) == (0, 32, 0)
    assert oracle.classify_block(empty, q180, [4, 14, 0], [7, 17, 3]) is None
    # a 240-degree field of view is not convex: a block behind the target whose
    # corners are all inside the wedge can hold viewpoints outside it
    q240 = Query(t, Grid((-44.0, -24.0, 0.0), (88.0, 8.0, 8.0), (11, 1, 1)), Params(mode=FULL, fov_deg=240.0))
    assert oracle.in_fov(t, q240.params, (40.0, -20.0, 4.0)) and not oracle.in_fov(t, q240.params, (0.0, -20.0, 4.0))
    assert oracle.classify_block(empty, q240, [0, 0, 0], [10, 0, 0]) is None
    assert oracle.classify_block(empty, q240, [5, 0, 0], [5, 0, 0]) == (0, 32, 0)
    # a block containing a viewpoint on the wall's face plane is still hidden
    qf = Query(t, Grid((-32.0, 21.0, 0.0), (64.0, 4.0, 32.0), (16, 2, 8)), Params(mode=FULL))
    assert oracle.classify_block(wall, qf, [0, 0, 0], [3, 1, 3]) == (0, 32, 1)
    # FRACTION mode: the pole hides a fixed subset of samples from a small
    # block straight behind it
    qr = Query(t, g, Params(mode=FRACTION))
    assert oracle.classify_block(pole, qr, *front) is None
    # cube: a block across a face plane sees different faces: undecided
    tc = Target(CUBE, (0.0, 0.0, 4.0), (4.0, 0.0), samples_u=2, samples_v=2)
    gc = Grid((-16.0, -16.0, 0.0), (32.0, 32.0, 32.0), (8, 8, 8))     # 4 m steps, z centres 2..30
    qc = Query(tc, gc, Params(mode=FULL))
    assert oracle.classify_block(empty, qc, [6, 6, 2], [7, 7, 3]) == (12, 12, 1)   # three faces
    assert oracle.classify_block(empty, qc, [3, 6, 2], [4, 7, 3]) == (8, 8, 1)     # x = -2, 2: on the planes
    assert oracle.classify_block(empty, qc, [2, 6, 2], [3, 7, 3]) is None         # x = -6, -2: across x = -2


@pytest.mark.parametrize("theta", [2, 4])
@pytest.mark.parametrize("mode", [FULL, FRACTION])
def test_pruned_gate_is_brute_force_where_decided_and_the_representative_elsewhere(theta, mode):
    sc, t, g = _tiny_scene(5)
    q = Query(t, g, Params(n_bins=16, mode=mode, method=1, theta_blocks=theta))
    vp = np.arange(g.count, dtype=np.int64)
    p = oracle.vcm_eval_pruned(sc, q, 1, theta, vp, nthreads=4)
    b = oracle.vcm_eval(sc, q, nthreads=4)
    reps = np.array([oracle.block_rep(g, 3, theta, v) for v in vp])
    dec = p["decided"].astype(bool)
    assert 0.2 < dec.mean() < 0.98
    assert np.array_equal(p["count"][dec], b["count"][dec])
    assert np.array_equal(p["count"][~dec], b["count"][reps[~dec]])
    # hence the whole map is every smallest block's representative's gate:
    # a decided block gives its representatives the gate it gives the block,
    # so the map does not depend on which levels of the tree are classified
    assert np.array_equal(p["count"], b["count"][reps])
