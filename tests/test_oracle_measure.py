"""Pins of the oracle's visibility measure (Eq. 1, Eq. 2) and colour bins."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1310_7297_amd.scenes import (BILLBOARD, CUBE, SEGMENT, BIN_LOG, Params,
                                         Target)

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def _targets(S):
    return [
        Target(SEGMENT, (0.0, 0.0, 0.0), (S, 0.0), normal_axis=1, samples_u=8, samples_v=1),
        Target(BILLBOARD, (0.0, 0.0, 0.0), (S, S / 2), normal_axis=1, samples_u=8, samples_v=4),
        Target(CUBE, (0.0, 0.0, 0.0), (S, 0.0), samples_u=4, samples_v=4),
    ]


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_worked_example(kind):
    """V = 41.11 deg facing and 21.23 deg at 45 degrees (Sec. II-B example)."""
    g = json.load(open(GOLD))
    t = _targets(g["S"])[kind]
    for case in g["cases"]:
        a = math.radians(case["alpha_deg"])
        D = g["D"]
        # line of sight at angle alpha to the target plane, in the plane z = 0
        q = (D * math.cos(a), D * math.sin(a), 0.0)
        m = oracle.measure(t, Params(), q)
        assert abs(m["D"] - D) < 1e-9
        assert abs(math.degrees(m["alpha"]) - case["alpha_deg"]) < 1e-9
        assert abs(math.degrees(m["V"]) - case["V_deg"]) < 0.01


def test_measure_monotone_in_distance_and_angle():
    t = _targets(30.0)[0]
    p = Params()
    prev = None
    for D in np.linspace(1.0, 5000.0, 200):
        V = oracle.measure(t, p, (0.0, D, 0.0))["V"]
        if prev is not None:
            assert V < prev
        prev = V
    prev = None
    for a in np.linspace(0.0, math.pi / 2, 91):
        V = oracle.measure(t, p, (100 * math.cos(a), 100 * math.sin(a), 0.0))["V"]
        if prev is not None:
            assert V > prev
        prev = V
    # edge-on: no perceived size
    assert oracle.measure(t, p, (100.0, 0.0, 0.0))["V"] == 0.0


def test_near_point_floor():
    """Closer than the near point d0 the lens cannot focus (Sec. III-A-1):
    the visual angle is capped at V0 = 2 arctan(S / 2 d0), so c = 1."""
    t = _targets(40.0)[0]
    p = Params(near_d0=0.25)
    for d in (0.125, 0.25, 0.0625):
        m = oracle.measure(t, p, (0.0, d, 0.0))
        assert m["V"] == m["V0"]
    m = oracle.measure(t, p, (0.0, 0.5, 0.0))
    assert m["V"] < m["V0"]


def test_reflection_symmetry():
    """The partition (and the measure) is symmetric about the target's
    parallel and normal axes (Sec. III-A-2)."""
    rng = np.random.default_rng(0)
    for t in _targets(12.0):
        for _ in range(50):
            q = rng.uniform(-300, 300, 3)
            if t.kind == SEGMENT:
                q[2] = 0
            V = oracle.measure(t, Params(), q)["V"]
            for flip in ([-1, 1, 1], [1, -1, 1], [1, 1, -1]):
                V2 = oracle.measure(t, Params(), q * np.array(flip))["V"]
                assert abs(V - V2) <= 1e-15 * max(1.0, V)


def test_cube_axis_choice():
    """Cube: the face axis is the one of largest |Delta|; from the +x axis the
    target is seen face-on, along a face diagonal at 45 degrees."""
    t = _targets(300.0)[2]
    m = oracle.measure(t, Params(), (400.0, 0.0, 0.0))
    assert abs(math.degrees(m["alpha"]) - 90.0) < 1e-12
    m = oracle.measure(t, Params(), (0.0, 0.0, -400.0))
    assert abs(math.degrees(m["alpha"]) - 90.0) < 1e-12
    m = oracle.measure(t, Params(), (400.0, 0.0, 400.0))
    assert abs(math.degrees(m["alpha"]) - 45.0) < 1e-12


def _one_vp_eval(t, p, q, dim):
    """Oracle at a single viewpoint, through a one-cell grid centred on q."""
    from paper_1310_7297_amd.scenes import Grid, Query, Scene
    ext = 1.0
    g = Grid((q[0] - 0.5, q[1] - 0.5, q[2] - 0.5 if dim == 3 else 0.0),
             (ext, ext, ext if dim == 3 else 0.0), (1, 1, 1))
    s = Scene(dim, np.zeros((3, 0)), np.zeros((3, 0)))
    return oracle.vcm_eval(s, Query(t, g, p))


def test_bins_linear_and_log():
    t = Target(SEGMENT, (0.0, 0.0, 0.0), (40.0, 0.0), normal_axis=1, samples_u=32, samples_v=1)
    # inside the near point, facing: c = 1 lands in the last bin
    for B in (2, 8, 16, 256):
        o = _one_vp_eval(t, Params(n_bins=B), (0.0, 0.125, 0.0), 2)
        assert o["c"][0] == 1.0 and o["bin"][0] == B - 1
    # far away: c small -> bin floor(c B)
    o = _one_vp_eval(t, Params(n_bins=16), (0.0, 100.0, 0.0), 2)
    assert o["bin"][0] == int(o["c"][0] * 16)
    # log scale: V0 maps to 1, mu maps to 0
    o = _one_vp_eval(t, Params(n_bins=16, bin_scale=BIN_LOG), (0.0, 0.125, 0.0), 2)
    assert o["cb"][0] == 1.0 and o["bin"][0] == 15
    small = Target(SEGMENT, (0.0, 0.0, 0.0), (4.0, 0.0), normal_axis=1, samples_u=8, samples_v=1)
    mu = 4.0 / 60.0 * math.pi / 180.0
    d_mu = 2.0 / math.tan(mu / 2)   # distance at which V = mu (Sec. IV-B)
    far = float(np.round(2 * d_mu * 256) / 256)
    o = _one_vp_eval(small, Params(n_bins=16, bin_scale=BIN_LOG), (0.0, far, 0.0), 2)
    assert o["c"][0] > 0.0 and o["cb"][0] == 0.0 and o["bin"][0] == 0
    near = float(np.round(0.5 * d_mu * 256) / 256)
    o = _one_vp_eval(small, Params(n_bins=16, bin_scale=BIN_LOG), (0.0, near, 0.0), 2)
    assert 0.0 < o["cb"][0] < 1.0
