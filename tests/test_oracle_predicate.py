"""Pins of the oracle's point-to-point visibility test (Def. 2.2, Def. 3.1).

The oracle intersects per-axis parameter intervals; the reference used here
is the separating-axis theorem on integer quanta (tests/independent.py)."""
import itertools

import numpy as np
import pytest

import oracle
from independent import seg_box_sat


def _lattice_cases(rng, n, dim, span=6, step=0.5):
    pts = lambda: rng.integers(-span, span + 1, dim) * step
    for _ in range(n):
        a, b = pts(), pts()
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        yield pts(), pts(), lo, hi


@pytest.mark.parametrize("dim", [2, 3])
def test_matches_separating_axis_reference(dim):
    """Coarse lattice coordinates make grazing contacts (rays in face planes,
    through edges and corners, endpoints on faces) common."""
    rng = np.random.default_rng(17 + dim)
    hits = 0
    for q, s, lo, hi in _lattice_cases(rng, 20000, dim):
        a = oracle.segment_meets_box(q, s, lo, hi, dim=dim)
        b = seg_box_sat(dim, q, s, lo, hi)
        assert a == int(b), (q, s, lo, hi)
        hits += a
    assert 2000 < hits < 18000


@pytest.mark.parametrize("dim", [2, 3])
def test_endpoint_symmetry(dim):
    """Visibility is symmetric (Sec. III-A): pred(q, s) == pred(s, q)."""
    rng = np.random.default_rng(5)
    for q, s, lo, hi in _lattice_cases(rng, 5000, dim):
        assert oracle.segment_meets_box(q, s, lo, hi, dim) == oracle.segment_meets_box(s, q, lo, hi, dim)


def test_hand_cases():
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    f = lambda q, s: oracle.segment_meets_box(q, s, lo, hi, 3)
    assert f((-1, 0.5, 0.5), (2, 0.5, 0.5)) == 1        # straight through
    assert f((-1, 1.0, 0.5), (2, 1.0, 0.5)) == 1        # lies in a face plane: touches
    assert f((-1, 1.0, 1.0), (2, 1.0, 1.0)) == 1        # along an edge
    assert f((-1, -1, -1), (2, 2, 2)) == 1              # through two corners
    assert f((-1, 0.0, 0.5), (1, 2.0, 0.5)) == 1        # grazes the edge x=0,y=1
    assert f((-1, 1.0, 0.5), (1, 3.0, 0.5)) == 0        # parallel line above it
    assert f((-1, 1.00390625, 0.5), (2, 1.00390625, 0.5)) == 0  # one quantum above
    assert f((-2, 0.5, 0.5), (0, 0.5, 0.5)) == 1        # ends on the face
    assert f((-2, 0.5, 0.5), (-0.00390625, 0.5, 0.5)) == 0      # stops one quantum short
    assert f((0.5, 0.5, 0.5), (0.5, 0.5, 0.5)) == 1     # degenerate inside
    assert f((0.5, 0.5, 1.5), (0.5, 0.5, 1.5)) == 0     # degenerate outside
    assert f((0.5, 0.5, 0.5), (5, 5, 5)) == 1           # starts inside: blocked
    assert f((-1, 2, 0.5), (2, -1, 0.5)) == 1           # diagonal across
    assert f((-1, 3.0, 0.5), (3, -1.0, 0.5)) == 1       # touches the edge x=y=1
    assert f((-1, 3.00390625, 0.5), (3, -0.99609375, 0.5)) == 0  # passes it by a quantum


def test_rejects_non_dyadic():
    with pytest.raises(ValueError):
        oracle.segment_meets_box((0.1, 0, 0), (1, 1, 1), (0, 0, 0), (1, 1, 1))
