"""Independent exact formulations used to pin the oracle (tests only).

These follow different algorithms from the oracle's, so that a slip in one is
unlikely to be repeated in the other:
  * segment/box contact by the separating-axis theorem on integer quanta
    (the oracle intersects per-axis parameter intervals instead);
  * target samples enumerated from the facet definitions with numpy.
"""
from fractions import Fraction

import numpy as np


def q(x):
    """Exact integer quanta of a multiple of 2^-8."""
    y = Fraction(x) * 256
    assert y.denominator == 1, x
    return int(y)


def seg_box_sat(dim, p0, p1, lo, hi):
    """Closed segment [p0,p1] vs closed box [lo,hi], exact, by separating axes.

    Candidate axes: the box face normals and the cross products of the segment
    direction with the box edge directions (3-D), or the segment's normal (2-D).
    Disjoint iff some axis separates the projections strictly."""
    P0 = [q(v) for v in p0[:dim]]
    P1 = [q(v) for v in p1[:dim]]
    L = [q(v) for v in lo[:dim]]
    H = [q(v) for v in hi[:dim]]
    d = [P1[k] - P0[k] for k in range(dim)]
    axes = []
    for k in range(dim):
        e = [0] * dim
        e[k] = 1
        axes.append(e)
    if dim == 3:
        for k in range(3):
            e = [0, 0, 0]
            e[k] = 1
            cr = [d[1] * e[2] - d[2] * e[1], d[2] * e[0] - d[0] * e[2], d[0] * e[1] - d[1] * e[0]]
            if any(cr):
                axes.append(cr)
    else:
        nrm = [-d[1], d[0]]
        if any(nrm):
            axes.append(nrm)
    for a in axes:
        s0 = sum(a[k] * P0[k] for k in range(dim))
        s1 = sum(a[k] * P1[k] for k in range(dim))
        bmin = sum(min(a[k] * L[k], a[k] * H[k]) for k in range(dim))
        bmax = sum(max(a[k] * L[k], a[k] * H[k]) for k in range(dim))
        if max(s0, s1) < bmin or bmax < min(s0, s1):
            return False
    return True


def visible_count(dim, lo, hi, q_pt, samples):
    """Number of samples whose segment from q_pt meets no box (exact, SAT)."""
    n = 0
    for s in samples:
        ok = True
        for b in range(lo.shape[1]):
            if seg_box_sat(dim, q_pt, s, lo[:, b], hi[:, b]):
                ok = False
                break
        n += ok
    return n
