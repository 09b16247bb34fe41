"""Comparison of the HIP path's outputs with the oracle's, to the stated bar:
visible counts bit-exact; colour bins bit-exact except where the oracle's
colour (in the bin's scale) lies within 1e-6 of an interior bin edge; colours within
1e-5 relative of the oracle's, with an absolute floor of 1e-9."""
import math

import numpy as np

from paper_1310_7297_amd import scenes

C_REL = 1e-5
C_ABS = 1e-9
EDGE = 1e-6


def near_edge(cb, n_bins):
    """Colours (in the bin's scale) within 1e-6 of an interior bin edge k/B,
    0 < k < B: only there can two correct roundings fall in different bins
    (0 and 1 decide no bin: bin = min(B - 1, floor(c B)))."""
    x = np.asarray(cb, dtype=np.float64) * n_bins
    k = np.round(x)
    return (np.abs(x - k) < EDGE * n_bins) & (k >= 1) & (k <= n_bins - 1)


def compare(gpu, orc, n_bins, idx=None, label=""):
    """gpu: dict of full-map arrays; orc: oracle dict at `idx` (or full map)."""
    g_bin, g_c, g_cnt = gpu["bin"], gpu["c"], gpu["count"]
    if idx is not None:
        g_bin, g_c, g_cnt = g_bin[idx], g_c[idx], g_cnt[idx]
    bad_cnt = np.nonzero(g_cnt.astype(np.int64) != orc["count"].astype(np.int64))[0]
    assert bad_cnt.size == 0, f"{label}: {bad_cnt.size} count mismatches, first at {bad_cnt[:5]}: " \
        f"gpu {g_cnt[bad_cnt[:5]]} oracle {orc['count'][bad_cnt[:5]]}"
    edge = near_edge(orc["cb"], n_bins)
    bad_bin = np.nonzero((g_bin != orc["bin"]) & ~edge)[0]
    assert bad_bin.size == 0, f"{label}: {bad_bin.size} bin mismatches at {bad_bin[:5]}: " \
        f"gpu {g_bin[bad_bin[:5]]} oracle {orc['bin'][bad_bin[:5]]} cb {orc['cb'][bad_bin[:5]]}"
    err = np.abs(g_c.astype(np.float64) - orc["c"])
    tol = C_REL * np.abs(orc["c"]) + C_ABS
    bad_c = np.nonzero(err > tol)[0]
    assert bad_c.size == 0, f"{label}: {bad_c.size} colour mismatches at {bad_c[:5]}: " \
        f"gpu {g_c[bad_c[:5]]} oracle {orc['c'][bad_c[:5]]}"
    return {"n": int(len(orc["count"])), "edge_skipped": int(edge.sum()),
            "max_rel_c": float(np.max(err / np.maximum(np.abs(orc["c"]), 1e-30), initial=0.0))}


METHOD = {1: "E", 2: "M", 3: "T"}


def target_cells(query):
    """The oracle's cells for a query (a viewer's: rings alone, of the size
    whose visual angle at d_max is mu)."""
    import oracle
    t, p = query.target, query.params
    mu = p.mu_arcmin / 60 * math.pi / 180
    if t.kind == scenes.VIEWER:
        return oracle.Cells(2 * t.size[0] * math.tan(mu / 2), mu, p.near_d0, rings_only=True)
    S = max(t.size[0], t.size[1]) if t.kind == scenes.BILLBOARD else t.size[0]
    return oracle.Cells(S, mu, p.near_d0)


def compare_pruned(gpu, orc, scene, query, vp, method):
    """counts exact; colours within 1e-5 relative except at cell-boundary ties."""
    n_bins = query.params.n_bins
    g_cnt = gpu["count"][vp].astype(np.int64)
    assert np.array_equal(g_cnt, orc["count"].astype(np.int64)), "gate counts differ"
    gc = gpu["c"][vp].astype(np.float64)
    oc = orc["c"]
    bad = np.nonzero(np.abs(gc - oc) > 1e-5 * np.abs(oc) + 1e-9)[0]
    ties = 0
    if len(bad):
        import oracle
        t = query.target
        cells = target_cells(query)
        pts = oracle.viewpoint_coords(query.grid, vp[bad])
        for b, qpt in zip(bad, pts):
            D, a = oracle.meridian(t, qpt)
            base = cells.colours(D, a)[METHOD[method]]
            assert oc[b] > 0 and base > 0, (b, gc[b], oc[b])
            gate = oc[b] / base
            ok = False
            for dd, da in ((1 + 1e-9, 0), (1 - 1e-9, 0), (1, 1e-9), (1, -1e-9)):
                alt = cells.colours(D * dd, min(max(a + da, 0.0), math.pi / 2))[METHOD[method]]
                if abs(gc[b] - gate * alt) <= 1e-5 * abs(gc[b]) + 1e-9:
                    ok = True
                    break
            assert ok, f"viewpoint {vp[b]}: gpu {gc[b]} oracle {oc[b]} (D {D}, alpha {a})"
            ties += 1
    assert ties <= max(2, 1e-3 * len(vp)), ties
    tie = np.zeros(len(vp), bool)
    tie[bad] = True
    edge = near_edge(orc["cb"], n_bins)
    badb = np.nonzero((gpu["bin"][vp] != orc["bin"]) & ~edge & ~tie)[0]
    assert badb.size == 0, f"bins differ at {vp[badb[:5]]}"
    return ties


