"""Comparison of the HIP path's outputs with the oracle's, to the stated bar:
visible counts bit-exact; colour bins bit-exact except where the oracle's
colour (in the bin's scale) lies within 1e-6 of a bin edge; colours within
1e-5 relative of the oracle's, with an absolute floor of 1e-9."""
import numpy as np

C_REL = 1e-5
C_ABS = 1e-9
EDGE = 1e-6


def near_edge(cb, n_bins):
    x = np.asarray(cb, dtype=np.float64) * n_bins
    return np.abs(x - np.round(x)) < EDGE * n_bins


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
