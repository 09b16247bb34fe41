"""The oracle's pins catch plausible slips.

Each case copies oracle/vcm_oracle.c, plants one mistake of the kind a reader
of the paper could make (a dropped term, a wrong index, a reversed order, a
strict comparison where the closed one is meant), builds the copy, and runs
the pins that should notice it against that build (the oracle module loads
the library named by VCM_ORACLE_LIB).  Every case must make those pins fail;
the same pins pass on the real oracle in the rest of the suite.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "vcm_oracle.c")

P = "tests/test_oracle_pruned.py::"
MUTANTS = [
    # (what goes wrong, text in the oracle, planted text, pins that must fail)
    ("segment and box that touch at the segment's far end do not meet",
     "        if (a > e || b < 0)", "        if (a >= e || b < 0)",
     ["tests/test_oracle_predicate.py"]),
    ("oblique foreshortening of Eq. 2 dropped",
     "    double s_alpha = (alpha / (VO_PI / 2.0)) * S; /* Eq. 2 */",
     "    double s_alpha = S; /* Eq. 2 */",
     ["tests/test_oracle_measure.py::test_worked_example"]),
    ("field-of-view wedge open instead of closed",
     "        return dn >= 0.0 && dn * dn >= c2 * d2;", "        return dn >= 0.0 && dn * dn > c2 * d2;",
     ["tests/test_oracle_map.py::test_fov_wedge"]),
    ("wide field-of-view wedge open instead of closed",
     "    return dn >= 0.0 || dn * dn <= c2 * d2;", "    return dn >= 0.0 || dn * dn < c2 * d2;",
     ["tests/test_oracle_map.py::test_fov_wedge"]),
    ("cube faces live from their own plane",
     "        if (!(sgn * (q[k] - plane) > 0.0))", "        if (!(sgn * (q[k] - plane) >= 0.0))",
     ["tests/test_oracle_map.py::test_cube_live_counts"]),
    ("ring boundaries one mu step late",
     "        double V = V0 - k * mu;", "        double V = V0 - (k + 1) * mu;",
     [P + "test_rings_step_the_facing_angle_by_mu"]),
    ("cell colour taken at the ring's inner radius",
     "    double dp = 0.5 * (c->d[i] + c->d[i + 1]);\n    double gm = 0.5 * (g[j] + g[j + 1]);\n    if",
     "    double dp = c->d[i];\n    double gm = 0.5 * (g[j] + g[j + 1]);\n    if",
     [P + "test_cell_colour_is_the_visual_angle_at_the_parameter_midpoint"]),
    ("cell colour taken at the band's upper edge",
     "    double gm = 0.5 * (g[j] + g[j + 1]);\n    if (c->rings_only)",
     "    double gm = g[j];\n    if (c->rings_only)",
     [P + "test_cell_colour_is_the_visual_angle_at_the_parameter_midpoint"]),
    ("VCM_M takes the highest ring instead of the lowest",
     "    for (int i = 0; i < c->nring && !found; ++i) {",
     "    for (int i = c->nring - 1; i >= 0 && !found; --i) {",
     [P + "test_m_takes_the_lowest_cell_whose_mbr_holds_q"]),
    ("VCM_M scans a ring's bands from the last one",
     "        for (int j = 0; j < L; ++j) {\n            double r0 = c->d[i] * cos(g[j])",
     "        for (int j = L - 1; j >= 0; --j) {\n            double r0 = c->d[i] * cos(g[j])",
     [P + "test_m_takes_the_lowest_cell_whose_mbr_holds_q"]),
    ("VCM_M box height from the wrong band edge",
     "            double h0 = c->d[i] * sin(g[j + 1]), h1 = c->d[i + 1] * sin(g[j]);",
     "            double h0 = c->d[i] * sin(g[j]), h1 = c->d[i + 1] * sin(g[j]);",
     [P + "test_m_takes_the_lowest_cell_whose_mbr_holds_q"]),
    ("VCM_T projects on the band's upper edge instead of its middle",
     "        double gm = 0.5 * (g[j] + g[j + 1]);\n        double p = D * cos(alpha - gm);",
     "        double gm = g[j];\n        double p = D * cos(alpha - gm);",
     [P + "test_t_takes_the_lowest_ring_whose_tangent_trapezoid_holds_q",
      P + "test_t_single_band_rings_project_on_the_diagonal"]),
    ("VCM_T takes the highest ring instead of the lowest",
     "    for (int i = 0; i < c->nring; ++i) {\n        int j = band_of(c, i, alpha);",
     "    for (int i = c->nring - 1; i >= 0; --i) {\n        int j = band_of(c, i, alpha);",
     [P + "test_t_takes_the_lowest_ring_whose_tangent_trapezoid_holds_q"]),
    ("hull test keeps the looser lower bound of lambda",
     "                if (-y * ld > ln * -x) {", "                if (-y * ld < ln * -x) {",
     ["tests/test_oracle_blocks.py::test_hull_of_a_point_block_is_the_segment_test",
      "tests/test_oracle_blocks.py::test_hull_test_matches_a_linear_program"]),
    ("a sample counts as hidden when one corner's segment is cut",
     "            for (int c = 0; c < nc && all; ++c)", "            for (int c = 0; c < 1 && all; ++c)",
     ["tests/test_oracle_blocks.py::test_decided_blocks_agree_with_brute_force_everywhere"]),
    ("wide field of view taken as convex",
     "            wedge = all_front ? 1 : (all_out ? 0 : -1);", "            wedge = all_in ? 1 : (all_out ? 0 : -1);",
     ["tests/test_oracle_blocks.py::test_block_hand_cases"]),
    ("live faces not checked for the whole block",
     "        uniform = m == n && memcmp(smp, tmp, sizeof(double) * 3 * (size_t)n) == 0;",
     "        uniform = 1;",
     ["tests/test_oracle_blocks.py::test_decided_blocks_agree_with_brute_force_everywhere",
      "tests/test_oracle_blocks.py::test_block_hand_cases"]),
    ("FRACTION-mode block decided with one sample undecided",
     "    if (seen + hidden == n) {", "    if (seen + hidden >= n - 1) {",
     ["tests/test_oracle_blocks.py::test_decided_blocks_agree_with_brute_force_everywhere"]),
    ("viewer size taken as d_max mu instead of 2 d_max tan(mu / 2)",
     "        return 2.0 * t->size[0] * tan(mu_rad(p) / 2.0);", "        return t->size[0] * mu_rad(p);",
     ["tests/test_oracle_viewer.py::test_size_gives_mu_at_dmax"]),
    ("viewer region open at d_max",
     "    return r2 <= t->size[0] * t->size[0];", "    return r2 < t->size[0] * t->size[0];",
     ["tests/test_oracle_viewer.py::test_region_is_the_closed_ball"]),
    ("viewer cells coloured at the band's middle angle",
     "    if (c->rings_only)\n        gm = VO_PI / 2.0;\n", "",
     ["tests/test_oracle_viewer.py::test_viewer_cells_are_rings"]),
    ("error bounds count the bands above the stated angle",
     "                if (g[j + 1] < lim[m])", "                if (g[j + 1] > lim[m])",
     [P + "test_measured_error_within_the_printed_bounds"]),
]


@pytest.mark.parametrize("what,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_fails_on_planted_slip(tmp_path, what, old, new, pins):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not found once: {old!r}"
    mutant = tmp_path / "vcm_oracle.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libvcm_oracle_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(lib), str(mutant),
                           "-lm", "-lpthread"])
    env = dict(os.environ, VCM_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    # exit status 1: tests ran and at least one failed (2 and up: errors)
    assert r.returncode == 1, f"{what}: pins did not fail (status {r.returncode})\n{r.stdout[-2000:]}"
