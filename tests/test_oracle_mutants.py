"""The pins are strong enough: each plausible mistake, planted in a copy of
the C oracle compiled on the CPU, makes at least one pin fail.

The copies live in a temporary directory; the real oracle is untouched.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import build as OB
from oracle import oracle as O
from tests import test_oracle_pins as P

MUTANTS = {
    # tie-break direction reversed (equal values: smaller index wins)
    "tie_break": ("return c > 0 || (c == 0 && a > b);", "return c > 0 || (c == 0 && a < b);"),
    # mixed-sign offsets accepted: the 3^n - 1 box neighbourhood instead of Alg. 1
    "adjacency_mixed_signs": ("if (!(d == 0 || d == -1)) in0m1 = 0;",
                              "if (!(d == 0 || d == -1 || d == 1)) in0m1 = 0;"),
    # only the axis-aligned neighbours (a cube grid without the tessellation)
    "adjacency_axis_only": ("return !same && (in01 || in0m1);",
                            "int nz = 0; for (int i = 0; i < n; ++i) nz += (p[i] != q[i]);"
                            " return !same && (in01 || in0m1) && nz == 1;"),
    # lowest instead of highest vertex of each upper-link component
    "rep_lowest": ("if (above(g, ids[up[x]], rep)) rep = ids[up[x]];",
                   "if (above(g, rep, ids[up[x]])) rep = ids[up[x]];"),
    # gradient = first upper neighbour found instead of the highest
    "gradient_first": ("if (above(g, ids[up[a]], best)) best = ids[up[a]];",
                       "if (best == v) best = ids[up[a]];"),
    # link edge test on the wrong operand (index confusion)
    "bfs_index": ("if (grid_adjacent(g->n, coords[up[x]], coords[up[b]])) {",
                  "if (grid_adjacent(g->n, coords[x], coords[up[b]])) {"),
    # coordinates decoded in Fortran order while indices are C order
    "transposed_coords": ("for (int i = g->n - 1; i >= 0; --i) {\n        c[i] = v % g->dims[i];",
                          "for (int i = 0; i < g->n; ++i) {\n        c[i] = v % g->dims[i];"),
    # duplicates kept in the arc rows
    "no_dedup": ("if (len == 0 || row[len - 1] != row[j]) row[len++] = row[j];",
                 "row[len++] = row[j];"),
    # minima graph obtained by negating values but keeping the index tie-break
    "minima_negate_only": ("return c < 0 || (c == 0 && b > a);",
                           "return c < 0 || (c == 0 && a > b);"),
    # float64 samples compared after rounding to float32
    "f64_as_f32": ("case EGO_F64: EGO_CMP(double)", "case EGO_F64: EGO_CMP(float)"),
    # 64-bit integers compared through double (exact only below 2^53)
    "i64_as_double": ("case EGO_I64: EGO_CMP(int64_t)",
                      "case EGO_I64: { const double x = (double)((const int64_t*)g->f)[a],"
                      " y = (double)((const int64_t*)g->f)[b]; return (x > y) - (x < y); }"),
    # unsigned 32-bit samples compared as signed
    "u32_as_signed": ("case EGO_U32: EGO_CMP(uint32_t)", "case EGO_U32: EGO_CMP(int32_t)"),
    # paths of a saddle ordered by their reps instead of the components' smallest vertex
    "paths_order_by_rep": ("int64_t x = ((const comp_t*)a)->lo, y = ((const comp_t*)b)->lo;",
                           "int64_t x = ((const comp_t*)a)->rep, y = ((const comp_t*)b)->rep;"),
    # a component's smallest vertex tracked as its largest
    "paths_lo_as_hi": ("if (ids[up[x]] < lo) lo = ids[up[x]];", "if (ids[up[x]] > lo) lo = ids[up[x]];"),
    # the walk starts one step past the rep
    "paths_skip_rep": ("            int64_t r = comps[j].rep;\n            vertices[at++] = saddles[i];\n"
                       "            vertices[at++] = (int32_t)r;",
                       "            int64_t r = comps[j].rep;\n            vertices[at++] = saddles[i];\n"
                       "            r = ptr[r];\n            vertices[at++] = (int32_t)r;"),
}


def _pins():
    P.test_golden_worked_examples("worked_1d.json")
    P.test_golden_worked_examples("worked_2d_3x3.json")
    P.test_neighbour_counts_and_link_fvectors()
    for shape in [(9,), (6, 7), (5, 4, 3), (3, 3, 2, 3), (3, 2, 3, 2, 2)]:
        for kind in ("uniform", "ties"):
            P.test_oracle_matches_brute(shape, kind)
    P.test_constant_field((4, 5, 3))
    P.test_banchoff_2d_from_beta()
    P.test_minima_graph_is_flipped_negated_maxima_graph((5, 4, 6))
    for shape in [(6, 7), (5, 4, 3)]:
        P.test_paths_match_brute(shape, "uniform")
    for dt in P.TYPED:
        P.test_typed_fields_match_brute(dt)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    old, new = MUTANTS[name]
    src = open(OB.SRC).read()
    assert src.count(old) == 1, "mutation site moved"
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "m.c")
        so = os.path.join(td, "libm.so")
        with open(c, "w") as fh:
            fh.write(src.replace(old, new))
        subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-o", so, c, "-lm"],
                       check=True)
        prev = O.use_library(so)
        try:
            with pytest.raises((AssertionError, O.OracleError)):
                _pins()
        finally:
            O._lib = prev


def test_unmutated_passes_same_pins():
    _pins()
    assert np.all(np.isfinite([1.0]))
