"""Planted mistakes in the oracle must be caught by its pins.

Each mutant is a copy of the oracle's C source with one plausible mistake (a
dropped term, a wrong index, a transposed operand, a flipped comparison),
compiled on the CPU into a temporary library.  The pin checks below run
against it and at least one must fail.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import test_oracle_pins as pins
from tests import test_oracle_raster as rpins
from tests import test_oracle_scan as spins

SRC = os.path.join(os.path.dirname(oracle.__file__), "lbl_oracle.c")

MUTANTS = {
    "drop_last_entry": ("k < j->row_ptr[t + 1]; ++k", "k + 1 < j->row_ptr[t + 1]; ++k"),
    "skip_first_entry": ("uint64_t k = j->row_ptr[t];", "uint64_t k = j->row_ptr[t] + 1;"),
    "low_bit_truth": ("(Oc[p] != 0)", "(Oc[p] & 1)"),
    "transposed_O": ("const uint8_t *Oc = j->O + c * j->n_props;", "const uint8_t *Oc = j->O + (c % j->n_props) * j->n_props;"),
    "and_not_or": ("(uint8_t)(Lt[p] | (Oc[p] != 0))", "(uint8_t)(Lt[p] ^ (Oc[p] != 0))"),
    "dense_and": ("acc = acc || (M[", "acc = acc && (M["),
    "zorder_tie_low": ("if (z[j] >= piv[j])", "if (z[j] > piv[j])"),
    "zorder_step": ("(i - 1) / k + 2", "i / k + 2"),
    "zorder_msb": ("(uint64_t)1 << (d - i)", "(uint64_t)1 << (i - 1)"),
}


# mistakes in the proposition encoding (oracle_raster_shapes)
RASTER_MUTANTS = {
    "disc_closed": ("ex * ex + ey * ey < a[s] * a[s]", "ex * ex + ey * ey <= a[s] * a[s]"),
    "disc_radius_unsquared": ("ey * ey < a[s] * a[s]", "ey * ey < a[s]"),
    "disc_drops_y": ("const double ex = cx[s] - qx, ey = cy[s] - qy;", "const double ex = cx[s] - qx, ey = 0.0;"),
    "rect_closed": ("hit = ox > 0.0 && oy > 0.0;", "hit = ox >= 0.0 && oy >= 0.0;"),
    "rect_height_from_a": ("fmin(y1, cy[s] + b[s])", "fmin(y1, cy[s] + a[s])"),
    "cell_without_height": ("y1 = y0 + cell;", "y1 = y0;"),
    "cells_transposed": ("((uint64_t)iy * nx + ix) * n_props", "((uint64_t)ix * ny + iy) * n_props"),
    "last_shape_dropped": ("for (uint64_t s = 0; s < n_shapes; ++s) {", "for (uint64_t s = 0; s + 1 < n_shapes; ++s) {"),
}

# mistakes in the early-termination scan counter (oracle_scan_lengths)
SCAN_MUTANTS = {
    "scan_off_by_one": ("out[i] = c + 1;", "out[i] = c;"),
    "scan_counts_entries": ("out[i] = c + 1;", "out[i] = k - row_ptr[t] + 1;"),
    "scan_ignores_prop": ("if (O[c * n_props + prop] != 0) {", "if (O[c * n_props] != 0) {"),
    "scan_last_hit": ("                out[i] = c + 1;\n                break;\n", "                out[i] = c + 1;\n"),
    "scan_miss_is_zero": ("        out[i] = n_cells;\n", "        out[i] = 0;\n"),
}


def run_scan_pins():
    for args in [(0, 0.05, 0.1), (1, 0.2, 0.02), (2, 0.01, 0.5), (3, 0.3, 0.3)]:
        spins.test_brute_force(*args)
    spins.test_special_cases()
    spins.test_stops_early_iff_labeled()
    spins.test_bernoulli_scan_length_law(0.9)


def run_raster_pins():
    for args in [(1, 64, 0.5, 8, 0), (2, 128, 0.25, 16, 2)]:
        rpins.test_matches_generator_rasterizer(*args)
    rpins.test_grid_aligned_rectangle_marks_enclosed_cells()
    rpins.test_disc_on_corner_marks_four_cells()
    rpins.test_small_disc_inside_one_cell()
    rpins.test_touching_is_not_intersecting()
    rpins.test_outside_and_clipped()
    rpins.test_sampled_brute_force()
    rpins.test_union_is_or()


def run_pins():
    pins.test_csr_demo_identity_recovers_matrix()
    pins.test_csr_demo_matches_dense_and_matmul()
    pins.test_csr_demo_single_cell_columns()
    for s in range(6):
        pins.test_matches_integer_matmul(s)
    pins.test_pure_python_brute_force()
    for s in range(2):
        pins.test_invariants(s)
    for b in (1, 2, 3):
        pins.test_zorder_equals_bit_interleaving_2d(b)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-o", str(so), str(path), "-lm", "-lpthread"])
    saved = oracle._lib
    oracle._lib = oracle._bind(str(so))
    try:
        with pytest.raises((AssertionError, ValueError)):
            run_pins()
    finally:
        oracle._lib = saved


@pytest.mark.parametrize("name", sorted(RASTER_MUTANTS))
def test_raster_mutant_is_caught(name, tmp_path):
    old, new = RASTER_MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-o", str(so), str(path), "-lm", "-lpthread"])
    saved = oracle._lib
    oracle._lib = oracle._bind(str(so))
    try:
        with pytest.raises((AssertionError, ValueError)):
            run_raster_pins()
    finally:
        oracle._lib = saved


@pytest.mark.parametrize("name", sorted(SCAN_MUTANTS))
def test_scan_mutant_is_caught(name, tmp_path):
    old, new = SCAN_MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-o", str(so), str(path), "-lm", "-lpthread"])
    saved = oracle._lib
    oracle._lib = oracle._bind(str(so))
    try:
        with pytest.raises((AssertionError, ValueError)):
            run_scan_pins()
    finally:
        oracle._lib = saved


def test_unmutated_passes():
    run_pins()
    run_raster_pins()
    run_scan_pins()
