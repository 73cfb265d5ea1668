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


def test_unmutated_passes():
    run_pins()
