"""Pins for the oracle's early-termination scan counter (Sec. 5.1, Eq.
prob_term): the number of cells a serial scan of Eq. bool_dot compares before
it meets the first cell shared by the trajectory and the proposition.

  - brute force: the first index of the dense row AND the dense proposition
    column, on small random inputs;
  - special cases: an empty row or an empty proposition scans every cell; a
    proposition covering every cell stops at the row's first cell;
  - agreement with the labeling oracle: the scan stops early exactly when
    L[t][p] is 1;
  - the paper's law: on Bernoulli subsets (cells occupied with bias p by the
    trajectory and q by the proposition, independently) the scan length is
    geometric with success probability pq, truncated at the cell count N, so
    its mean is (1 - (1 - pq)^N) / (pq), which is 1 / (pq) when pq N is large.
    Checked at the paper's occupancy p = 0.0223% for q = 90% and q = 1%, and
    the ratio of the two means against the factor of about 90 that the paper
    derives from it.
"""
import math

import numpy as np
import pytest

import gen
import oracle


def dense_first_hit(M, O, p):
    hit = (M != 0) & (O[:, p] != 0)[None, :]
    any_hit = hit.any(axis=1)
    return np.where(any_hit, hit.argmax(axis=1) + 1, M.shape[1]).astype(np.uint64)


def to_csr(M):
    rows, cols = np.nonzero(M)
    row_ptr = np.zeros(M.shape[0] + 1, np.uint64)
    np.cumsum(np.bincount(rows, minlength=M.shape[0]), out=row_ptr[1:])
    return row_ptr, cols.astype(np.uint32)


@pytest.mark.parametrize("seed,pm,po", [(0, 0.05, 0.1), (1, 0.2, 0.02), (2, 0.01, 0.5), (3, 0.3, 0.3)])
def test_brute_force(seed, pm, po):
    rng = np.random.default_rng(seed)
    n_traj, n_cells, n_props = 60, 500, 3
    M = (rng.uniform(size=(n_traj, n_cells)) < pm).astype(np.uint8)
    O = (rng.uniform(size=(n_cells, n_props)) < po).astype(np.uint8)
    rp, ci = to_csr(M)
    for p in range(n_props):
        assert np.array_equal(oracle.scan_lengths(rp, ci, n_cells, O, p), dense_first_hit(M, O, p))


def test_special_cases():
    n_cells = 100
    rp = np.array([0, 0, 3, 4], np.uint64)  # row 0 empty
    ci = np.array([7, 20, 99, 0], np.uint32)
    ones = np.ones((n_cells, 2), np.uint8)
    zeros = np.zeros((n_cells, 2), np.uint8)
    assert list(oracle.scan_lengths(rp, ci, n_cells, ones, 1)) == [100, 8, 1]
    assert list(oracle.scan_lengths(rp, ci, n_cells, zeros, 0)) == [100, 100, 100]
    only99 = zeros.copy()
    only99[99, 0] = 1
    assert list(oracle.scan_lengths(rp, ci, n_cells, only99, 0)) == [100, 100, 100]  # hit at the last cell
    only20 = zeros.copy()
    only20[20, 1] = 1
    assert list(oracle.scan_lengths(rp, ci, n_cells, only20, 1)) == [100, 21, 100]
    assert list(oracle.scan_lengths(rp, ci, n_cells, only20, 1, rows=[2, 1])) == [100, 21]


def test_rejects_unsorted_and_out_of_range():
    O = np.ones((10, 1), np.uint8)
    with pytest.raises(ValueError):
        oracle.scan_lengths(np.array([0, 2], np.uint64), np.array([5, 3], np.uint32), 10, O, 0)
    with pytest.raises(ValueError):
        oracle.scan_lengths(np.array([0, 1], np.uint64), np.array([10], np.uint32), 10, O, 0)


def test_stops_early_iff_labeled():
    g = gen.SpaceTimeGrid(n=128, n_tau=16)
    A = gen.spacetime_abstraction(3000, g)
    O = gen.spacetime_frame(g, frame=1)
    L = oracle.label_csr(A.row_ptr, A.col_idx, g.n_cells, O)
    for p in range(2):
        s = oracle.scan_lengths(A.row_ptr, A.col_idx, g.n_cells, O, p)
        # a hit exactly at the last cell also reads n_cells; the workload has none there
        assert np.array_equal(s < g.n_cells, L[:, p] == 1)


def truncated_geometric_mean(r, n):
    return (1.0 - (1.0 - r) ** n) / r


@pytest.mark.parametrize("q", [0.9, 0.01])
def test_bernoulli_scan_length_law(q):
    n_cells, p, n_rows = 1 << 21, 2.23e-4, 4000
    A = gen.bernoulli_abstraction(n_rows, n_cells, p, seed=11)
    O = gen.bernoulli_frame(n_cells, 1, q, seed=12)
    s = oracle.scan_lengths(A.row_ptr, A.col_idx, n_cells, O, 0).astype(np.float64)
    want = truncated_geometric_mean(p * q, n_cells)
    se = s.std(ddof=1) / math.sqrt(n_rows)
    assert abs(s.mean() - want) < 5 * se, (s.mean(), want, se)
    if q == 0.9:  # far from the truncation: the untruncated 1 / (pq)
        assert abs(want - 1.0 / (p * q)) / want < 1e-6


def test_bernoulli_ratio_of_ninety():
    """The paper's factor: 1/(0.9 p) against 1/(0.01 p) is 90; on 2^21 cells
    the truncated means differ by slightly less, and the sampled means agree
    with that within their error."""
    n_cells, p, n_rows = 1 << 21, 2.23e-4, 3000
    A = gen.bernoulli_abstraction(n_rows, n_cells, p, seed=21)
    means = []
    for q, seed in ((0.9, 22), (0.01, 23)):
        O = gen.bernoulli_frame(n_cells, 1, q, seed=seed)
        means.append(oracle.scan_lengths(A.row_ptr, A.col_idx, n_cells, O, 0).astype(np.float64).mean())
    exact = truncated_geometric_mean(0.01 * p, n_cells) / truncated_geometric_mean(0.9 * p, n_cells)
    assert 85 < exact < 90
    assert abs(means[1] / means[0] - exact) / exact < 0.1
