"""Pins for the oracle: each ties it to something other than itself.

  - the CSR worked example printed in Sec. 4.3 (Eq. csr_demo), golden file;
  - the special case that reduces Eq. approx to an integer matrix product
    (numpy) followed by a test for a positive count;
  - a pure-Python brute force of Eq. bool_dot on tiny inputs;
  - algebraic invariants of the Boolean product;
  - bit interleaving, the closed form that Sec. 4.1 states for Alg. zcurve;
  - a geometric brute force (tests/_geom.py) of Eq. labeling_op restricted to
    the grid, on tiny generated workloads.
"""
import itertools
import math
import os

import numpy as np
import pytest

import gen
import oracle
from tests import _geom

HERE = os.path.dirname(os.path.abspath(__file__))


def read_csr_demo():
    rows, arrays = [], []
    with open(os.path.join(HERE, "golden", "csr_demo.txt")) as f:
        lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    M = np.array([[int(v) for v in ln] for ln in lines[:5]], np.uint8)
    r = np.array([int(v) for v in lines[5]], np.uint64)
    c = np.array([int(v) for v in lines[6]], np.uint32)
    return M, r, c


def random_csr(rng, n_traj, n_cells, density, allow_dup=False):
    M = (rng.random((n_traj, n_cells)) < density).astype(np.uint8)
    rows, cols = np.nonzero(M)
    row_ptr = np.zeros(n_traj + 1, np.uint64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.uint64)
    return M, row_ptr, cols.astype(np.uint32)


# ---------------------------------------------------------------- worked example

def test_csr_demo_identity_recovers_matrix():
    M, r, c = read_csr_demo()
    L = oracle.label_csr(r, c, 5, np.eye(5, dtype=np.uint8))
    assert np.array_equal(L, M)


def test_csr_demo_matches_dense_and_matmul():
    M, r, c = read_csr_demo()
    rng = np.random.default_rng(0)
    for n_props in (1, 3, 8):
        O = (rng.random((5, n_props)) < 0.4).astype(np.uint8)
        want = (M.astype(np.int64) @ O.astype(np.int64)) > 0
        assert np.array_equal(oracle.label_csr(r, c, 5, O), want)
        assert np.array_equal(oracle.label_dense(M, O), want)


def test_csr_demo_single_cell_columns():
    # O = e_k selects column k of M: rows 1 and 3 contain cell 2, etc.
    M, r, c = read_csr_demo()
    for k in range(5):
        O = np.zeros((5, 1), np.uint8)
        O[k, 0] = 1
        assert np.array_equal(oracle.label_csr(r, c, 5, O)[:, 0], M[:, k])


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("seed", range(6))
def test_matches_integer_matmul(seed):
    rng = np.random.default_rng(seed)
    n_traj, n_cells, n_props = rng.integers(1, 40), rng.integers(1, 300), rng.integers(1, 70)
    M, rp, ci = random_csr(rng, n_traj, n_cells, rng.uniform(0.0, 0.2))
    O = rng.integers(0, 256, (n_cells, n_props)).astype(np.uint8)
    O[rng.random(O.shape) < rng.uniform(0.3, 0.99)] = 0  # nonzero bytes mean true
    want = ((M.astype(np.int64) @ (O != 0).astype(np.int64)) > 0).astype(np.uint8)
    assert np.array_equal(oracle.label_csr(rp, ci, n_cells, O), want)
    assert np.array_equal(oracle.label_csr(rp, ci, n_cells, O, threads=3), want)
    assert np.array_equal(oracle.label_dense(M, O), want)


def test_pure_python_brute_force():
    rng = np.random.default_rng(11)
    M, rp, ci = random_csr(rng, 7, 13, 0.25)
    O = (rng.random((13, 5)) < 0.3).astype(np.uint8)
    want = np.array([[int(any(M[t, c] and O[c, p] for c in range(13))) for p in range(5)]
                     for t in range(7)], np.uint8)
    assert np.array_equal(oracle.label_csr(rp, ci, 13, O), want)
    assert np.array_equal(oracle.label_dense(M, O), want)


def test_output_is_zero_one_and_rows_subset():
    rng = np.random.default_rng(5)
    M, rp, ci = random_csr(rng, 30, 100, 0.1)
    O = rng.integers(0, 256, (100, 9)).astype(np.uint8)
    full = oracle.label_csr(rp, ci, 100, O)
    assert set(np.unique(full)) <= {0, 1}
    rows = np.array([29, 0, 7, 7, 13], np.uint64)
    assert np.array_equal(oracle.label_csr(rp, ci, 100, O, rows=rows), full[rows.astype(int)])


def test_unsorted_and_duplicate_columns_accepted():
    # OR is idempotent and commutative: order and repetition inside a row do not matter
    rp = np.array([0, 4, 4, 7], np.uint64)
    ci = np.array([3, 1, 3, 1, 0, 0, 2], np.uint32)
    O = np.eye(4, dtype=np.uint8)
    L = oracle.label_csr(rp, ci, 4, O)
    assert L.tolist() == [[0, 1, 0, 1], [0, 0, 0, 0], [1, 0, 1, 0]]


def test_rejects_out_of_range_column():
    with pytest.raises(ValueError):
        oracle.label_csr(np.array([0, 1], np.uint64), np.array([5], np.uint32), 5,
                         np.ones((5, 1), np.uint8))


# ---------------------------------------------------------------- invariants

def _case(seed, n_traj=25, n_cells=150, n_props=12):
    rng = np.random.default_rng(100 + seed)
    M, rp, ci = random_csr(rng, n_traj, n_cells, 0.05)
    O = (rng.random((n_cells, n_props)) < 0.1).astype(np.uint8)
    return rng, M, rp, ci, O


def _csr_of(M):
    rows, cols = np.nonzero(M)
    rp = np.zeros(M.shape[0] + 1, np.uint64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp).astype(np.uint64), cols.astype(np.uint32)


@pytest.mark.parametrize("seed", range(4))
def test_invariants(seed):
    rng, M, rp, ci, O = _case(seed)
    n_traj, n_cells = M.shape
    L = oracle.label_csr(rp, ci, n_cells, O)
    # empty swept set -> all-false label
    M2 = M.copy()
    M2[3] = 0
    L2 = oracle.label_csr(*_csr_of(M2), n_cells, O)
    assert not L2[3].any()
    # monotone as cells are added to O and to T
    Oplus = O | (rng.random(O.shape) < 0.05).astype(np.uint8)
    assert np.all(oracle.label_csr(rp, ci, n_cells, Oplus) >= L)
    Mplus = M | (rng.random(M.shape) < 0.05).astype(np.uint8)
    assert np.all(oracle.label_csr(*_csr_of(Mplus), n_cells, O) >= L)
    # label of a union of trajectories is the OR of their labels
    Mu = M[:12] | M[12:24]
    Lu = oracle.label_csr(*_csr_of(Mu), n_cells, O)
    assert np.array_equal(Lu, L[:12] | L[12:24])
    # column union in O
    Ocat = np.concatenate([O[:, :5] | O[:, 5:10]], 1)
    assert np.array_equal(oracle.label_csr(rp, ci, n_cells, Ocat), L[:, :5] | L[:, 5:10])
    # consistent permutation of the cells leaves L unchanged
    perm = rng.permutation(n_cells)
    Mp = M[:, perm]
    Op = O[perm]
    assert np.array_equal(oracle.label_csr(*_csr_of(Mp), n_cells, Op), L)
    # O = identity -> L = T; all-true column -> row non-empty
    assert np.array_equal(oracle.label_csr(rp, ci, n_cells, np.eye(n_cells, dtype=np.uint8)), M)
    ones = np.ones((n_cells, 1), np.uint8)
    assert np.array_equal(oracle.label_csr(rp, ci, n_cells, ones)[:, 0], (M.sum(1) > 0).astype(np.uint8))


# ---------------------------------------------------------------- z-order

def interleave(ix, iy, bits):
    n = 0
    for b in range(bits):
        n |= ((ix >> b) & 1) << (2 * b + 1)
        n |= ((iy >> b) & 1) << (2 * b)
    return n


@pytest.mark.parametrize("bits", range(1, 7))
def test_zorder_equals_bit_interleaving_2d(bits):
    side = 1 << bits
    seen = set()
    for ix in range(side):
        for iy in range(side):
            # cell centre and the low corner (a point on splitting planes)
            for fx, fy in ((0.5, 0.5), (0.0, 0.0)):
                z = oracle.zorder([(ix + fx) / side * 7.0 - 2.0, (iy + fy) / side * 3.0 + 1.0],
                                  [-2.0, 1.0], [5.0, 4.0], 2 * bits)
                assert z == interleave(ix, iy, bits)
            seen.add(z)
    assert len(seen) == side * side


def test_zorder_3d_interleaving():
    bits = 3
    for ix, iy, iz in itertools.product(range(8), repeat=3):
        z = oracle.zorder([(ix + .5) / 8, (iy + .5) / 8, (iz + .5) / 8], [0, 0, 0], [1, 1, 1], 3 * bits)
        want = 0
        for b in range(bits):
            want |= ((ix >> b) & 1) << (3 * b + 2) | ((iy >> b) & 1) << (3 * b + 1) | ((iz >> b) & 1) << (3 * b)
        assert z == want


# ---------------------------------------------------------------- geometric brute force

def _tiny_workload(seed, n=16, res=0.75, n_traj=12, n_props=4):
    grid = gen.Grid(n, res)
    rng = np.random.default_rng([seed, 7])
    tr = gen.draw_trajectories(rng, n_traj, grid, 2.0, 10.0, 0.5)
    a = gen.raster_trajectories(tr, grid, threads=2)
    sh = gen.draw_shapes(rng, grid, rng.uniform(0.02, 0.15, n_props))
    O = gen.raster_shapes(sh, grid, n_props)
    return grid, tr, a, sh, O


@pytest.mark.parametrize("seed", range(3))
def test_oracle_matches_geometric_brute_force(seed):
    grid, tr, a, sh, O = _tiny_workload(seed)
    n, res = grid.n, grid.res
    L = oracle.label_csr(a.row_ptr, a.col_idx, grid.n_cells, O)
    region = np.zeros((grid.n_cells, O.shape[1]), bool)
    for i in range(len(sh.kind)):
        region[:, sh.prop[i]] |= _geom.brute_cover_shape(sh.kind[i], sh.cx[i], sh.cy[i], sh.a[i], sh.b[i], n, res)
    # the generator's O is the brute-force region encoding
    assert np.array_equal(region, O.astype(bool))
    T = a.dense().astype(bool)
    for t in range(len(tr)):
        poses = gen.trajectory_poses(tr, t, grid)
        swept = _geom.brute_cover_footprints(poses, n, res)
        assert np.array_equal(swept, T[t]), f"row {t}"
        # Eq. labeling_op on the grid: some footprint and some region meet a common cell
        for p in range(O.shape[1]):
            assert L[t, p] == int(np.any(swept & region[:, p]))


def test_label_is_sound_and_bounded():
    grid, tr, a, sh, O = _tiny_workload(5, n=24, res=0.5, n_traj=10, n_props=5)
    L = oracle.label_csr(a.row_ptr, a.col_idx, grid.n_cells, O)
    rng = np.random.default_rng(3)
    pts = rng.uniform(0.0, grid.extent, (20000, 2))
    for t in range(len(tr)):
        poses = gen.trajectory_poses(tr, t, grid)
        F = _geom.footprint_polys(poses)
        in_foot = np.zeros(len(pts), bool)
        for P in F:
            in_foot |= _geom.point_in_convex(pts, P)
        for p in range(O.shape[1]):
            idx = np.nonzero(sh.prop == p)[0]
            in_reg = np.zeros(len(pts), bool)
            for i in idx:
                if sh.kind[i] == 0:
                    in_reg |= _geom.point_in_convex(pts, _geom.shape_poly(0, sh.cx[i], sh.cy[i], sh.a[i], sh.b[i]))
                else:
                    in_reg |= np.hypot(pts[:, 0] - sh.cx[i], pts[:, 1] - sh.cy[i]) <= sh.a[i]
            # soundness: a point inside both a footprint and the region forces the label
            if np.any(in_foot & in_reg):
                assert L[t, p] == 1
            # bounded over-approximation: a true label means some footprint lies
            # within one cell diagonal of the region
            if L[t, p]:
                d = math.inf
                for P in F:
                    for i in idx:
                        if sh.kind[i] == 0:
                            d = min(d, _geom.poly_poly_dist(P, _geom.shape_poly(0, sh.cx[i], sh.cy[i], sh.a[i], sh.b[i])))
                        else:
                            d = min(d, _geom.poly_disc_dist(P, sh.cx[i], sh.cy[i], sh.a[i]))
                assert d <= math.sqrt(2.0) * grid.res + 1e-9
