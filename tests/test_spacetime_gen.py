"""The time-augmented workload generator (Sec. 5: the plane times time, 2^21
cells) produces what its recipe states: transitions at the paper's mean
occupancy of 0.0223% per row (Table 1), one footprint per layer over the
transition's layers, cell ids ascending within a row, and the two
propositions at about 1% (moving vehicle) and 90% (not nominal lane) of the
workspace (Table 1's occupancies)."""
import numpy as np

import gen


def test_grid_shape():
    g = gen.SpaceTimeGrid()
    assert (g.nx, g.ny, g.n_cells) == (128, 128 * 128, 1 << 21)


def test_transitions_occupancy_and_layers():
    g = gen.SpaceTimeGrid()
    n = 20000
    A = gen.spacetime_abstraction(n, g)
    counts = np.diff(A.row_ptr.astype(np.int64))
    occ = counts.mean() / g.n_cells
    assert abs(occ - 2.23e-4) / 2.23e-4 < 0.03, occ
    assert counts.min() > 0
    rng = np.random.default_rng([gen.SEED0, gen.ST_SEED, 1, 0])
    tr = gen.draw_transitions(rng, n, g)
    layer = A.col_idx.astype(np.int64) // (g.n * g.n)
    rows = np.repeat(np.arange(n), counts)
    assert np.all(layer >= tr["tau0"][rows])
    assert np.all(layer < tr["tau0"][rows] + tr["dur"][rows])
    # every layer of a transition holds part of the footprint
    per_row_layers = [len(np.unique(layer[A.row_ptr[t]:A.row_ptr[t + 1]])) for t in range(0, n, 997)]
    assert per_row_layers == [int(tr["dur"][t]) for t in range(0, n, 997)]
    # ascending within rows
    d = np.diff(A.col_idx.astype(np.int64))
    starts = A.row_ptr[1:-1].astype(np.int64)
    d[starts - 1] = 1
    assert np.all(d > 0)


def test_rows_ordered_by_start_layer():
    g = gen.SpaceTimeGrid()
    rng = np.random.default_rng([gen.SEED0, gen.ST_SEED, 1, 0])
    tr = gen.draw_transitions(rng, 4096, g)
    assert np.all(np.diff(tr["tau0"]) >= 0)
    assert np.all(tr["tau0"] + tr["dur"] <= g.n_tau)


def test_proposition_occupancies():
    g = gen.SpaceTimeGrid()
    for frame in range(3):
        O = gen.spacetime_frame(g, frame)
        assert O.shape == (g.n_cells, 2)
        dens = O.mean(axis=0)
        assert 0.005 < dens[0] < 0.015, dens
        assert 0.88 < dens[1] < 0.92, dens
        # the static proposition repeats in every layer
        lay = O[:, 1].reshape(g.n_tau, -1)
        assert np.all(lay == lay[0])


def test_bernoulli_inputs():
    A = gen.bernoulli_abstraction(500, 1 << 16, 0.01, seed=3)
    counts = np.diff(A.row_ptr.astype(np.int64))
    assert abs(counts.mean() - 655.36) < 10
    for t in range(0, 500, 50):
        r = A.col_idx[A.row_ptr[t]:A.row_ptr[t + 1]]
        assert np.all(np.diff(r.astype(np.int64)) > 0)
    O = gen.bernoulli_frame(1 << 16, 2, 0.3, seed=4)
    assert abs(O.mean() - 0.3) < 0.01


def test_shuffled_rows_are_a_permutation_and_short_grids_work():
    g = gen.SpaceTimeGrid(n=64, n_tau=8, res=1.0)
    A = gen.spacetime_abstraction(2000, g)
    B = gen.spacetime_abstraction(2000, g, shuffle_rows=True)
    rows = lambda X: sorted(tuple(X.col_idx[X.row_ptr[t]:X.row_ptr[t + 1]]) for t in range(2000))
    assert rows(A) == rows(B)
    assert not np.array_equal(A.row_ptr, B.row_ptr)
    assert int(A.col_idx.max()) < g.n_cells


def test_roadmap_edges():
    """Transition t leaves vertex t // 8 and ends at a vertex that starts no
    earlier than its end layer (or at the sink), at a cost of at least 1."""
    g = gen.SpaceTimeGrid()
    n = 30000
    n_v, src, dst, cost = gen.spacetime_roadmap(n, g)
    assert n_v == -(-n // 8) + 1
    assert np.array_equal(src, np.arange(n) // 8)
    assert cost.min() >= 1 and dst.max() < n_v
    rng = np.random.default_rng([gen.SEED0, gen.ST_SEED, 1, 0])
    tr = gen.draw_transitions(rng, n, g)
    v_layer = tr["tau0"][::8]
    real = dst < n_v - 1
    assert real.mean() > 0.8
    assert np.all(v_layer[dst[real]] >= tr["tau0"][real] + tr["dur"][real])
    # the first layer at or after the end: no vertex starts in between
    layers = np.unique(v_layer)
    end = tr["tau0"][real] + tr["dur"][real]
    assert np.array_equal(v_layer[dst[real]], layers[np.searchsorted(layers, end)])
    # a sink only when no vertex starts that late
    assert np.all(tr["tau0"][~real] + tr["dur"][~real] > layers.max())
