"""Pins for the oracle's proposition encoding (Sec. 4.1: a cell's entry is 1
iff the region intersects it; read as an overlap of positive area with the
closed cell square).  Each ties the oracle to something other than itself:

  - the generator's separate bounding-box rasterizer (gen/raster.c), on the
    generated frames of the workloads;
  - closed forms on exactly representable geometry: a grid-aligned rectangle
    marks exactly the cells it encloses, a disc of radius cell/2 centred on a
    grid corner marks the four cells around that corner, a small disc inside
    one cell marks that cell alone;
  - touching is not intersecting: shapes whose boundary lies on a cell edge or
    corner do not mark the cell on the other side;
  - a sampled brute force: a cell holding a sample point strictly inside a
    shape is marked, and a marked cell's overlap is confirmed by sampling;
  - the encoding of a union is the OR of the encodings of its parts.
"""
import numpy as np
import pytest

import gen
import oracle


def raster(shapes, nx, ny, cell, n_props):
    kind, prop, cx, cy, a, b = (np.array([s[i] for s in shapes]) for i in range(6))
    return oracle.raster_shapes(kind, prop, cx, cy, a, b, nx, ny, cell, n_props)


def grid_of(O, nx, ny, p=0):
    return O[:, p].reshape(ny, nx)


@pytest.mark.parametrize("cfg,n,res,n_props,frame", [(1, 64, 0.5, 8, 0), (1, 64, 0.5, 8, 1), (2, 128, 0.25, 16, 2),
                                                     (4, 128, 0.8, 37, 3)])
def test_matches_generator_rasterizer(cfg, n, res, n_props, frame):
    g = gen.Grid(n, res)
    sh = gen.frame_shapes(cfg, g, n_props, frame, rho_lo=0.02, rho_hi=0.4)
    want = gen.raster_shapes(sh, g, n_props)
    got = oracle.raster_shapes(sh.kind.astype(np.uint32), sh.prop, sh.cx, sh.cy, sh.a, sh.b, n, n, res, n_props)
    assert np.array_equal(got, want)
    assert 0 < got.sum() < got.size


def test_grid_aligned_rectangle_marks_enclosed_cells():
    # cells 2..5 in x, 1..2 in y on a 0.5 m grid: centre and half sizes exact in binary
    O = raster([(0, 0, 2.0, 1.0, 1.0, 0.5)], 8, 8, 0.5, 1)
    want = np.zeros((8, 8), np.uint8)
    want[1:3, 2:6] = 1
    assert np.array_equal(grid_of(O, 8, 8), want)


def test_disc_on_corner_marks_four_cells():
    O = raster([(1, 0, 2.0, 1.5, 0.25, 0.0)], 8, 8, 0.5, 1)  # corner (4, 3) of the 0.5 m grid
    want = np.zeros((8, 8), np.uint8)
    want[2:4, 3:5] = 1
    assert np.array_equal(grid_of(O, 8, 8), want)


def test_small_disc_inside_one_cell():
    O = raster([(1, 0, 1.25, 0.75, 0.1, 0.0)], 8, 8, 0.5, 1)
    want = np.zeros((8, 8), np.uint8)
    want[1, 2] = 1
    assert np.array_equal(grid_of(O, 8, 8), want)


def test_touching_is_not_intersecting():
    # rectangle [1, 2] x [1, 2] exactly: its edges lie on cell boundaries
    O = raster([(0, 0, 1.5, 1.5, 0.5, 0.5)], 8, 8, 0.5, 1)
    assert grid_of(O, 8, 8).sum() == 4
    # zero-width rectangle on a cell edge, and a disc touching a cell from outside
    O = raster([(0, 0, 1.0, 1.5, 0.0, 0.5), (1, 1, 0.25, 0.25, 0.0, 0.0)], 8, 8, 0.5, 2)
    assert O.sum() == 0
    O = raster([(1, 0, 1.75, 1.25, 0.25, 0.0)], 8, 8, 0.5, 1)  # radius reaches the edges x = 1.5, 2.0, y = 1.0, 1.5
    assert grid_of(O, 8, 8).sum() == 1 and grid_of(O, 8, 8)[2, 3] == 1


def test_outside_and_clipped():
    O = raster([(1, 0, -5.0, -5.0, 1.0, 0.0), (0, 0, 100.0, 1.0, 3.0, 3.0)], 8, 8, 0.5, 1)
    assert O.sum() == 0
    O = raster([(0, 0, 0.0, 0.0, 0.75, 0.75)], 8, 8, 0.5, 1)  # straddles the corner of the workspace
    want = np.zeros((8, 8), np.uint8)
    want[0:2, 0:2] = 1
    assert np.array_equal(grid_of(O, 8, 8), want)


def test_sampled_brute_force():
    rng = np.random.default_rng(5)
    n, cell, k = 16, 0.5, 24  # k x k samples strictly inside each cell
    shapes = []
    for i in range(12):
        kind = int(rng.integers(0, 2))
        shapes.append((kind, i, rng.uniform(0, 8), rng.uniform(0, 8), rng.uniform(0.05, 2.0), rng.uniform(0.05, 2.0)))
    O = raster(shapes, n, n, cell, 12)
    off = (np.arange(k) + 0.5) / k * cell
    for s, (kind, p, cx, cy, a, b) in enumerate(shapes):
        G = grid_of(O, n, n, p)
        for iy in range(n):
            for ix in range(n):
                xs = ix * cell + off[None, :]
                ys = iy * cell + off[:, None]
                if kind == 0:
                    inside = (np.abs(xs - cx) < a) & (np.abs(ys - cy) < b)
                else:
                    inside = (xs - cx) ** 2 + (ys - cy) ** 2 < a * a
                if inside.any():
                    assert G[iy, ix] == 1, (s, ix, iy)
                elif G[iy, ix] == 1:
                    # marked without a sample inside: the overlap must be thinner than the lattice spacing
                    x0, y0 = ix * cell, iy * cell
                    if kind == 0:
                        ox = min(x0 + cell, cx + a) - max(x0, cx - a)
                        oy = min(y0 + cell, cy + b) - max(y0, cy - b)
                        assert 0 < min(ox, oy) < cell / k * 1.01, (s, ix, iy)
                    else:
                        qx, qy = min(max(cx, x0), x0 + cell), min(max(cy, y0), y0 + cell)
                        assert a - np.hypot(cx - qx, cy - qy) < cell / k * 1.5, (s, ix, iy)


def test_union_is_or():
    rng = np.random.default_rng(9)
    shapes = [(int(rng.integers(0, 2)), 0, rng.uniform(0, 16), rng.uniform(0, 16), rng.uniform(0.1, 3), rng.uniform(0.1, 3))
              for _ in range(6)]
    whole = raster(shapes, 32, 32, 0.5, 1)
    parts = [raster([s], 32, 32, 0.5, 1) for s in shapes]
    assert np.array_equal(whole, np.bitwise_or.reduce(parts))


def test_rejects_bad_shapes():
    with pytest.raises(ValueError):
        raster([(2, 0, 1.0, 1.0, 1.0, 1.0)], 8, 8, 0.5, 1)
    with pytest.raises(ValueError):
        raster([(0, 3, 1.0, 1.0, 1.0, 1.0)], 8, 8, 0.5, 2)
