"""CPU checks of the C ABI: the library loads, exports every declared entry
point, computes the device cell order on the host, and rejects bad arguments
before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1810_02612_amd import lbl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lbl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbl_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = lbl.lib()
    names = declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(L, name), name
    assert set(lbl.EXPORTS) == set(names)


def test_version_and_empty_error():
    assert "gfx950" in lbl.version()


@pytest.mark.parametrize("bits", [1, 3, 6])
def test_cell_order_is_zorder_on_square_power_of_two_grids(bits):
    # side 2^bits tiles of 8 cells: word * 64 + bit must be the cell's z-order
    # index from the oracle's reading of the z-curve descent
    n = 8 << bits
    d = 2 * (bits + 3)
    rng = np.random.default_rng(bits)
    cells = rng.choice(n * n, size=min(n * n, 600), replace=False)
    for c in cells:
        ix, iy = int(c) % n, int(c) // n
        w, b = lbl.cell_position(n, n, int(c))
        z = oracle.zorder([ix + 0.5, iy + 0.5], [0.0, 0.0], [float(n), float(n)], d)
        assert w * 64 + b == z


@pytest.mark.parametrize("nx,ny", [(8, 8), (24, 40), (64, 16), (8, 72)])
def test_cell_order_is_a_bijection_with_tiles_in_words(nx, ny):
    seen = set()
    for c in range(nx * ny):
        w, b = lbl.cell_position(nx, ny, c)
        assert 0 <= b < 64 and 0 <= w < nx * ny // 64
        seen.add((w, b))
        ix, iy = c % nx, c // nx
        # all 64 cells of an 8x8 tile share a word
        w0, _ = lbl.cell_position(nx, ny, (iy // 8 * 8) * nx + ix // 8 * 8)
        assert w == w0
    assert len(seen) == nx * ny


def test_morton_cell_ids_address_the_same_device_position():
    """With LBL_MORTON the caller's id is the z-order index of Alg. zcurve (as
    the oracle's descent computes it); the library must place that cell where
    the row-major id of the same cell goes."""
    import oracle
    for n in (8, 16, 64):
        d = 2 * (n.bit_length() - 1)
        seen = set()
        for iy in range(n):
            for ix in range(n):
                z = oracle.zorder([ix + 0.5, iy + 0.5], [0.0, 0.0], [float(n), float(n)], d)
                wz, bz = lbl.cell_position(n, n, z, lbl.MORTON)
                assert (wz, bz) == lbl.cell_position(n, n, iy * n + ix), (n, ix, iy, z)
                seen.add(z)
        assert seen == set(range(n * n))
    with pytest.raises(lbl.LblError):
        lbl.cell_position(64, 64, 64 * 64, lbl.MORTON)


def test_invalid_arguments_are_rejected_without_a_device():
    rp = np.array([0, 1], np.uint64)
    ci = np.array([0], np.uint32)
    with pytest.raises(lbl.LblError) as e:
        lbl.load_abstraction(12, 8, rp, ci)
    assert e.value.status == lbl.EINVAL and "multiples of 8" in str(e.value)
    with pytest.raises(lbl.LblError) as e:
        lbl.load_abstraction(8, 8, np.array([1, 2], np.uint64), ci)
    assert e.value.status == lbl.EINVAL
    with pytest.raises(lbl.LblError) as e:
        lbl.load_abstraction(8, 8, np.array([0, 3, 2], np.uint64), np.zeros(3, np.uint32))
    assert "non-decreasing" in str(e.value)
    with pytest.raises(lbl.LblError) as e:
        lbl.load_abstraction(8, 8, rp, ci, flags=0x100)
    assert e.value.status == lbl.EINVAL
    # sparse only excludes the int8 copy and the no-sparse flag
    for f in (lbl.LOAD_SPARSE_ONLY | lbl.LOAD_KEEP_INT8, lbl.LOAD_SPARSE_ONLY | lbl.LOAD_NO_SPARSE):
        with pytest.raises(lbl.LblError) as e:
            lbl.load_abstraction(8, 8, rp, ci, flags=f)
        assert e.value.status == lbl.EINVAL and "SPARSE_ONLY" in str(e.value)
    # the dense loader has no sparse-only mode
    with pytest.raises(lbl.LblError) as e:
        lbl.load_abstraction_dense(8, 8, np.zeros((1, 64), np.uint8), flags=lbl.LOAD_SPARSE_ONLY)
    assert e.value.status == lbl.EINVAL
    with pytest.raises(lbl.LblError):
        lbl.label_frame(None, 1, 8, 1)
    with pytest.raises(lbl.LblError):
        lbl.cell_position(8, 8, 64)
    # n_traj == 0
    g = lbl.Grid(8, 8, 0.5, 0)
    h = ctypes.c_void_p()
    st = lbl.lib().lbl_load_abstraction(ctypes.byref(g), 0, rp.ctypes.data, ci.ctypes.data, 0, ctypes.byref(h))
    assert st == lbl.EINVAL and h.value is None
    # cell_order must be known; z-order ids need a square grid of power-of-two side
    for g in (lbl.Grid(8, 8, 0.5, 2), lbl.Grid(24, 24, 0.5, lbl.MORTON), lbl.Grid(16, 8, 0.5, lbl.MORTON)):
        st = lbl.lib().lbl_load_abstraction(ctypes.byref(g), 1, rp.ctypes.data, ci.ctypes.data, 0, ctypes.byref(h))
        assert st == lbl.EINVAL and h.value is None
        assert "cell_order" in lbl.last_error() or "LBL_MORTON" in lbl.last_error()
        T1 = np.zeros((1, g.nx * g.ny), np.uint8)
        st = lbl.lib().lbl_load_abstraction_dense(ctypes.byref(g), 1, T1.ctypes.data, 0, ctypes.byref(h))
        assert st == lbl.EINVAL and h.value is None


def test_batch_and_serve_reject_bad_arguments():
    with pytest.raises(lbl.LblError):
        lbl.label_batch([], 0)
    with pytest.raises(lbl.LblError):
        lbl.serve_start(max_batch_frames=0)


def test_raster_rejects_bad_arguments_without_a_device():
    L = lbl.lib()
    g = lbl.Grid(16, 16, 0.5, 0)
    fake_O = ctypes.c_void_p(0x1000)  # validation fails before any device access
    good = lbl.shapes_array([0], [0], [1.0], [1.0], [0.5], [0.5])

    def call(shapes, n_props=4, cell=0.5, grid=g, O=fake_O, n=None):
        ptr = shapes.ctypes.data if shapes is not None and len(shapes) else None
        n = len(shapes) if n is None else n
        return L.lbl_raster_frame(ctypes.byref(grid) if grid is not None else None, cell, ptr, n, n_props, O, None)

    cases = [
        lambda: call(good, grid=None),
        lambda: call(good, O=None),
        lambda: call(None, n=3),
        lambda: call(good, grid=lbl.Grid(12, 16, 0.5, 0)),
        lambda: call(good, grid=lbl.Grid(16, 16, 0.5, 2)),
        lambda: call(good, grid=lbl.Grid(24, 24, 0.5, lbl.MORTON)),
        lambda: call(good, n_props=0),
        lambda: call(good, n_props=65),
        lambda: call(good, cell=0.0),
        lambda: call(good, cell=float("nan")),
        lambda: call(lbl.shapes_array([2], [0], [1.0], [1.0], [0.5], [0.5])),
        lambda: call(lbl.shapes_array([0], [4], [1.0], [1.0], [0.5], [0.5])),
        lambda: call(lbl.shapes_array([1], [0], [float("inf")], [1.0], [0.5], [0.0])),
        lambda: call(lbl.shapes_array([1], [0], [1.0], [1.0], [-0.5], [0.0])),
        lambda: call(lbl.shapes_array([0], [0], [1.0], [1.0], [0.5], [-0.5])),
    ]
    for i, c in enumerate(cases):
        assert c() == lbl.EINVAL, i
        assert lbl.last_error(), i


def test_planner_rejects_bad_arguments_without_a_device():
    f = lbl.lib().lbl_product_shortest_paths
    d2 = np.zeros(2, np.uint8)
    fake = 0x1000  # never dereferenced: every call below fails its host checks first
    cases = [
        lambda: f(0, 1, fake, fake, fake, fake, 1, 1, 1, d2.ctypes.data, 0, 0, fake, fake, None, None),   # no vertices
        lambda: f(4, 1, fake, fake, fake, fake, 0, 0, 1, d2.ctypes.data, 0, 0, fake, fake, None, None),   # n_props 0
        lambda: f(4, 1, fake, fake, fake, fake, 9, 9, 1, d2.ctypes.data, 0, 0, fake, fake, None, None),   # n_props 9
        lambda: f(4, 1, fake, fake, fake, fake, 1, 1, 9, d2.ctypes.data, 0, 0, fake, fake, None, None),   # 9 states
        lambda: f(4, 1, fake, fake, fake, fake, 1, 1, 1, d2.ctypes.data, 4, 0, fake, fake, None, None),   # v0 out of range
        lambda: f(4, 1, fake, fake, fake, fake, 1, 1, 1, d2.ctypes.data, 0, 1, fake, fake, None, None),   # q0 out of range
        lambda: f(4, 1, None, fake, fake, fake, 1, 1, 1, d2.ctypes.data, 0, 0, fake, fake, None, None),   # null src
        lambda: f(4, 1, fake, fake, fake, fake, 1, 1, 1, None, 0, 0, fake, fake, None, None),             # null delta
        lambda: f(4, 1, fake, fake, fake, fake, 1, 1, 1, np.array([0, 3], np.uint8).ctypes.data, 0, 0, fake, fake,
                  None, None),                                                                      # bad next state
        lambda: f(1 << 31, 1, fake, fake, fake, fake, 1, 1, 2, np.zeros(4, np.uint8).ctypes.data, 0, 0, fake, fake,
                  None, None),                                                                      # 2^32 product vertices
        lambda: f(4, 1, fake, fake, fake, fake, 1, 2, 1, np.zeros(4, np.uint8).ctypes.data, 0, 0, fake, fake,
                  None, None),                                                                      # rows narrower than n_props
    ]
    for i, c in enumerate(cases):
        assert c() == lbl.EINVAL, i
