"""GPU parity: the HIP library's labels equal the oracle's, byte for byte.

Every case prints what it runs (flushed) before touching the device.  Inputs
come from the seeded generator; expected labels only from the oracle.
"""
import os
import sys

import numpy as np
import pytest

import gen
import oracle

torch = pytest.importorskip("torch")
from paper_1810_02612_amd import lbl  # noqa: E402

pytestmark = pytest.mark.gpu

KERNELS = {"sparse": lbl.KERNEL_SPARSE, "bits": lbl.KERNEL_BITS, "mfma": lbl.KERNEL_MFMA,
           "mfma_i8": lbl.KERNEL_MFMA_I8, "auto": lbl.KERNEL_AUTO}
THREADS = min(16, os.cpu_count() or 1)


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def expect(a, O, rows=None):
    return oracle.label_csr(a.row_ptr, a.col_idx, a.grid.n_cells, O, rows=rows, threads=THREADS)


def load(a, flags=0):
    return lbl.load_abstraction(a.grid.nx if hasattr(a.grid, "nx") else a.grid.n,
                                a.grid.ny if hasattr(a.grid, "ny") else a.grid.n, a.row_ptr, a.col_idx, flags)


def label(h, O, n_traj, kernel, host=False, stream=None):
    n_props = O.shape[1]
    if host:
        L = np.full((n_traj, n_props), 9, np.uint8)
        lbl.label_frame(h, np.ascontiguousarray(O), n_props, L, flags=kernel | lbl.HOST_PTRS)
        return L
    Od = torch.from_numpy(np.ascontiguousarray(O)).cuda()
    Ld = torch.full((n_traj, n_props), 9, dtype=torch.uint8, device="cuda")
    lbl.label_frame(h, Od, n_props, Ld, flags=kernel, stream=stream)
    torch.cuda.synchronize()
    return Ld.cpu().numpy()


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{what}: {len(bad)} labels differ, first at {bad[:5].tolist()} "
                             f"got {got[tuple(bad[0])]} want {want[tuple(bad[0])]}")


class Csr:
    """A T in CSR form on an nx x ny grid (cells row-major)."""

    def __init__(self, nx, ny, row_ptr, col_idx):
        self.grid = type("G", (), {"nx": nx, "ny": ny, "n_cells": nx * ny})()
        self.row_ptr = np.ascontiguousarray(row_ptr, np.uint64)
        self.col_idx = np.ascontiguousarray(col_idx, np.uint32)
        self.n_traj = len(self.row_ptr) - 1


def random_csr(rng, n_traj, nx, ny, density, empty_frac=0.1, dup=True):
    n_cells = nx * ny
    counts = rng.binomial(n_cells, density, n_traj)
    counts[rng.random(n_traj) < empty_frac] = 0
    cols = [rng.choice(n_cells, size=c, replace=False) for c in counts]
    if dup:
        cols = [np.concatenate([c, c[: len(c) // 3]]) for c in cols]  # repeated ids, unsorted
        cols = [rng.permutation(c) for c in cols]
    counts = np.array([len(c) for c in cols])
    rp = np.zeros(n_traj + 1, np.uint64)
    np.cumsum(counts, out=rp[1:])
    ci = np.concatenate(cols).astype(np.uint32) if counts.sum() else np.zeros(0, np.uint32)
    return Csr(nx, ny, rp, ci)


# ------------------------------------------------------------------ configs

@pytest.fixture(scope="module")
def cfg1():
    say("generate 1k x 64^2 abstraction")
    return gen.make_abstraction(1)


@pytest.fixture(scope="module")
def cfg2():
    say("generate 50k x 256^2 abstraction")
    return gen.make_abstraction(2)


@pytest.mark.parametrize("host", [False, True])
def test_cfg1_every_kernel(cfg1, host):
    a = cfg1
    h = lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx, lbl.LOAD_KEEP_INT8)
    try:
        for f in range(3):
            O = gen.make_frame(1, a.grid, 8, frame=f)
            want = expect(a, O)
            for name, k in KERNELS.items():
                say(f"cfg1 frame {f} kernel {name} host={host}")
                assert_same(label(h, O, a.n_traj, k, host), want, f"cfg1/{name}/frame{f}")
    finally:
        lbl.free_abstraction(h)


def test_cfg2_every_kernel(cfg2):
    a = cfg2
    say("cfg2 load with int8 copy")
    h = lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx, lbl.LOAD_KEEP_INT8)
    try:
        info = lbl.abstraction_info(h)
        assert info["set_cells"] == len(np.unique(a.row_ptr[:-1]))*0 + int(a.row_ptr[-1])  # generator ids are unique
        for f in range(2):
            O = gen.make_frame(2, a.grid, 32, frame=f)
            want = expect(a, O)
            for name, k in KERNELS.items():
                say(f"cfg2 frame {f} kernel {name}")
                assert_same(label(h, O, a.n_traj, k), want, f"cfg2/{name}/frame{f}")
    finally:
        lbl.free_abstraction(h)


@pytest.mark.parametrize("rho", [0.01, 0.10, 0.40])
def test_cfg3_rows_subset_densities(rho):
    say(f"cfg3 20k-row subset, rho={rho}")
    a = gen.make_abstraction(3, n_traj=20000)
    h = lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx, lbl.LOAD_KEEP_INT8)
    try:
        O = gen.make_frame(3, a.grid, 64, frame=0, rho=rho)
        want = expect(a, O)
        for name, k in KERNELS.items():
            say(f"cfg3 subset rho={rho} kernel {name}")
            assert_same(label(h, O, a.n_traj, k), want, f"cfg3/{name}/rho{rho}")
    finally:
        lbl.free_abstraction(h)


@pytest.fixture(scope="module")
def cfg3_full():
    say("cfg3 full 200k x 512^2: generate")
    a = gen.make_abstraction(3)
    say("cfg3 full: load with the int8 copy (52 GB)")
    h = lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx, lbl.LOAD_KEEP_INT8)
    yield a, h
    lbl.free_abstraction(h)


@pytest.mark.parametrize("rho", [0.01, 0.10, 0.40])
def test_cfg3_full_size_whole_L(cfg3_full, rho):
    """The headline workload (200,000 x 512^2 x 64), every row and column
    compared with the oracle, for every kernel, at the three O densities."""
    a, h = cfg3_full
    info = lbl.abstraction_info(h)
    assert info["set_cells"] == int(a.row_ptr[-1])
    O = gen.make_frame(3, a.grid, 64, frame=1, rho=rho)
    say(f"cfg3 full rho={rho}: oracle")
    want = expect(a, O)
    empty = np.nonzero(np.diff(a.row_ptr) == 0)[0]
    for name, k in KERNELS.items():
        say(f"cfg3 full rho={rho} kernel {name}")
        L = label(h, O, a.n_traj, k)
        assert_same(L, want, f"cfg3-full/{name}/rho{rho}")
        assert not L[empty].any()


# ------------------------------------------------------------------ edges

@pytest.mark.parametrize("nx,ny,n_traj,n_props", [
    (8, 8, 1, 1), (8, 8, 3, 64), (24, 8, 65, 7), (24, 40, 130, 17), (64, 64, 1007, 33),
    (40, 24, 257, 63), (136, 8, 33, 16), (8, 136, 77, 2),
    # three and four propositions (direct per-word masks), two row blocks
    (24, 24, 8300, 3), (56, 8, 700, 4),
    # 48 and 32 columns (three and two 16-byte units per row), 8257 rows: two
    # row blocks of the sparse layout, the second one 65 rows long
    (16, 16, 8257, 48), (32, 16, 130, 32),
])
def test_ragged_shapes(nx, ny, n_traj, n_props):
    rng = np.random.default_rng(nx * 1000 + ny + n_traj)
    a = random_csr(rng, n_traj, nx, ny, 0.05)
    say(f"ragged nx={nx} ny={ny} n_traj={n_traj} n_props={n_props}")
    h = lbl.load_abstraction(nx, ny, a.row_ptr, a.col_idx, lbl.LOAD_KEEP_INT8)
    try:
        O = rng.integers(0, 256, (nx * ny, n_props)).astype(np.uint8)
        O[rng.random(O.shape) < 0.9] = 0
        want = expect(a, O)
        for name, k in KERNELS.items():
            assert_same(label(h, O, n_traj, k), want, f"ragged/{name}")
        # host O and L (staged through device buffers), whichever mask width
        assert_same(label(h, O, n_traj, lbl.KERNEL_SPARSE, host=True), want, "ragged/sparse/host")
    finally:
        lbl.free_abstraction(h)


def test_identity_and_single_cell_frames():
    rng = np.random.default_rng(9)
    nx = ny = 16
    a = random_csr(rng, 200, nx, ny, 0.03)
    T = np.zeros((200, nx * ny), np.uint8)
    for t in range(200):
        T[t, a.col_idx[a.row_ptr[t]:a.row_ptr[t + 1]].astype(np.int64)] = 1
    h = lbl.load_abstraction(nx, ny, a.row_ptr, a.col_idx, lbl.LOAD_KEEP_INT8)
    try:
        for name, k in KERNELS.items():
            say(f"identity frames kernel {name}")
            for c0 in range(0, nx * ny, 64):
                O = np.zeros((nx * ny, 64), np.uint8)
                O[np.arange(c0, c0 + 64), np.arange(64)] = 1  # O = e_c columns
                assert_same(label(h, O, 200, k), T[:, c0:c0 + 64], f"identity/{name}/{c0}")
            ones = np.full((nx * ny, 3), 255, np.uint8)
            assert_same(label(h, ones, 200, k), np.repeat((T.sum(1) > 0)[:, None], 3, 1).astype(np.uint8),
                        f"ones/{name}")
    finally:
        lbl.free_abstraction(h)


def test_dense_and_device_csr_loads_agree(cfg1):
    a = cfg1
    O = gen.make_frame(1, a.grid, 8, frame=5)
    want = expect(a, O)
    say("dense host load")
    h1 = lbl.load_abstraction_dense(a.grid.n, a.grid.n, a.dense())
    say("dense device load")
    h2 = lbl.load_abstraction_dense(a.grid.n, a.grid.n, torch.from_numpy(a.dense()).cuda(), lbl.LOAD_INPUT_DEVICE)
    say("csr device load")
    h3 = lbl.load_abstraction(a.grid.n, a.grid.n, torch.from_numpy(a.row_ptr.astype(np.int64)).cuda(),
                              torch.from_numpy(a.col_idx.astype(np.int32)).cuda(), lbl.LOAD_INPUT_DEVICE)
    try:
        for h in (h1, h2, h3):
            for k in (lbl.KERNEL_BITS, lbl.KERNEL_SPARSE):
                assert_same(label(h, O, a.n_traj, k), want, "alt-load")
    finally:
        for h in (h1, h2, h3):
            lbl.free_abstraction(h)


def zorder_ids(n):
    """z-order index (Alg. zcurve, the oracle's descent) of every row-major cell
    of an n x n grid."""
    d = 2 * (n.bit_length() - 1)
    z = np.empty(n * n, np.int64)
    for iy in range(n):
        for ix in range(n):
            z[iy * n + ix] = oracle.zorder([ix + 0.5, iy + 0.5], [0.0, 0.0], [float(n), float(n)], d)
    assert np.array_equal(np.sort(z), np.arange(n * n))
    return z


@pytest.mark.parametrize("cfg", [1, 2])
def test_morton_cell_ids_give_the_row_major_labels(cfg, cfg1, cfg2):
    """T and O numbered by z-order index (LBL_MORTON) label exactly as the
    same T and O numbered row-major."""
    a = cfg1 if cfg == 1 else cfg2
    n, n_props = a.grid.n, (8 if cfg == 1 else 32)
    z = zorder_ids(n)
    O = gen.make_frame(cfg, a.grid, n_props, frame=3)
    want = expect(a, O)
    Oz = np.empty_like(O)
    Oz[z] = O
    col_z = z[a.col_idx.astype(np.int64)].astype(np.uint32)
    say(f"morton cfg{cfg}: csr load")
    h = lbl.load_abstraction(n, n, a.row_ptr, col_z, lbl.LOAD_KEEP_INT8, cell_order=lbl.MORTON)
    try:
        for name, k in KERNELS.items():
            say(f"morton cfg{cfg} kernel {name}")
            assert_same(label(h, Oz, a.n_traj, k), want, f"morton/cfg{cfg}/{name}")
        for p in (1, 2, 3, 4):
            say(f"morton cfg{cfg} sparse kernel, first {p} propositions")
            assert_same(label(h, np.ascontiguousarray(Oz[:, :p]), a.n_traj, lbl.KERNEL_SPARSE), want[:, :p],
                        f"morton/cfg{cfg}/{p} props")
    finally:
        lbl.free_abstraction(h)
    if cfg == 1:
        say("morton cfg1: dense load")
        Tz = np.zeros_like(a.dense())
        Tz[:, z] = a.dense()
        h = lbl.load_abstraction_dense(n, n, Tz, cell_order=lbl.MORTON)
        try:
            for k in (lbl.KERNEL_SPARSE, lbl.KERNEL_BITS):
                assert_same(label(h, Oz, a.n_traj, k), want, "morton/dense")
        finally:
            lbl.free_abstraction(h)
        say("morton cfg1: rasterizer writes z-order rows")
        sh = gen.frame_shapes(1, a.grid, 8, 3)
        shapes = lbl.shapes_array(sh.kind, sh.prop, sh.cx, sh.cy, sh.a, sh.b)
        Or = torch.empty((n * n, 8), dtype=torch.uint8, device="cuda")
        lbl.raster_frame(n, n, a.grid.res, shapes, 8, Or, cell_order=lbl.MORTON)
        torch.cuda.synchronize()
        assert np.array_equal(Or.cpu().numpy(), Oz)




@pytest.mark.parametrize("n_props", [1, 2, 4, 8, 64])
def test_empty_and_single_entry_abstractions(n_props):
    """Degenerate layouts: no set cell at all (every label 0, every byte of L
    still written), and one trajectory with one set cell (labels equal that
    cell's row of O), with every kernel and the direct-mask, narrow and wide
    mask widths."""
    rng = np.random.default_rng(n_props)
    nx = ny = 64
    O = rng.integers(0, 2, (nx * ny, n_props)).astype(np.uint8)
    O[1234] = 1  # the single entry's cell meets every proposition
    cases = {
        "empty": (np.zeros(301, np.uint64), np.zeros(0, np.uint32), 300),
        "one cell": (np.array([0, 1], np.uint64), np.array([1234], np.uint32), 1),
    }
    for what, (row_ptr, col_idx, n_traj) in cases.items():
        say(f"degenerate {what}, {n_props} propositions")
        h = lbl.load_abstraction(nx, ny, row_ptr, col_idx, lbl.LOAD_KEEP_INT8)
        try:
            want = oracle.label_csr(row_ptr, col_idx, nx * ny, O)
            assert want.sum() == (0 if what == "empty" else n_props)
            for name, k in KERNELS.items():
                assert_same(label(h, O, n_traj, k), want, f"{what}/{name}/{n_props}")
        finally:
            lbl.free_abstraction(h)


@pytest.mark.parametrize("n_props", [1, 2, 3, 8, 64])
def test_unaligned_L_and_bytes_around_it(n_props):
    """L starting 3 bytes into a larger device buffer (and ending off a
    16-byte boundary): every label byte equals the oracle's and no byte
    outside L changes (the direct-mask path zeroes L before the tiles set
    it, by whole 16-byte units inside L only)."""
    rng = np.random.default_rng(300 + n_props)
    a = random_csr(rng, 5003, 48, 40, 0.06)
    O = (rng.random((48 * 40, n_props)) < 0.2).astype(np.uint8)
    want = expect(a, O)
    h = lbl.load_abstraction(48, 40, a.row_ptr, a.col_idx)
    try:
        n = a.n_traj * n_props
        buf = torch.full((n + 64,), 0xA5, dtype=torch.uint8, device="cuda")
        Lv = buf[3:3 + n]
        say(f"unaligned L, {n_props} propositions")
        lbl.label_frame(h, torch.from_numpy(O).cuda(), n_props, Lv, flags=lbl.KERNEL_SPARSE)
        torch.cuda.synchronize()
        got = buf.cpu().numpy()
        assert (got[:3] == 0xA5).all() and (got[3 + n:] == 0xA5).all()
        assert_same(got[3:3 + n].reshape(a.n_traj, n_props), want, f"unaligned L, {n_props} propositions")
    finally:
        lbl.free_abstraction(h)

@pytest.mark.parametrize("n_props", [2, 3, 4, 6, 12, 20, 34, 48, 60, 62, 64])
@pytest.mark.parametrize("o_off", [0, 1, 2, 4])
def test_frame_bytes_at_every_load_width(n_props, o_off):
    """O starting o_off bytes into a larger device buffer, for proposition
    counts whose rows the table kernels read in 16-byte units taken in
    memory order (64), in 16-, 4- or 2-byte pieces per cell (48, 60 and 12
    and 20, 6 and 34 and 62: more than one group of four loads for 20, 34, 60
    and 62) or, once O is moved off those alignments, byte by byte; and
    frames of 2, 3 and 4 propositions, whose per-word masks are read in 2-,
    1- and 4-byte pieces: every label equals the oracle's."""
    rng = np.random.default_rng(500 + 7 * n_props + o_off)
    nx, ny = 48, 40
    a = random_csr(rng, 9000, nx, ny, 0.04)
    O = rng.integers(0, 256, (nx * ny, n_props)).astype(np.uint8)
    O[rng.random(O.shape) < 0.85] = 0
    want = expect(a, O)
    h = lbl.load_abstraction(nx, ny, a.row_ptr, a.col_idx)
    try:
        n = O.size
        buf = torch.zeros((n + 16,), dtype=torch.uint8, device="cuda")
        buf[o_off:o_off + n] = torch.from_numpy(O.reshape(-1)).cuda()
        Ov = buf[o_off:o_off + n]
        L = torch.full((a.n_traj, n_props), 9, dtype=torch.uint8, device="cuda")
        say(f"O at offset {o_off}, {n_props} propositions")
        lbl.label_frame(h, Ov, n_props, L, flags=lbl.KERNEL_SPARSE)
        torch.cuda.synchronize()
        assert_same(L.cpu().numpy(), want, f"O offset {o_off}, {n_props} propositions")
    finally:
        lbl.free_abstraction(h)


def test_direct_masks_and_their_fallback():
    """Frames of at most 4 propositions take the direct-mask kernels (per-word
    masks, no combine) unless a tile part's segment masks would not fit the
    kernel's LDS; then the 32-bit nibble kernels run.  1,966,080 rows of one
    random cell each on a 1024 x 1024 grid (240 row blocks of ~6,400 segments
    of about one entry) put about 3,000 segments in a part: under the
    one-proposition budget (6,144), over the four-proposition one (1,536).
    The kernels that ran are told apart by the profile counts (the nibble
    path launches a combine); both must equal the oracle."""
    n_side, n_traj = 1024, 240 * 8192
    rng = np.random.default_rng(240)
    row_ptr = np.arange(n_traj + 1, dtype=np.uint64)
    col_idx = rng.integers(0, n_side * n_side, n_traj).astype(np.uint32)
    say(f"direct fallback: sparse-only load of {n_traj} single-cell rows on {n_side}^2")
    h = lbl.load_abstraction(n_side, n_side, row_ptr, col_idx, lbl.LOAD_SPARSE_ONLY)
    try:
        info = lbl.abstraction_info(h)
        assert info["sparse_tiles_direct"] > 0 and info["sparse_frame_bytes_direct"] > 0
        O = (rng.random((n_side * n_side, 4)) < 0.3).astype(np.uint8)
        want = oracle.label_csr(row_ptr, col_idx, n_side * n_side, O, threads=THREADS)
        for n_props, direct in ((1, True), (4, False)):
            say(f"direct fallback: {n_props} propositions, direct expected {direct}")
            lbl.profile_enable(True)
            L = label(h, O[:, :n_props], n_traj, lbl.KERNEL_SPARSE)
            prof = lbl.profile_read()
            lbl.profile_enable(False)
            assert prof["label_launches"] == 1
            assert (prof["emit_launches"] == 0) == direct, prof
            assert_same(L, want[:, :n_props], f"direct fallback, {n_props} propositions")
    finally:
        lbl.free_abstraction(h)

def test_errors_on_device():
    rng = np.random.default_rng(1)
    a = random_csr(rng, 10, 8, 8, 0.2)
    say("error paths")
    bad = a.col_idx.copy()
    bad[-1] = 64
    with pytest.raises(lbl.LblError) as e:
        lbl.load_abstraction(8, 8, a.row_ptr, bad)
    assert e.value.status == lbl.EINVAL
    h = lbl.load_abstraction(8, 8, a.row_ptr, a.col_idx)
    try:
        O = torch.zeros((64, 8), dtype=torch.uint8, device="cuda")
        L = torch.zeros((10, 8), dtype=torch.uint8, device="cuda")
        with pytest.raises(lbl.LblError):
            lbl.label_frame(h, O, 65, L)
        with pytest.raises(lbl.LblError):
            lbl.label_frame(h, O, 0, L)
        with pytest.raises(lbl.LblError) as e:
            lbl.label_frame(h, O, 8, L, flags=lbl.KERNEL_MFMA_I8)
        assert "KEEP_INT8" in str(e.value)
    finally:
        lbl.free_abstraction(h)


def test_two_streams_same_abstraction(cfg1):
    a = cfg1
    h = lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx)
    try:
        Os = [gen.make_frame(1, a.grid, 8, frame=10 + i) for i in range(2)]
        wants = [expect(a, O) for O in Os]
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        Od = [torch.from_numpy(O).cuda() for O in Os]
        Ld = [torch.zeros((a.n_traj, 8), dtype=torch.uint8, device="cuda") for _ in Os]
        torch.cuda.synchronize()
        say("two streams")
        for rep in range(5):
            for i in range(2):
                lbl.label_frame(h, Od[i], 8, Ld[i], flags=(lbl.KERNEL_BITS, lbl.KERNEL_SPARSE)[rep % 2],
                                stream=streams[i])
        torch.cuda.synchronize()
        for i in range(2):
            assert_same(Ld[i].cpu().numpy(), wants[i], f"stream{i}")
    finally:
        lbl.free_abstraction(h)
