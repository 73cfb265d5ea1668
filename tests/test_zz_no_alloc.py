"""GPU checks of lbl_label_frame_noalloc (the variant of lbl_label_frame that
allocates nothing: its intermediates live in the library's static device
array).  Through the C ABI, its labels equal lbl_label_frame's and the
oracle's byte for byte on two calls in a row, the second on a smaller
input; a frame whose intermediates do not fit is rejected before any device
work; the calls do not lower the device's free memory.

Every case prints what it runs (flushed) before touching the device.
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


def expect(a, O):
    return oracle.label_csr(a.row_ptr, a.col_idx, a.grid.n_cells, O, threads=THREADS)


def both(h, O, n_traj, stream):
    """Labels of lbl_label_frame_noalloc and of lbl_label_frame (the sparse
    kernel), on one stream, L pre-filled with 9 so unwritten bytes show."""
    n_props = O.shape[1]
    Od = torch.from_numpy(np.ascontiguousarray(O)).cuda()
    La = torch.full((n_traj, n_props), 9, dtype=torch.uint8, device="cuda")
    Lb = torch.full((n_traj, n_props), 9, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    lbl.label_frame_noalloc(h, Od, n_props, La, stream=stream)
    lbl.label_frame(h, Od, n_props, Lb, flags=lbl.KERNEL_AUTO, stream=stream)
    torch.cuda.synchronize()
    return La.cpu().numpy(), Lb.cpu().numpy()


def same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{what}: {len(bad)} labels differ, first at {bad[:5].tolist()}")


def test_noalloc_equals_label_frame_large_then_small():
    big = gen.make_abstraction(3)  # 200,000 x 512^2
    small = gen.make_abstraction(1)  # 1,000 x 64^2
    say(f"noalloc: load {big.n_traj} x {big.grid.n}^2 and {small.n_traj} x {small.grid.n}^2")
    hb = lbl.load_abstraction(big.grid.n, big.grid.n, big.row_ptr, big.col_idx)
    hs = lbl.load_abstraction(small.grid.n, small.grid.n, small.row_ptr, small.col_idx)
    try:
        s = torch.cuda.Stream()
        Ob = gen.make_frame(3, big.grid, 64, frame=2, rho=0.10)
        Os = gen.make_frame(1, small.grid, 8, frame=3)
        say("noalloc: oracle labels")
        wb, ws = expect(big, Ob), expect(small, Os)
        say("noalloc: call 1, 200,000 x 512^2 x 64")
        a1, b1 = both(hb, Ob, big.n_traj, s)
        same(a1, b1, "large: noalloc vs label_frame")
        same(a1, wb, "large: noalloc vs oracle")
        say("noalloc: call 2, 1,000 x 64^2 x 8")
        a2, b2 = both(hs, Os, small.n_traj, s)
        same(a2, b2, "small: noalloc vs label_frame")
        same(a2, ws, "small: noalloc vs oracle")
        # again large, then small, on a new stream: the array keeps the last
        # call's contents, which must not leak into the next
        s2 = torch.cuda.Stream()
        say("noalloc: calls 3 and 4 on another stream")
        a3, _ = both(hb, Ob, big.n_traj, s2)
        same(a3, wb, "large again: noalloc vs oracle")
        a4, _ = both(hs, Os, small.n_traj, s2)
        same(a4, ws, "small again: noalloc vs oracle")
        # two propositions: the direct-mask kernels, whose word masks take the
        # array's front and which write L without a combine
        say("noalloc: call 5, 200,000 x 512^2 x 2")
        a5, b5 = both(hb, np.ascontiguousarray(Ob[:, :2]), big.n_traj, s2)
        same(a5, b5, "two propositions: noalloc vs label_frame")
        same(a5, wb[:, :2], "two propositions: noalloc vs oracle")
    finally:
        lbl.free_abstraction(hb)
        lbl.free_abstraction(hs)


def test_noalloc_bitpacked_abstraction_and_ragged_rows():
    # an abstraction without the sparse layout takes the bitpacked kernel;
    # 8257 rows (two row blocks, the second 65 rows) on a 24 x 40 grid
    rng = np.random.default_rng(7)
    nx, ny, n_traj, n_props = 24, 40, 8257, 17
    counts = rng.binomial(nx * ny, 0.05, n_traj)
    counts[rng.random(n_traj) < 0.1] = 0
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint64)
    col_idx = rng.integers(0, nx * ny, int(row_ptr[-1])).astype(np.uint32)
    a = type("A", (), {"row_ptr": row_ptr, "col_idx": col_idx,
                       "grid": type("G", (), {"n_cells": nx * ny})()})()
    O = (rng.random((nx * ny, n_props)) < 0.1).astype(np.uint8) * rng.integers(1, 255, (nx * ny, n_props)).astype(np.uint8)
    want = expect(a, O)
    for flags, what in ((0, "sparse"), (lbl.LOAD_NO_SPARSE, "bitpacked")):
        say(f"noalloc: ragged {n_traj} x {nx}x{ny} x {n_props}, {what} layout")
        h = lbl.load_abstraction(nx, ny, row_ptr, col_idx, flags)
        try:
            got, ref = both(h, O, n_traj, torch.cuda.current_stream())
            same(got, ref, f"ragged {what}: noalloc vs label_frame")
            same(got, want, f"ragged {what}: noalloc vs oracle")
        finally:
            lbl.free_abstraction(h)


def test_noalloc_rejects_what_does_not_fit_and_allocates_nothing():
    # 2048^2 cells = 65,536 words: a frame of 40 propositions needs 128 MiB of
    # 64-bit nibble tables, more than the array; one of 4 needs 2 MiB of
    # per-word masks (the direct-mask kernels) and fits
    n = 2048
    row_ptr = np.array([0, 3, 3, 5], np.uint64)
    col_idx = np.array([0, n * n - 1, 12345, 7, 4000000], np.uint32)
    say("noalloc: 2048^2 grid, expect a size error at 40 propositions")
    h = lbl.load_abstraction(n, n, row_ptr, col_idx)
    try:
        Od = torch.zeros((n * n, 40), dtype=torch.uint8, device="cuda")
        Ld = torch.full((3, 40), 9, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(lbl.LblError) as e:
            lbl.label_frame_noalloc(h, Od, 40, Ld)
        assert "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert (Ld.cpu().numpy() == 9).all()
        say("noalloc: 2048^2 grid, 4 propositions fit")
        rng = np.random.default_rng(4)
        O4 = (rng.random((n * n, 4)) < 0.5).astype(np.uint8)
        L4 = torch.full((3, 4), 9, dtype=torch.uint8, device="cuda")
        lbl.label_frame_noalloc(h, torch.from_numpy(O4).cuda(), 4, L4)
        torch.cuda.synchronize()
        same(L4.cpu().numpy(), oracle.label_csr(row_ptr, col_idx, n * n, O4), "2048^2, 4 propositions")
    finally:
        lbl.free_abstraction(h)
    # free device memory is unchanged by calls on a stream lbl_label_frame
    # never used (which would allocate that stream's workspace)
    small = gen.make_abstraction(1)
    hs = lbl.load_abstraction(small.grid.n, small.grid.n, small.row_ptr, small.col_idx)
    try:
        O = gen.make_frame(1, small.grid, 8, frame=5)
        Od = torch.from_numpy(O).cuda()
        Ld = torch.full((small.n_traj, 8), 9, dtype=torch.uint8, device="cuda")
        s = torch.cuda.Stream()
        # the runtime sets up a stream's hardware queue on its first launch
        # (memory of its own): a fill on that stream does that first
        with torch.cuda.stream(s):
            Ld.fill_(9)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        say("noalloc: two calls on a new stream, free memory before and after")
        for _ in range(2):
            lbl.label_frame_noalloc(hs, Od, 8, Ld, stream=s)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert free0 - free1 < (1 << 20), (free0, free1)
        same(Ld.cpu().numpy(), expect(small, O), "new stream: noalloc vs oracle")
    finally:
        lbl.free_abstraction(hs)
