"""GPU parity on the time-augmented workload of Sec. 5 (the plane times time,
2^21 cells, transitions at 0.0223% occupancy, the two propositions of Table 1
at about 1% and 90%), and the sparse-only load that holds the largest of
Table 1's transition systems (1,097,702 rows; 288 GB as bitpacked rows).

Expected labels come only from the oracle (whole L at every size, Table 1's
five included); every case prints what it runs first.
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
TABLE1_ROWS = (154776, 295700, 568958, 836276, 1097702)


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


def load(A, flags=0):
    return lbl.load_abstraction(A.grid.nx, A.grid.ny, A.row_ptr, A.col_idx, flags)


def label(h, O, n_traj, kernel=lbl.KERNEL_SPARSE):
    n_props = O.shape[1]
    Od = torch.from_numpy(np.ascontiguousarray(O)).cuda()
    Ld = torch.full((n_traj, n_props), 9, dtype=torch.uint8, device="cuda")
    lbl.label_frame(h, Od, n_props, Ld, flags=kernel)
    torch.cuda.synchronize()
    return Ld.cpu().numpy()


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{what}: {len(bad)} labels differ, first at {bad[:5].tolist()}")


@pytest.mark.parametrize("n_traj,g", [
    (20000, gen.SpaceTimeGrid(n=128, n_tau=16)),   # 2^18 cells, 3 row blocks, ragged tail, one run
    (40000, gen.SpaceTimeGrid()),                  # 2^21 cells: three sparse-only runs
])
def test_spacetime_whole_L(n_traj, g):
    say(f"spacetime whole L: {n_traj} transitions, grid {g.nx}x{g.ny}")
    A = gen.spacetime_abstraction(n_traj, g, threads=THREADS)
    frames = [gen.spacetime_frame(g, f) for f in range(2)]
    want = [oracle.label_csr(A.row_ptr, A.col_idx, g.n_cells, O, threads=THREADS) for O in frames]
    assert 0 < want[0][:, 0].mean() < 1 and 0 < want[0][:, 1].mean() < 1  # both labels occur
    for flags, kernels in ((0, (lbl.KERNEL_SPARSE, lbl.KERNEL_BITS)), (lbl.LOAD_SPARSE_ONLY, (lbl.KERNEL_SPARSE,))):
        h = load(A, flags)
        try:
            info = lbl.abstraction_info(h)
            assert (info["bits_bytes"] == 0) == bool(flags & lbl.LOAD_SPARSE_ONLY)
            for O, w in zip(frames, want):
                for k in kernels:
                    say(f"  load flags {flags:#x} kernel {k:#x}")
                    assert_same(label(h, O, n_traj, k), w, f"load {flags:#x} kernel {k:#x}")
                    # one proposition at a time, as each of Table 1's columns
                    assert_same(label(h, O[:, 1:2], n_traj, k), w[:, 1:2], f"prop 1 alone, kernel {k:#x}")
        finally:
            lbl.free_abstraction(h)


def test_sparse_only_from_device_csr():
    g = gen.SpaceTimeGrid()
    n = 20000
    say(f"sparse-only load from device CSR: {n} transitions")
    A = gen.spacetime_abstraction(n, g, threads=THREADS)
    O = gen.spacetime_frame(g, 3)
    rp = torch.from_numpy(A.row_ptr.view(np.int64)).cuda()
    ci = torch.from_numpy(A.col_idx.view(np.int32)).cuda()
    h = lbl.load_abstraction(g.nx, g.ny, rp, ci, lbl.LOAD_SPARSE_ONLY | lbl.LOAD_INPUT_DEVICE)
    try:
        assert_same(label(h, O, n), oracle.label_csr(A.row_ptr, A.col_idx, g.n_cells, O, threads=THREADS),
                    "device CSR, sparse only")
    finally:
        lbl.free_abstraction(h)


def test_sparse_only_rejects_bitpacked_kernels_and_mixed_batches():
    g = gen.SpaceTimeGrid(n=128, n_tau=16)
    A = gen.spacetime_abstraction(3000, g, threads=THREADS)
    O = gen.spacetime_frame(g, 0)
    say("sparse-only: kernel and batch rejections")
    hs = load(A, lbl.LOAD_SPARSE_ONLY)
    hn = load(A, lbl.LOAD_NO_SPARSE)
    try:
        for k in (lbl.KERNEL_BITS, lbl.KERNEL_MFMA, lbl.KERNEL_MFMA_I8):
            with pytest.raises(lbl.LblError) as e:
                label(hs, O, 3000, k)
            assert e.value.status == lbl.EINVAL
        Od = torch.from_numpy(O).cuda()
        L1 = torch.zeros((3000, 2), dtype=torch.uint8, device="cuda")
        L2 = torch.zeros((3000, 2), dtype=torch.uint8, device="cuda")
        with pytest.raises(lbl.LblError) as e:
            lbl.label_batch([(hs, Od, 2, L1), (hn, Od, 2, L2)])
        assert e.value.status == lbl.EINVAL
        torch.cuda.synchronize()
        # the autotuner only times the sparse kernel, and AUTO then uses it
        lbl.tune(hs, Od, 2)
        assert "sparse" in lbl.tune_describe(hs, 2)
        want = oracle.label_csr(A.row_ptr, A.col_idx, g.n_cells, O)
        assert_same(label(hs, O, 3000, lbl.KERNEL_AUTO), want, "sparse only, auto after tuning")
    finally:
        lbl.free_abstraction(hs)
        lbl.free_abstraction(hn)


@pytest.mark.parametrize("n_traj", TABLE1_ROWS)
def test_table1_sizes_whole_L(n_traj):
    """Every transition of each of Table 1's five systems, both propositions
    together and each alone (as Table 1 times them), against the oracle."""
    g = gen.SpaceTimeGrid()
    say(f"Table 1 size {n_traj}: generating")
    A = gen.spacetime_abstraction(n_traj, g, threads=THREADS)
    O = gen.spacetime_frame(g, 0)
    say("  oracle")
    want = oracle.label_csr(A.row_ptr, A.col_idx, g.n_cells, O, threads=THREADS)
    assert 0 < want[:, 0].mean() < 1 and 0 < want[:, 1].mean() < 1
    say(f"  sparse-only load, {len(A.col_idx)} cells")
    h = load(A, lbl.LOAD_SPARSE_ONLY)
    try:
        info = lbl.abstraction_info(h)
        assert info["bits_bytes"] == 0 and info["set_cells"] == len(A.col_idx)
        say(f"  label, {info['sparse_entries']} entries")
        L = label(h, O, n_traj)
        assert_same(L, want, f"{n_traj} rows, both propositions")
        for p in range(2):
            say(f"  proposition {p} alone")
            assert_same(label(h, np.ascontiguousarray(O[:, p:p + 1]), n_traj), want[:, p:p + 1],
                        f"{n_traj} rows, proposition {p} alone")
    finally:
        lbl.free_abstraction(h)
    if n_traj == TABLE1_ROWS[0]:
        # the full load (bitpacked rows, 40.6 GB) labels identically
        say("  full load for comparison")
        h = load(A)
        try:
            assert_same(label(h, O, n_traj), want, "full load, sparse kernel")
            assert_same(label(h, O, n_traj, lbl.KERNEL_BITS), want, "full load, bitpacked kernel")
        finally:
            lbl.free_abstraction(h)
