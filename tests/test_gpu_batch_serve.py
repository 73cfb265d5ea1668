"""GPU parity of the batched and served paths against the oracle, graph
replays, admission by memory, and the alone-versus-mix identity."""
import os
import sys
import threading

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


class Abs:
    def __init__(self, a):
        self.a = a
        self.h = lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx)

    def expect(self, O):
        return oracle.label_csr(self.a.row_ptr, self.a.col_idx, self.a.grid.n_cells, O, threads=THREADS)


@pytest.fixture(scope="module")
def abstractions():
    say("generate six scaled uneven abstractions (128^2, 256^2, 512^2 grids)")
    out = [Abs(gen.make_batch_abstraction(i, scale=0.03)) for i in range(6)]
    yield out
    for x in out:
        lbl.free_abstraction(x.h)


def frames_for(x, i, k, n_props=None):
    n_props = n_props or gen.batch_frame_props(4, i, k)
    return gen.make_frame(4, x.a.grid, n_props, frame=k, abstraction=i, rho_lo=0.05, rho_hi=0.30)


def make_jobs(abstractions, per_abs=3, seed=0):
    jobs, wants = [], []
    for i, x in enumerate(abstractions):
        for k in range(per_abs):
            O = frames_for(x, i, k + seed)
            n_props = O.shape[1]
            Od = torch.from_numpy(O).cuda()
            Ld = torch.full((x.a.n_traj, n_props), 9, dtype=torch.uint8, device="cuda")
            jobs.append((x.h, Od, n_props, Ld))
            wants.append(x.expect(O))
    return jobs, wants


def check_jobs(jobs, wants, what):
    torch.cuda.synchronize()
    for j, ((h, Od, n_props, Ld), want) in enumerate(zip(jobs, wants)):
        got = Ld.cpu().numpy()
        if not np.array_equal(got, want):
            raise AssertionError(f"{what}: job {j} differs in {(got != want).sum()} labels")


def test_batch_matches_oracle_and_replays(abstractions):
    jobs, wants = make_jobs(abstractions, per_abs=3)
    say(f"batch of {len(jobs)} jobs")
    lbl.label_batch(jobs)
    check_jobs(jobs, wants, "first launch")
    # replays of the cached graph, with eager work and synchronizations between them
    for rep in range(3):
        for (_, _, _, Ld) in jobs:
            Ld.fill_(7)
        torch.cuda.synchronize()
        lbl.label_batch(jobs)
        check_jobs(jobs, wants, f"replay {rep}")
    # same buffers, new frame contents: the replayed graph reads the new data
    new_wants = []
    for j, (h, Od, n_props, Ld) in enumerate(jobs):
        i = j // 3
        O = frames_for(abstractions[i], i, 50 + j, n_props=n_props)
        Od.copy_(torch.from_numpy(O))
        new_wants.append(abstractions[i].expect(O))
    torch.cuda.synchronize()
    lbl.label_batch(jobs)
    check_jobs(jobs, new_wants, "replay with new frames")


def test_batch_splits_more_than_1024_columns_on_one_abstraction(abstractions):
    x = abstractions[0]
    jobs, wants = [], []
    for k in range(18):  # 18 x 64 = 1152 columns > 1024 -> two passes
        O = frames_for(x, 0, 100 + k, n_props=64)
        jobs.append((x.h, torch.from_numpy(O).cuda(), 64,
                     torch.full((x.a.n_traj, 64), 9, dtype=torch.uint8, device="cuda")))
        wants.append(x.expect(O))
    say("batch with 1152 columns on one abstraction")
    lbl.label_batch(jobs)
    check_jobs(jobs, wants, "split")


def test_tuned_batch_still_matches(abstractions):
    jobs, wants = make_jobs(abstractions, per_abs=2, seed=7)
    say("tune batch tiles")
    lbl.tune_batch(jobs)
    for (_, _, _, Ld) in jobs:
        Ld.fill_(5)
    lbl.label_batch(jobs)
    check_jobs(jobs, wants, "tuned")


def test_batch_with_frames_and_labels_off_alignment(abstractions):
    """Every job's O and L start 1, 2 or 3 bytes into larger device buffers
    (the pack stages a job's bytes from a dword boundary, the combine writes
    the ends of each L block byte by byte): labels equal the oracle's and no
    byte around an L changes."""
    jobs, wants, bufs = [], [], []
    for i, x in enumerate(abstractions[:4]):
        for k in range(3):
            O = frames_for(x, i, 200 + k)
            n_props = O.shape[1]
            off = 1 + (i + k) % 3
            ob = torch.zeros((O.size + 8,), dtype=torch.uint8, device="cuda")
            ob[off:off + O.size] = torch.from_numpy(O.reshape(-1)).cuda()
            n_l = x.a.n_traj * n_props
            lb = torch.full((n_l + 8,), 0xA5, dtype=torch.uint8, device="cuda")
            jobs.append((x.h, ob[off:off + O.size], n_props, lb[off:off + n_l]))
            wants.append(x.expect(O))
            bufs.append((lb, off, n_l, n_props, x.a.n_traj))
    say(f"batch of {len(jobs)} jobs with O and L at byte offsets 1-3")
    lbl.label_batch(jobs)
    torch.cuda.synchronize()
    for j, ((lb, off, n_l, n_props, n_traj), want) in enumerate(zip(bufs, wants)):
        got = lb.cpu().numpy()
        assert (got[:off] == 0xA5).all() and (got[off + n_l:] == 0xA5).all(), f"job {j}: bytes around L changed"
        if not np.array_equal(got[off:off + n_l].reshape(n_traj, n_props), want):
            raise AssertionError(f"job {j} (offset {off}, {n_props} propositions) differs from the oracle")


def test_batch_equals_single_frames(abstractions):
    jobs, wants = make_jobs(abstractions[:2], per_abs=2, seed=3)
    singles = []
    for (h, Od, n_props, Ld) in jobs:
        L1 = torch.empty_like(Ld)
        lbl.label_frame(h, Od, n_props, L1, flags=lbl.KERNEL_BITS)
        singles.append(L1)
    lbl.label_batch(jobs)
    torch.cuda.synchronize()
    for (_, _, _, Ld), L1 in zip(jobs, singles):
        assert torch.equal(Ld, L1)


# ------------------------------------------------------------------ serving

def serve_and_check(server, reqs, n_threads=3):
    """Submit (h, Od, n_props, Ld, want) from several threads; wait and compare."""
    errors = []

    def client(chunk):
        try:
            tickets = [lbl.serve_submit(server, h, Od, n_props, Ld) for (h, Od, n_props, Ld, _) in chunk]
            for t, (_, _, _, Ld, want) in zip(tickets, chunk):
                st = lbl.serve_wait(server, t)
                if st != lbl.OK:
                    errors.append(f"ticket {t}: status {st} {lbl.last_error()}")
                    continue
                got = Ld.cpu().numpy()
                if not np.array_equal(got, want):
                    errors.append(f"ticket {t}: {(got != want).sum()} labels differ")
        except Exception as e:  # noqa: BLE001
            errors.append(repr(e))

    chunks = [reqs[i::n_threads] for i in range(n_threads)]
    th = [threading.Thread(target=client, args=(c,)) for c in chunks]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors[:5]


def requests(abstractions, n, seed, props=(8, 65)):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        i = int(rng.integers(0, len(abstractions)))
        x = abstractions[i]
        O = frames_for(x, i, 200 + seed * 1000 + k, n_props=int(rng.integers(*props)))
        out.append((x.h, torch.from_numpy(O).cuda(), O.shape[1],
                    torch.full((x.a.n_traj, O.shape[1]), 9, dtype=torch.uint8, device="cuda"), x.expect(O)))
    torch.cuda.synchronize()
    return out


def test_serve_matches_oracle_under_concurrency(abstractions):
    reqs = requests(abstractions, 40, seed=1)
    say("serve 40 requests from 3 threads")
    s = lbl.serve_start(hbm_budget_bytes=256 << 20, max_batch_frames=8, max_wait_us=0, n_streams=2)
    try:
        serve_and_check(s, reqs)
        st = lbl.serve_stats(s)
        assert st["completed"] == 40 and st["failed"] == 0
        assert st["p50_ms"] > 0 and st["p99_ms"] >= st["p50_ms"]
        assert st["budget_high_water"] <= 256 << 20
    finally:
        lbl.serve_stop(s)


def test_serve_few_propositions_match_oracle(abstractions):
    # frames of one to four propositions: a request served alone runs the
    # one-frame kernels for so few propositions (the direct-mask kernels
    # where the layout has them) in its slot's arena, requests served
    # together the batch kernels
    reqs = requests(abstractions, 24, seed=7, props=(1, 5))
    say("serve 24 requests of 1-4 propositions: 8 one at a time, 16 from 3 threads")
    s = lbl.serve_start(hbm_budget_bytes=256 << 20, max_batch_frames=8, max_wait_us=0, n_streams=2)
    try:
        for (h, Od, n_props, Ld, want) in reqs[:8]:
            assert lbl.serve_wait(s, lbl.serve_submit(s, h, Od, n_props, Ld)) == lbl.OK
            assert np.array_equal(Ld.cpu().numpy(), want)
        serve_and_check(s, reqs[8:])
        st = lbl.serve_stats(s)
        assert st["completed"] == 24 and st["failed"] == 0, st
    finally:
        lbl.serve_stop(s)


@pytest.mark.parametrize("n_props", [1, 8, 64])
def test_serve_degenerate_abstractions(n_props):
    """Served one at a time: an abstraction with no set cell (every label 0,
    every byte of L still written over its 9s) and one trajectory with one
    set cell (labels equal that cell's row of O)."""
    rng = np.random.default_rng(40 + n_props)
    nx = ny = 64
    O = rng.integers(0, 2, (nx * ny, n_props)).astype(np.uint8)
    O[1234] = 1
    cases = [(np.zeros(301, np.uint64), np.zeros(0, np.uint32), 300),
             (np.array([0, 1], np.uint64), np.array([1234], np.uint32), 1)]
    hs = [lbl.load_abstraction(nx, ny, rp, ci) for rp, ci, _ in cases]
    s = lbl.serve_start(hbm_budget_bytes=64 << 20, max_batch_frames=4, max_wait_us=0, n_streams=1)
    try:
        Od = torch.from_numpy(O).cuda()
        for h, (rp, ci, n_traj) in zip(hs, cases):
            want = oracle.label_csr(rp, ci, nx * ny, O)
            assert want.sum() == (0 if ci.size == 0 else n_props)
            for _ in range(2):
                Ld = torch.full((n_traj, n_props), 9, dtype=torch.uint8, device="cuda")
                torch.cuda.synchronize()
                assert lbl.serve_wait(s, lbl.serve_submit(s, h, Od, n_props, Ld)) == lbl.OK
                assert np.array_equal(Ld.cpu().numpy(), want)
        st = lbl.serve_stats(s)
        assert st["completed"] == 4 and st["failed"] == 0, st
    finally:
        lbl.serve_stop(s)
        for h in hs:
            lbl.free_abstraction(h)


def test_serve_result_same_alone_and_in_the_mix(abstractions):
    x, i = abstractions[5], 5
    O = frames_for(x, i, 999, n_props=37)
    Od = torch.from_numpy(O).cuda()
    want = x.expect(O)
    s = lbl.serve_start(hbm_budget_bytes=512 << 20, max_batch_frames=16, n_streams=3)
    try:
        say("alone")
        La = torch.full((x.a.n_traj, 37), 9, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()  # O and L are written before the request is submitted
        assert lbl.serve_wait(s, lbl.serve_submit(s, x.h, Od, 37, La)) == lbl.OK
        alone = La.cpu().numpy()
        say("in the mix")
        mix = requests(abstractions, 30, seed=2)
        Lm = torch.full((x.a.n_traj, 37), 9, dtype=torch.uint8, device="cuda")
        mix.insert(15, (x.h, Od, 37, Lm, want))
        torch.cuda.synchronize()
        serve_and_check(s, mix, n_threads=4)
        assert np.array_equal(alone, want)
        assert np.array_equal(Lm.cpu().numpy(), alone)
    finally:
        lbl.serve_stop(s)


def test_serve_admission_by_memory(abstractions):
    x = big = abstractions[[k for k, y in enumerate(abstractions) if y.a.grid.n == 512][0]]
    # the device bytes one 64-column request takes, as the server accounts them
    s = lbl.serve_start(hbm_budget_bytes=1 << 30, max_batch_frames=1, n_streams=1)
    try:
        Od64 = torch.from_numpy(frames_for(x, 0, 0, n_props=64)).cuda()
        Ld64 = torch.empty((x.a.n_traj, 64), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        assert lbl.serve_wait(s, lbl.serve_submit(s, x.h, Od64, 64, Ld64)) == lbl.OK
        need = lbl.serve_stats(s)["budget_high_water"]
    finally:
        lbl.serve_stop(s)
    assert need > 0
    say(f"one 64-column request on {x.a.n_traj} x {x.a.grid.n}^2 takes {need} bytes")
    # a budget that holds only a few such requests per batch still serves everything
    s = lbl.serve_start(hbm_budget_bytes=3 * need, max_batch_frames=16, n_streams=1)
    try:
        reqs = requests([x] * 1, 12, seed=4)
        serve_and_check(s, reqs, n_threads=2)
        st = lbl.serve_stats(s)
        assert st["batches"] >= 2, st
        assert st["budget_high_water"] <= 3 * need
    finally:
        lbl.serve_stop(s)
    # a request larger than a slot's share is rejected with ENOMEM
    s = lbl.serve_start(hbm_budget_bytes=1 << 20, max_batch_frames=4, n_streams=1)
    try:
        Od = torch.zeros((big.a.grid.n_cells, 64), dtype=torch.uint8, device="cuda")
        Ld = torch.zeros((big.a.n_traj, 64), dtype=torch.uint8, device="cuda")
        with pytest.raises(lbl.LblError) as e:
            lbl.serve_submit(s, big.h, Od, 64, Ld)
        assert e.value.status == lbl.ENOMEM
        assert lbl.serve_stats(s)["rejected"] == 1
        with pytest.raises(lbl.LblError):
            lbl.serve_submit(s, big.h, Od, 65, Ld)
        assert lbl.serve_wait(s, 12345) == lbl.EINVAL
    finally:
        lbl.serve_stop(s)


def test_serve_keeps_serving_after_a_failed_batch(abstractions, monkeypatch):
    monkeypatch.setenv("LBL_FAULT_BATCH", "2")
    s = lbl.serve_start(hbm_budget_bytes=64 << 20, max_batch_frames=1, n_streams=1)
    monkeypatch.delenv("LBL_FAULT_BATCH")
    try:
        reqs = requests(abstractions[:2], 4, seed=6)
        statuses = []
        for (h, Od, n_props, Ld, want) in reqs:
            t = lbl.serve_submit(s, h, Od, n_props, Ld)
            st = lbl.serve_wait(s, t)
            statuses.append(st)
            if st == lbl.OK:
                assert np.array_equal(Ld.cpu().numpy(), want)
        assert statuses == [lbl.OK, lbl.EDEVICE, lbl.OK, lbl.OK]
        st = lbl.serve_stats(s)
        assert st["failed"] == 1 and st["completed"] == 3
    finally:
        lbl.serve_stop(s)
