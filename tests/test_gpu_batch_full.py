"""GPU parity of the batched and served paths at full size: the six uneven
abstractions (10k to 200k trajectories on 128^2 to 512^2 grids), 16 frames
each with 4..64 propositions, every job's whole L against the oracle.

Also the persistent bitpacked batch kernel (abstractions loaded without the
sparse layout), more than 1024 columns on one abstraction, before and after
tuning.  Every case prints what it runs first.
"""
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


def expect(a, O):
    return oracle.label_csr(a.row_ptr, a.col_idx, a.grid.n_cells, O, threads=THREADS)


def frame(a, i, k, n_props=None):
    n_props = n_props or gen.batch_frame_props(4, i, k)
    return gen.make_frame(4, a.grid, n_props, frame=k, abstraction=i, rho_lo=0.05, rho_hi=0.30)


@pytest.fixture(scope="module")
def six():
    out = []
    for i in range(6):
        a = gen.make_batch_abstraction(i)
        say(f"full batch abstraction {i}: {a.n_traj} x {a.grid.n}^2, load")
        out.append((a, lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx)))
    yield out
    for _, h in out:
        lbl.free_abstraction(h)


@pytest.fixture(scope="module")
def jobs96(six):
    """16 frames per abstraction on the device, their oracle labels."""
    jobs, wants, frames = [], [], []
    for i, (a, h) in enumerate(six):
        say(f"frames and oracle labels for abstraction {i}")
        for k in range(16):
            O = frame(a, i, k)
            n_props = O.shape[1]
            jobs.append((h, torch.from_numpy(O).cuda(),
                         n_props, torch.full((a.n_traj, n_props), 9, dtype=torch.uint8, device="cuda")))
            wants.append(expect(a, O))
            frames.append((i, k))
    return jobs, wants, frames


def check(jobs, wants, what):
    torch.cuda.synchronize()
    bad = []
    for j, ((_, _, _, Ld), want) in enumerate(zip(jobs, wants)):
        got = Ld.cpu().numpy()
        if not np.array_equal(got, want):
            bad.append(f"job {j}: {(got != want).sum()} of {got.size} labels differ")
    assert not bad, f"{what}: " + "; ".join(bad[:5])


def test_full_batch_matches_oracle_then_replays_new_frames(six, jobs96):
    jobs, wants, frames = jobs96
    say(f"full batch: {len(jobs)} jobs, {sum(six[i][0].n_traj * jobs[j][2] for j, (i, _) in enumerate(frames))} pairs")
    lbl.label_batch(jobs)
    check(jobs, wants, "full batch")
    say("full batch: replay after clearing L")
    for (_, _, _, Ld) in jobs:
        Ld.fill_(7)
    torch.cuda.synchronize()
    lbl.label_batch(jobs)
    check(jobs, wants, "full batch replay")
    say("full batch: new frame contents in the same buffers")
    new_wants = []
    for j, ((h, Od, n_props, Ld), (i, k)) in enumerate(zip(jobs, frames)):
        a = six[i][0]
        O = frame(a, i, 100 + k, n_props=n_props)
        Od.copy_(torch.from_numpy(O))
        new_wants.append(expect(a, O))
    torch.cuda.synchronize()
    lbl.label_batch(jobs)
    check(jobs, new_wants, "full batch, new frames")
    # restore the fixture's frames for the tests that follow
    for j, ((h, Od, n_props, Ld), (i, k)) in enumerate(zip(jobs, frames)):
        Od.copy_(torch.from_numpy(frame(six[i][0], i, k, n_props=n_props)))
    torch.cuda.synchronize()


def shape_key(jobs):
    return lbl.tune_batch_describe(jobs).split(" -> ")[0]


@pytest.mark.parametrize("tiling", [1, 2, 3, 4, 5])
def test_full_batch_every_launch_choice(six, jobs96, tiling, tmp_path):
    """Each tiling of the sparse layout (the one-frame tiling, 1, 2, 4 and 8
    tiles per row block), launched persistent and one workgroup per tile,
    forced through the tune cache file; every job against the oracle."""
    jobs, wants, _ = jobs96
    key = shape_key(jobs)
    for pers in (1, 0):
        path = str(tmp_path / f"tune_{tiling}_{pers}.json")
        with open(path, "w") as f:
            f.write('[\n  {"batch": "%s", "unroll": 8, "waves": 4, "rows": 128, "tiling": %d, "persistent": %d}\n]\n'
                    % (key, tiling, pers))
        lbl.tune_load(path)
        desc = lbl.tune_batch_describe(jobs)
        assert desc.startswith(key) and f"persistent={pers}" in desc and f"tiling={tiling - 1}" in desc, desc
        for (_, _, _, Ld) in jobs:
            Ld.fill_(6)
        torch.cuda.synchronize()
        say(f"full batch, {desc}")
        lbl.label_batch(jobs)
        check(jobs, wants, f"tiling {tiling} persistent {pers}")
        assert lbl.tune_batch_describe(jobs).endswith("cached")


def test_full_batch_tuned_graph_is_replayed(six, jobs96, tmp_path):
    """After lbl_tune_batch the cached graph for the jobs is the recorded
    winner's, and it labels like the oracle."""
    jobs, wants, _ = jobs96
    say("tune the full batch")
    lbl.tune_batch(jobs)
    desc = lbl.tune_batch_describe(jobs)
    say(f"tuned: {desc}")
    assert desc.endswith("cached"), desc
    path = str(tmp_path / "tuned.json")
    lbl.tune_save(path)
    text = open(path).read()
    assert '"batch": "%s"' % shape_key(jobs) in text
    for (_, _, _, Ld) in jobs:
        Ld.fill_(4)
    torch.cuda.synchronize()
    lbl.label_batch(jobs)
    check(jobs, wants, "tuned batch")
    assert lbl.tune_batch_describe(jobs) == desc


def test_full_batch_equals_one_frame_per_launch(six, jobs96):
    jobs, wants, _ = jobs96
    say("one frame per launch, sparse kernel, on the batch's jobs")
    for (h, Od, n_props, Ld) in jobs:
        Ld.fill_(3)
        lbl.label_frame(h, Od, n_props, Ld, flags=lbl.KERNEL_SPARSE)
    check(jobs, wants, "one frame per launch")


def test_full_serve_three_clients_three_streams(six, jobs96):
    """Every job of the batch submitted to the server from three client
    threads, three streams, batches of up to 16 frames formed as requests
    queue up; each result equals the oracle."""
    jobs, wants, _ = jobs96
    for (_, _, _, Ld) in jobs:
        Ld.fill_(9)
    torch.cuda.synchronize()  # L is fully written before any request is submitted
    s = lbl.serve_start(hbm_budget_bytes=4 << 30, max_batch_frames=16, max_wait_us=200, n_streams=3,
                        max_queue=1024)
    errors = []

    def client(idx):
        try:
            tickets = [(j, lbl.serve_submit(s, *jobs[j])) for j in idx]
            for j, t in tickets:
                st = lbl.serve_wait(s, t)
                if st != lbl.OK:
                    errors.append(f"job {j}: status {st}")
        except Exception as e:  # noqa: BLE001
            errors.append(repr(e))

    say("serve 96 full-size requests from 3 threads")
    order = np.random.default_rng(5).permutation(len(jobs))
    th = [threading.Thread(target=client, args=(order[c::3].tolist(),)) for c in range(3)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    st = lbl.serve_stats(s)
    lbl.serve_stop(s)
    assert not errors, errors[:5]
    assert st["completed"] == len(jobs) and st["failed"] == 0
    say(f"served in {st['batches']} batches, at most {st['max_in_flight']} requests in flight")
    check(jobs, wants, "served")


@pytest.fixture(scope="module")
def bits_only():
    """Two of the six abstractions loaded without the sparse layout."""
    out = []
    for i in range(6):
        n_traj, side, _ = gen.batch_layout()[i]
        if side == 512:
            continue
        a = gen.make_batch_abstraction(i)
        say(f"bitpacked-only load of abstraction {i}: {a.n_traj} x {a.grid.n}^2")
        out.append((i, a, lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx, lbl.LOAD_NO_SPARSE)))
        if len(out) == 2:
            break
    yield out
    for _, _, h in out:
        lbl.free_abstraction(h)


def test_persistent_bitpacked_batch(bits_only):
    """The persistent kernel over (abstraction, row range) items: 18 frames of
    64 propositions on one abstraction (1152 columns: two passes, 16 and 2
    lane groups) and ragged proposition counts on the other, before and after
    lbl_tune_batch."""
    (i0, a0, h0), (i1, a1, h1) = bits_only
    jobs, wants = [], []
    for k in range(18):
        O = frame(a0, i0, 200 + k, n_props=64)
        jobs.append((h0, torch.from_numpy(O).cuda(), 64, torch.full((a0.n_traj, 64), 9, dtype=torch.uint8,
                                                                     device="cuda")))
        wants.append(expect(a0, O))
    for k, n_props in enumerate((1, 7, 33, 64, 5)):
        O = frame(a1, i1, 300 + k, n_props=n_props)
        jobs.append((h1, torch.from_numpy(O).cuda(), n_props,
                     torch.full((a1.n_traj, n_props), 9, dtype=torch.uint8, device="cuda")))
        wants.append(expect(a1, O))
    say(f"persistent bitpacked batch: {len(jobs)} jobs")
    lbl.label_batch(jobs)
    check(jobs, wants, "bitpacked batch")
    say("tune the bitpacked batch, then replay")
    lbl.tune_batch(jobs)
    for (_, _, _, Ld) in jobs:
        Ld.fill_(5)
    torch.cuda.synchronize()
    lbl.label_batch(jobs)
    check(jobs, wants, "bitpacked batch, tuned")
