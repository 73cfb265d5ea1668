#!/usr/bin/env python3
"""Throughput of the labeling hot path on one MI355X.

One step labels one perception frame: the frame's cell-by-proposition map O
(uint8, already in device memory) is packed and multiplied with the
device-resident trajectory-by-cell matrix T (Boolean product, Sec. 4.2), and
the labels L (uint8, device memory) are written.  Workload: 200,000
trajectories on a 512 x 512 grid (0.2 m cells) with 64 propositions at 1%
cell density, synthetic (seeded generator; the paper's roadmap and scenario
are not available).

Prints one JSON line.  `value` is labeled (trajectory, proposition) pairs per
second over the timed steps, inputs resident in HBM.  `roofline` is for the
labeling kernel, timed with HIP events on the stream it runs on.
`cpu_baseline` is the plain CPU oracle timed on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "labeled traj-prop pairs/s & % roofline, 200k×512²×64; served p50/p99 ms"
HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=150)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--frames", type=int, default=8, help="distinct frames cycled through the steps")
    p.add_argument("--rho", type=float, default=0.01, help="O cell density of every proposition")
    p.add_argument("--kernel", default="auto", choices=["auto", "sparse", "bits", "mfma", "mfma_i8"])
    p.add_argument("--n-traj", type=int, default=200000)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=10.0)
    p.add_argument("--no-sweep", action="store_true", help="skip the kernel x density sweep")
    p.add_argument("--sweep-steps", type=int, default=10)
    p.add_argument("--no-pcie", action="store_true")
    p.add_argument("--no-raster", action="store_true", help="skip the proposition rasterizer leg")
    p.add_argument("--no-batch", action="store_true", help="skip the six-abstraction batched run")
    p.add_argument("--batch-reps", type=int, default=20)
    p.add_argument("--no-serve", action="store_true", help="skip the serving run")
    p.add_argument("--serve-seconds", type=float, default=60.0, help="seconds per arrival rate")
    p.add_argument("--serve-rates", default="200,500,1000,2000")
    p.add_argument("--serve-burst", type=int, default=4000,
                   help="requests of the closed-loop burst (every client submits as fast as it can)")
    p.add_argument("--no-configs", action="store_true", help="skip the small and medium configurations")
    p.add_argument("--no-mall", action="store_true", help="skip the headline over three resident abstractions")
    p.add_argument("--serve-budget-mib", type=int, default=2048)
    p.add_argument("--no-table1", action="store_true", help="skip the time-augmented workloads of Table 1's sizes")
    p.add_argument("--table1-sizes", default="154776,295700,568958,836276,1097702")
    p.add_argument("--table1-steps", type=int, default=20)
    p.add_argument("--table1-shuffle", action="store_true",
                   help="transitions in random row order instead of by source vertex")
    return p.parse_args()


def kernel_flag(lbl, name):
    return {"auto": lbl.KERNEL_AUTO, "bits": lbl.KERNEL_BITS, "mfma": lbl.KERNEL_MFMA,
            "mfma_i8": lbl.KERNEL_MFMA_I8, "sparse": lbl.KERNEL_SPARSE}[name]


def timed_steps(lbl, torch, h, Os, n_props, L, flags, steps, stream, profile=True):
    """Run `steps` frames; returns (wall seconds, profile totals or None).

    With profile=True the library records HIP events around each of its
    kernels (per-kernel durations); the wall time of such a run includes the
    event records, so headline throughput is taken with profile=False."""
    torch.cuda.synchronize()
    if profile:
        lbl.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(steps):
        lbl.label_frame(h, Os[k % len(Os)], n_props, L, flags=flags, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = None
    if profile:
        prof = lbl.profile_read()
        lbl.profile_enable(False)
    return t1 - t0, prof


def kernel_source_sha(name: str) -> str:
    path = os.path.join(ROOT, "paper_1810_02612_amd", "csrc", name)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def traffic_from_profile(kernel_file: str, summary: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None
    if it is missing or was taken from a different kernel source."""
    path = os.path.join(PROFILES, summary)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("kernel_src_sha") != kernel_source_sha(kernel_file):
        return None
    return d.get("hbm_bytes_per_launch")


def roofline(kernel: str, info: dict, n_traj: int, n_props: int, kernel_ms: float, issued_ops=None) -> dict:
    """Roofline of one labeling launch from its algorithmic bytes or ops.

    bits    : dense bitpacked T (8 B per 64-cell word of every row) + packed
              frame masks (W x 64 x 8 B) + L (1 B per pair)          -> HBM
    sparse  : sparse layout (10 B per (row, word) entry + the one-frame
              tiling's task and round tables) + cell masks (W x 64 x 8 B)
              + label bits (8 B per row)                              -> HBM
              (frames of at most 32 propositions: their own tiling's
              tables, 4 B cell masks and 4 B of label bits per row;
              frames of at most 4: the direct-mask kernel's entries, chunk,
              part and tile records, one bit per cell and proposition of
              frame data, and L itself, which that kernel writes)
    mfma    : the int8 multiply-adds the kernel issues (issued_ops, the
              blocks it does not skip), else the dense 2 N_t N_c N_p  -> MFMA
    mfma_i8 : int8 T (1 B per cell of every row) + masks + L           -> HBM
    """
    W = info["n_words"]
    t = kernel_ms * 1e-3
    if kernel == "mfma":
        dense = 2.0 * n_traj * W * 64 * n_props
        ops = float(issued_ops) if issued_ops is not None else dense
        return {"bound": "mfma", "achieved": ops / t / 1e12, "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                "frac": ops / t / 1e12 / INT8_PEAK_TOPS, "traffic": None, "kernel": "label_mfma",
                "kernel_ms": kernel_ms, "algorithmic_ops": ops, "dense_equivalent_ops": dense}
    if kernel == "sparse" and n_props <= 4 and info.get("sparse_frame_bytes_direct"):
        alg, src, summary = info["sparse_frame_bytes_direct"] + W * 8 * n_props + n_traj * n_props, "sparse.hip", None
    elif kernel == "sparse" and n_props <= 32 and info.get("sparse_frame_bytes_narrow"):
        alg, src, summary = info["sparse_frame_bytes_narrow"] + W * 64 * 4 + n_traj * 4, "sparse.hip", None
    elif kernel == "sparse":
        alg, src, summary = info["sparse_frame_bytes"] + W * 64 * 8 + n_traj * 8, "sparse.hip", "label_sparse_200k_512_64_traffic.json"
    elif kernel == "mfma_i8":
        alg, src, summary = n_traj * W * 64 + W * 64 * 8 + n_traj * n_props, "label_mfma.hip", None
    else:
        alg, src, summary = info["bits_bytes"] + W * 64 * 8 + n_traj * n_props, "label_bits.hip", "label_bits_200k_512_64_traffic.json"
    achieved = alg / t / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_from_profile(src, summary) if summary else None,
            "kernel": "label_" + kernel, "kernel_ms": kernel_ms, "algorithmic_bytes": alg}


def mfma_issued_ops(lbl, a, n_props: int, m_tiles: int = 2) -> int:
    """Multiply-add operations the int8 MFMA kernel issues on this T: a
    wavefront takes 16 * m_tiles rows and walks the row 8 words (512 cells) at
    a time, skipping a block whose words are zero in every one of its rows;
    each block it keeps costs m_tiles x ceil(n_props / 16) x 8 instructions of
    16 x 16 x 64 multiply-adds (2 operations each)."""
    n = a.grid.n
    W = n * n // 64
    cw = np.fromiter((lbl.cell_position(n, n, c)[0] for c in range(n * n)), np.int64, n * n)
    rows_per_wave = 16 * m_tiles
    n_blocks = (W + 7) // 8
    n_waves = (a.n_traj + rows_per_wave - 1) // rows_per_wave
    kept = np.zeros(n_waves * n_blocks, bool)
    rp = a.row_ptr.astype(np.int64)
    for r0 in range(0, a.n_traj, 16384):
        r1 = min(a.n_traj, r0 + 16384)
        cols = a.col_idx[rp[r0]:rp[r1]].astype(np.int64)
        rows = np.repeat(np.arange(r0, r1, dtype=np.int64), np.diff(rp[r0:r1 + 1]))
        kept[(rows // rows_per_wave) * n_blocks + cw[cols] // 8] = True
    nt = (n_props + 15) // 16
    return int(kept.sum()) * m_tiles * nt * 8 * 2 * 16 * 16 * 64


def bench_configs(args, lbl, torch, gen, stream):
    """The small configuration (1,000 x 64^2 x 8, cache-resident: per-frame
    latency) and the medium one (50,000 x 256^2 x 32: throughput and the label
    kernel's HBM roofline), each on the library's default path."""
    out = {}
    a = gen.make_abstraction(1)
    h = lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx)
    Oh = [gen.make_frame(1, a.grid, 8, frame=f) for f in range(8)]
    Os = [torch.from_numpy(o).cuda() for o in Oh]
    L = torch.empty((a.n_traj, 8), dtype=torch.uint8, device="cuda")
    for k in range(10):
        lbl.label_frame(h, Os[k % 8], 8, L, stream=stream)
    lat = []
    for k in range(150):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lbl.label_frame(h, Os[k % 8], 8, L, stream=stream)
        e1.record(stream)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    lat = np.array(lat)
    Lh = np.empty((a.n_traj, 8), np.uint8)
    host = []
    for k in range(150):
        t = time.perf_counter()
        lbl.label_frame(h, Oh[k % 8], 8, Lh, flags=lbl.HOST_PTRS)
        host.append(1000 * (time.perf_counter() - t))
    host = np.array(host)
    out["small"] = {"workload": "1000 trajectories x 64x64 cells x 8 propositions, O density 5-20%",
                    "frames": 150, "device_mean_ms": float(lat.mean()), "device_p50_ms": float(np.median(lat)),
                    "device_p99_ms": float(np.percentile(lat, 99)),
                    "host_ptrs_mean_ms": float(host.mean()), "host_ptrs_p50_ms": float(np.median(host)),
                    "host_ptrs_p99_ms": float(np.percentile(host, 99)),
                    "note": "device: GPU events around one frame's kernels; host_ptrs: O in and L out over PCIe, "
                            "wall time of the synchronous call"}
    lbl.free_abstraction(h)
    log("small", out["small"])

    a = gen.make_abstraction(2)
    h = lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx)
    info = lbl.abstraction_info(h)
    Os = [torch.from_numpy(gen.make_frame(2, a.grid, 32, frame=f)).cuda() for f in range(8)]
    L = torch.empty((a.n_traj, 32), dtype=torch.uint8, device="cuda")
    for k in range(10):
        lbl.label_frame(h, Os[k % 8], 32, L, stream=stream)
    steps = 150
    wall, _ = timed_steps(lbl, torch, h, Os, 32, L, 0, steps, stream, profile=False)
    _, prof = timed_steps(lbl, torch, h, Os, 32, L, 0, steps, stream, profile=True)
    label_ms = prof["label_ms"] / max(1, prof["label_launches"])
    roof = roofline("sparse", info, a.n_traj, 32, label_ms)
    roof["traffic"] = None
    out["medium"] = {"workload": "50000 trajectories x 256x256 cells x 32 propositions, O density 5-20%",
                     "steps": steps, "ms_per_step": 1000 * wall / steps,
                     "pairs_per_s": a.n_traj * 32 * steps / wall, "label_kernel_roofline": roof,
                     "t_row_density": info["set_cells"] / (a.n_traj * a.grid.n_cells)}
    lbl.free_abstraction(h)
    log("medium", out["medium"])
    return out


def bench_mall(args, lbl, torch, gen, Os, n_props, stream):
    """The headline frame over three resident 200,000 x 512^2 abstractions
    (distinct seeds) taken in turn: their sparse layouts (about 100 MB each)
    exceed the 256 MB last-level cache together, so T streams from HBM."""
    hs, infos, n_traj = [], [], None
    for k in (11, 12, 13):
        a = gen.make_abstraction(3, abstraction=k)
        hs.append(lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx, lbl.LOAD_SPARSE_ONLY))
        infos.append(lbl.abstraction_info(hs[-1]))
        n_traj = a.n_traj
        del a
    L = torch.empty((n_traj, n_props), dtype=torch.uint8, device="cuda")
    for k in range(6):
        lbl.label_frame(hs[k % 3], Os[k % len(Os)], n_props, L, stream=stream)
    steps = 150

    def run(profile):
        torch.cuda.synchronize()
        if profile:
            lbl.profile_enable(True)
        t0 = time.perf_counter()
        for k in range(steps):
            lbl.label_frame(hs[k % 3], Os[k % len(Os)], n_props, L, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = None
        if profile:
            prof = lbl.profile_read()
            lbl.profile_enable(False)
        return dt, prof

    wall, _ = run(False)
    _, prof = run(True)
    label_ms = prof["label_ms"] / max(1, prof["label_launches"])
    mean_info = {k: float(np.mean([i[k] for i in infos])) for k in ("sparse_frame_bytes", "n_words")}
    mean_info["n_words"] = int(mean_info["n_words"])
    roof = roofline("sparse", mean_info, n_traj, n_props, label_ms)
    roof["traffic"] = None
    for h in hs:
        lbl.free_abstraction(h)
    out = {"abstractions": 3, "sparse_bytes_total": int(sum(i["sparse_bytes"] for i in infos)),
           "ms_per_step": 1000 * wall / steps, "pairs_per_s": n_traj * n_props * steps / wall,
           "label_kernel_roofline": roof}
    log("mall", out)
    return out


def load_batch_abstractions(lbl, gen):
    """The six uneven abstractions (10k..200k trajectories on 128^2..512^2 grids)."""
    out = []
    for i in range(6):
        a = gen.make_batch_abstraction(i)
        h = lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx)
        out.append((a, h))
        log(f"  batch abstraction {i}: {a.n_traj} x {a.grid.n}^2")
    return out


def bench_batch(args, lbl, torch, gen, abss, stream):
    """16 frames per abstraction (4..64 propositions, density 5..30%): one
    persistent launch per batch versus one launch per frame."""
    jobs = []
    for i, (a, h) in enumerate(abss):
        for k in range(16):
            n_props = gen.batch_frame_props(4, i, k)
            O = gen.make_frame(4, a.grid, n_props, frame=k, abstraction=i, rho_lo=0.05, rho_hi=0.30)
            jobs.append((h, torch.from_numpy(O).cuda(), n_props,
                         torch.empty((a.n_traj, n_props), dtype=torch.uint8, device="cuda")))
    pairs = sum(abss[j // 16][0].n_traj * jobs[j][2] for j in range(len(jobs)))

    def per_frame(kflag):
        for (h, Od, n, Ld) in jobs:
            lbl.label_frame(h, Od, n, Ld, flags=kflag, stream=stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.batch_reps):
            for (h, Od, n, Ld) in jobs:
                lbl.label_frame(h, Od, n, Ld, flags=kflag, stream=stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / args.batch_reps

    # one frame per launch: the library's default (sparse) kernel, and the
    # plain bitpacked kernel
    single_sparse_s = per_frame(lbl.KERNEL_SPARSE)
    ref = [Ld.clone() for (_, _, _, Ld) in jobs]
    single_s = per_frame(lbl.KERNEL_BITS)
    # batched: tune the launch for this shape class, then replay the cached graph
    lbl.tune_batch(jobs, stream=stream)
    for (_, _, _, Ld) in jobs:
        Ld.fill_(5)
    lbl.label_batch(jobs, stream=stream)
    torch.cuda.synchronize()
    # the batch's labels are the one-frame path's, byte for byte
    same = sum(int(torch.equal(Ld, r)) for (_, _, _, Ld), r in zip(jobs, ref))
    tuned = lbl.tune_batch_describe(jobs, stream=stream)
    # timed without the library's profiling events (as the one-frame runs
    # are), then a second pass with them for the GPU time
    t = time.perf_counter()
    for _ in range(args.batch_reps):
        lbl.label_batch(jobs, stream=stream)
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - t) / args.batch_reps
    lbl.profile_enable(True)
    for _ in range(args.batch_reps):
        lbl.label_batch(jobs, stream=stream)
    torch.cuda.synchronize()
    prof = lbl.profile_read()
    lbl.profile_enable(False)
    t_bytes = sum(lbl.abstraction_info(h)["bits_bytes"] for _, h in abss)
    gpu_ms = prof["batch_ms"] / max(1, prof["batch_launches"])
    return {"frames": len(jobs), "abstractions": [[a.n_traj, a.grid.n] for a, _ in abss],
            "pairs_per_batch": pairs,
            "one_frame_per_launch": {"ms": 1000 * single_sparse_s, "pairs_per_s": pairs / single_sparse_s,
                                     "kernel": "sparse (the library's default)"},
            "one_frame_per_launch_bits": {"ms": 1000 * single_s, "pairs_per_s": pairs / single_s,
                                          "kernel": "bits"},
            "batched": {"ms": 1000 * batch_s, "gpu_ms": gpu_ms, "pairs_per_s": pairs / batch_s,
                        "launch": tuned},
            "speedup": single_sparse_s / batch_s,
            "speedup_vs_bits_per_frame": single_s / batch_s,
            "jobs_equal_to_one_frame_path": f"{same}/{len(jobs)}"}


def bench_serve(args, lbl, torch, gen, abss):
    """Poisson arrivals; each request one frame (8..64 propositions, density
    5..30%) against one of the six resident abstractions, chosen uniformly.
    Each rate runs for --serve-seconds with batches launched as soon as a
    stream is free (max_wait_us 0: the lowest latency at these rates).  A
    closed-loop burst follows: the client submits as fast as it can while
    up to 48 requests per abstraction are outstanding, and batches wait up to
    200 us for company, so they form (batches well below requests)."""
    import queue
    import threading

    rng = np.random.default_rng([181002612, 5])
    pool = []  # per abstraction: list of (Od, n_props)
    for i, (a, h) in enumerate(abss):
        frames = []
        for k in range(8):
            n_props = int(rng.integers(8, 65))
            O = gen.make_frame(5, a.grid, n_props, frame=k, abstraction=i, rho_lo=0.05, rho_hi=0.30)
            frames.append((torch.from_numpy(O).cuda(), n_props))
        pool.append(frames)
    ring = 48
    Lbuf = [[torch.empty(a.n_traj * 64, dtype=torch.uint8, device="cuda") for _ in range(ring)] for a, _ in abss]
    torch.cuda.synchronize()

    def run(lam, n_req, max_wait_us):
        s = lbl.serve_start(hbm_budget_bytes=args.serve_budget_mib << 20, max_batch_frames=16,
                            max_wait_us=max_wait_us, max_queue=8192, n_streams=3)
        free = [queue.Queue() for _ in abss]
        for q in free:
            for k in range(ring):
                q.put(k)
        inflight = queue.Queue()
        samples, errors = [], []
        gaps = rng.exponential(1.0 / lam, n_req) if lam else np.zeros(n_req)
        choice = rng.integers(0, len(abss), n_req)
        fpick = rng.integers(0, 8, n_req)
        sample_every = 100

        def submitter():
            t0 = time.perf_counter()
            t_next = 0.0
            for r in range(n_req):
                t_next += gaps[r]
                dt = t0 + t_next - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                i, f = int(choice[r]), int(fpick[r])
                Od, n_props = pool[i][f]
                k = free[i].get()
                Ld = Lbuf[i][k][: abss[i][0].n_traj * n_props]
                try:
                    tk = lbl.serve_submit(s, abss[i][1], Od, n_props, Ld)
                except lbl.LblError as e:
                    errors.append(str(e))
                    free[i].put(k)
                    continue
                inflight.put((tk, i, k, f, r))
            inflight.put(None)

        def waiter():
            while True:
                item = inflight.get()
                if item is None:
                    return
                tk, i, k, f, r = item
                st = lbl.serve_wait(s, tk)
                if st != lbl.OK:
                    errors.append(f"ticket {tk}: {st}")
                elif r % sample_every == 0:
                    n_props = pool[i][f][1]
                    samples.append((i, f, Lbuf[i][k][: abss[i][0].n_traj * n_props].clone()))
                free[i].put(k)

        ts = [threading.Thread(target=submitter), threading.Thread(target=waiter)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        st = lbl.serve_stats(s)
        lbl.serve_stop(s)
        # identity: each sampled request labeled alone (the library's default
        # one-frame path) gives the same bytes
        same = 0
        for i, f, Lmix in samples:
            Od, n_props = pool[i][f]
            La = torch.empty_like(Lmix)
            lbl.label_frame(abss[i][1], Od, n_props, La)
            torch.cuda.synchronize()
            same += int(torch.equal(La, Lmix))
        out = {"rate_per_s": lam if lam else "closed loop", "max_wait_us": max_wait_us,
               "submitted": st["submitted"], "completed": st["completed"], "rejected": st["rejected"],
               "failed": st["failed"], "batches": st["batches"],
               "frames_per_batch": st["completed"] / max(1, st["batches"]), "p50_ms": st["p50_ms"],
               "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"], "max_ms": st["max_ms"], "wall_s": st["wall_s"],
               "req_per_s": st["completed"] / st["wall_s"], "pairs_per_s": st["pairs_per_s"],
               "max_in_flight": st["max_in_flight"], "budget_high_water": st["budget_high_water"],
               "identity_checked": len(samples), "identity_same": same, "errors": errors[:3]}
        log("serve", out)
        return out

    results = []
    for lam in [float(x) for x in args.serve_rates.split(",") if x]:
        r = run(lam, int(lam * args.serve_seconds), 0)
        r["seconds"] = args.serve_seconds
        results.append(r)
    if args.serve_burst > 0:
        results.append(run(None, args.serve_burst, 200))
    return results


# Table 1 of the paper (GTX 1080, PCIe transfers included, one proposition
# per labeling): transitions -> (moving_vehicle ms, not_nominal_lane ms).
PAPER_TABLE1 = {154776: (3.67, 2.01), 295700: (6.60, 3.25), 568958: (12.77, 5.95), 836276: (18.46, 8.40),
                1097702: (24.40, 11.02)}


def bench_table1(args, lbl, torch, gen, stream):
    """Time-augmented workloads at Table 1's transition counts (2^21 cells,
    0.0223% occupancy, the two propositions at about 1% and 90%): each loaded
    sparse-only, labeled per frame with both propositions on the device, per
    proposition on the device, and per proposition with host O in and host L
    out (the paper's timing scope)."""
    g = gen.SpaceTimeGrid()
    frames = [gen.spacetime_frame(g, f) for f in range(4)]
    dens = np.mean([o.mean(axis=0) for o in frames], axis=0)
    O2 = [torch.from_numpy(o).cuda() for o in frames]
    O1 = [[torch.from_numpy(np.ascontiguousarray(o[:, p:p + 1])).cuda() for o in frames] for p in range(2)]
    O1h = [[np.ascontiguousarray(o[:, p:p + 1]) for o in frames] for p in range(2)]
    flags = lbl.KERNEL_SPARSE
    rows_out = []
    for n in [int(x) for x in args.table1_sizes.split(",") if x]:
        log(f"table1: {n} transitions")
        t = time.perf_counter()
        A = gen.spacetime_abstraction(n, g, shuffle_rows=args.table1_shuffle)
        t_gen = time.perf_counter() - t
        t = time.perf_counter()
        h = lbl.load_abstraction(g.nx, g.ny, A.row_ptr, A.col_idx, lbl.LOAD_SPARSE_ONLY)
        t_load = time.perf_counter() - t
        del A
        info = lbl.abstraction_info(h)
        L2 = torch.empty((n, 2), dtype=torch.uint8, device="cuda")
        L1 = torch.empty((n, 1), dtype=torch.uint8, device="cuda")
        for k in range(3):
            lbl.label_frame(h, O2[k % 4], 2, L2, flags=flags, stream=stream)
        wall2, _ = timed_steps(lbl, torch, h, O2, 2, L2, flags, args.table1_steps, stream, profile=False)
        _, prof = timed_steps(lbl, torch, h, O2, 2, L2, flags, args.table1_steps, stream, profile=True)
        label_ms = prof["label_ms"] / max(1, prof["label_launches"])
        per_prop, pcie = [], []
        for p in range(2):
            w1, _ = timed_steps(lbl, torch, h, O1[p], 1, L1, flags, args.table1_steps, stream, profile=False)
            per_prop.append(1000 * w1 / args.table1_steps)
            Lh = np.empty((n, 1), np.uint8)
            lbl.label_frame(h, O1h[p][0], 1, Lh, flags=flags | lbl.HOST_PTRS)
            reps = 10
            t = time.perf_counter()
            for k in range(reps):
                lbl.label_frame(h, O1h[p][k % 4], 1, Lh, flags=flags | lbl.HOST_PTRS)
            pcie.append(1000 * (time.perf_counter() - t) / reps)
        roof = roofline("sparse", info, n, 2, label_ms)
        lab = L2.float().mean(dim=0).tolist()
        lbl.free_abstraction(h)
        # the step after labeling: least-cost paths on the product with a
        # monitor (never off the nominal lane twice in a row), from vertex 0
        n_v, src, dst, cost = gen.spacetime_roadmap(n, g)
        dsrc, ddst, dcost = (torch.from_numpy(x.view(np.int32)).cuda() for x in (src, dst, cost))
        delta = np.array([0, 0, 1, 1, 0, 0, lbl.MONITOR_REJECT, lbl.MONITOR_REJECT], np.uint8)
        dist = torch.empty(n_v * 2, dtype=torch.int32, device="cuda")
        pred = torch.empty(n_v * 2, dtype=torch.int32, device="cuda")
        lbl.product_shortest_paths(n_v, dsrc, ddst, dcost, L2, 2, delta, 0, 0, dist, pred, stream=stream)
        t = time.perf_counter()
        sweeps = lbl.product_shortest_paths(n_v, dsrc, ddst, dcost, L2, 2, delta, 0, 0, dist, pred, stream=stream)
        plan_ms = 1000 * (time.perf_counter() - t)
        reached = int((dist != -1).sum().item())
        row = {"transitions": n, "entries": info["sparse_entries"], "set_cells": info["set_cells"],
               "occupancy": info["set_cells"] / (n * g.n_cells), "device_bytes": info["sparse_bytes"],
               "gen_s": t_gen, "load_s": t_load,
               "ms_per_frame_both_props": 1000 * wall2 / args.table1_steps,
               "pairs_per_s": 2 * n * args.table1_steps / wall2, "label_kernel_ms": label_ms,
               "label_kernel_hbm_frac": roof["frac"],
               "ms_per_prop_device": {"moving_vehicle": per_prop[0], "not_nominal_lane": per_prop[1]},
               "ms_per_prop_pcie": {"moving_vehicle": pcie[0], "not_nominal_lane": pcie[1]},
               "label_true_frac": {"moving_vehicle": lab[0], "not_nominal_lane": lab[1]},
               "plan": {"vertices": n_v, "monitor_states": 2, "ms": plan_ms, "sweeps": sweeps,
                        "product_vertices_reached": reached},
               "paper_gtx1080_ms_pcie": dict(zip(("moving_vehicle", "not_nominal_lane"), PAPER_TABLE1.get(n, (None, None))))}
        log("table1", row)
        rows_out.append(row)
    return {"grid": "128 x 128 cells of 0.5 m x 128 layers of 0.1 s (2^21 cells)",
            "prop_density": {"moving_vehicle": float(dens[0]), "not_nominal_lane": float(dens[1])},
            "load": "LBL_LOAD_SPARSE_ONLY", "kernel": "sparse",
            "row_order": "shuffled" if args.table1_shuffle else "by source vertex", "rows": rows_out,
            "note": "paper figures are context (another GPU, PCIe included), not a baseline"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                          "(the multi-GPU design shards trajectory rows and is described, not built)"}))
        sys.exit(2)
    import torch

    import gen
    from paper_1810_02612_amd import lbl

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n_props = 64
    log(f"generate T: {args.n_traj} trajectories on 512x512")
    t = time.perf_counter()
    a = gen.make_abstraction(3, n_traj=args.n_traj)
    log(f"  {time.perf_counter() - t:.1f}s, nnz {int(a.row_ptr[-1])}")
    need_i8 = args.kernel == "mfma_i8"
    h = lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx, lbl.LOAD_KEEP_INT8 if need_i8 else 0)
    info = lbl.abstraction_info(h)
    log("loaded", info)
    Os_host = [gen.make_frame(3, a.grid, n_props, frame=f, rho=args.rho) for f in range(args.frames)]
    rho_meas = float(np.mean([o.mean() for o in Os_host]))
    Os = [torch.from_numpy(o).cuda() for o in Os_host]
    L = torch.empty((a.n_traj, n_props), dtype=torch.uint8, device="cuda")
    flags = kernel_flag(lbl, args.kernel)
    if args.kernel == "auto":
        log("autotune on frame 0")
        lbl.tune(h, Os[0], n_props, int(round(100 * args.rho)), stream=stream)
    plan = lbl.tune_describe(h, n_props)
    log("plan", plan)

    for k in range(args.warmup):
        lbl.label_frame(h, Os[k % len(Os)], n_props, L, flags=flags, stream=stream)
    # headline: plain timed region, no profiling events between kernels
    wall, _ = timed_steps(lbl, torch, h, Os, n_props, L, flags, args.steps, stream, profile=False)
    # per-kernel durations: a second region of the same steps with HIP events
    _, prof = timed_steps(lbl, torch, h, Os, n_props, L, flags, args.steps, stream, profile=True)
    ms_per_step = 1000.0 * wall / args.steps
    pairs = a.n_traj * n_props
    value = pairs * args.steps / wall
    label_ms = prof["label_ms"] / max(1, prof["label_launches"])
    pack_ms = prof["pack_ms"] / max(1, prof["pack_launches"])
    emit_ms = prof["emit_ms"] / max(1, prof["emit_launches"]) if prof["emit_launches"] else 0.0
    W = info["n_words"]
    kernel = plan.split("-> ")[-1].split("(")[0] if args.kernel == "auto" else args.kernel
    roof = roofline(kernel, info, a.n_traj, n_props, label_ms,
                    issued_ops=mfma_issued_ops(lbl, a, n_props) if kernel == "mfma" else None)
    log(f"step {ms_per_step:.3f} ms, label kernel {label_ms:.4f} ms, pack {pack_ms:.4f} ms, emit {emit_ms:.4f} ms, "
        f"{roof['achieved']:.0f} {roof['unit']} ({100 * roof['frac']:.1f}%)")

    # per-frame latency over 150 frames (the paper's 150 queries per size):
    # events on the library's stream around each frame's three kernels
    lat = []
    for k in range(150):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lbl.label_frame(h, Os[k % len(Os)], n_props, L, flags=flags, stream=stream)
        e1.record(stream)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    lat = np.array(lat)
    frame_latency = {"frames": len(lat), "mean_ms": float(lat.mean()), "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)), "var_ms2": float(lat.var()),
                     "note": "one frame at a time, GPU events around its kernels (host waits between frames)"}
    log("frame latency", frame_latency)

    # the same frames issued alternately on two streams, each with its own L
    # and workspace: one frame's pack and combine overlap the other's label
    # kernel.  Reported beside the headline (one stream), not as it.
    s2 = [torch.cuda.Stream(), torch.cuda.Stream()]
    L2 = [L, torch.empty_like(L)]
    for k in range(4):
        lbl.label_frame(h, Os[k % len(Os)], n_props, L2[k % 2], flags=flags, stream=s2[k % 2])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(args.steps):
        lbl.label_frame(h, Os[k % len(Os)], n_props, L2[k % 2], flags=flags, stream=s2[k % 2])
    torch.cuda.synchronize()
    w2 = time.perf_counter() - t
    two_streams = {"streams": 2, "frames": args.steps, "ms_per_frame": 1000.0 * w2 / args.steps,
                   "pairs_per_s": pairs * args.steps / w2,
                   "note": "consecutive frames alternate between two streams (separate L and workspace); "
                           "not the headline value"}
    log("two streams", two_streams)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded generator: arcs and clothoids swept by a 4.5x2 m footprint; "
                "propositions as unions of rectangles and discs)",
        "config": {"workload": f"{a.n_traj} trajectories x 512x512 cells x {n_props} propositions, "
                               f"O density {args.rho:.0%}",
                   "n_traj": a.n_traj, "grid": 512, "cell_m": 0.2, "n_props": n_props,
                   "rho_target": args.rho, "rho_measured": rho_meas,
                   "t_row_density": info["set_cells"] / (a.n_traj * a.grid.n_cells),
                   "t_nonzero_word_frac": info["nonzero_words"] / (a.n_traj * W),
                   "plan": plan, "frames": args.frames},
        "roofline": roof,
        "stages_ms": {"pack_O": pack_ms, "label": label_ms, "emit_L": emit_ms},
        "frame_latency": frame_latency,
        "two_streams": two_streams,
    }

    if not args.no_pcie:
        # paper-comparable end-to-end: host O in, host L out (transfers included)
        n = 20
        Lh = np.empty((a.n_traj, n_props), np.uint8)
        lbl.label_frame(h, Os_host[0], n_props, Lh, flags=flags | lbl.HOST_PTRS)
        t = time.perf_counter()
        for k in range(n):
            lbl.label_frame(h, Os_host[k % len(Os_host)], n_props, Lh, flags=flags | lbl.HOST_PTRS)
        dt = (time.perf_counter() - t) / n
        out["pcie_inclusive"] = {"ms_per_frame": 1000 * dt, "pairs_per_s": pairs / dt,
                                 "note": "host O in and host L out per frame; not the headline value"}

    if not args.no_raster:
        # the frames' proposition shapes rasterized on the device (the step
        # before the labeling path), then shapes -> O -> L per frame; the
        # rasterized frames are the ones the headline labels
        shapes = []
        for f in range(args.frames):
            sh = gen.frame_shapes(3, a.grid, n_props, f, rho=args.rho)
            shapes.append(lbl.shapes_array(sh.kind, sh.prop, sh.cx, sh.cy, sh.a, sh.b))
        Or = torch.empty((a.grid.n_cells, n_props), dtype=torch.uint8, device="cuda")
        lbl.raster_frame(a.grid.n, a.grid.n, a.grid.res, shapes[0], n_props, Or, stream=stream)
        torch.cuda.synchronize()
        same = bool(torch.equal(Or, Os[0]))
        n = args.steps
        t = time.perf_counter()
        for k in range(n):
            lbl.raster_frame(a.grid.n, a.grid.n, a.grid.res, shapes[k % len(shapes)], n_props, Or, stream=stream)
        torch.cuda.synchronize()
        dt_r = (time.perf_counter() - t) / n
        t = time.perf_counter()
        for k in range(n):
            lbl.raster_frame(a.grid.n, a.grid.n, a.grid.res, shapes[k % len(shapes)], n_props, Or, stream=stream)
            lbl.label_frame(h, Or, n_props, L, flags=flags, stream=stream)
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t) / n
        o_bytes = a.grid.n_cells * n_props
        out["raster"] = {"shapes_per_frame": float(np.mean([len(x) for x in shapes])), "ms_per_frame": 1000 * dt_r,
                         "o_bytes": o_bytes, "o_written_gb_per_s": o_bytes / dt_r / 1e9,
                         "equals_headline_frames": same, "shapes_to_L_ms_per_frame": 1000 * dt_s,
                         "shapes_to_L_pairs_per_s": pairs / dt_s,
                         "note": "wall time per call, host validation and the shape upload included"}
        log("raster", out["raster"])

    if not args.no_sweep:
        sweep = []
        h8 = lbl.load_abstraction(a.grid.n, a.grid.n, a.row_ptr, a.col_idx, lbl.LOAD_KEEP_INT8)
        info8 = lbl.abstraction_info(h8)
        mfma_ops = mfma_issued_ops(lbl, a, n_props)
        for rho in (0.01, 0.10, 0.40):
            Ox = [torch.from_numpy(gen.make_frame(3, a.grid, n_props, frame=100 + f, rho=rho)).cuda()
                  for f in range(2)]
            for name in ("sparse", "bits", "mfma", "mfma_i8"):
                kf = kernel_flag(lbl, name)
                lbl.label_frame(h8, Ox[0], n_props, L, flags=kf, stream=stream)
                w, pr = timed_steps(lbl, torch, h8, Ox, n_props, L, kf, args.sweep_steps, stream)
                kms = pr["label_ms"] / max(1, pr["label_launches"])
                # MFMA: only the blocks the kernel multiplies count, not the
                # dense 2 N_t N_c N_p of the product
                r = roofline(name, info8, a.n_traj, n_props, kms, issued_ops=mfma_ops if name == "mfma" else None)
                row = {"rho": rho, "kernel": name, "kernel_ms": kms, "step_ms": 1000 * w / args.sweep_steps,
                       "label_kernel_pairs_per_s": pairs / (kms * 1e-3), "roofline_bound": r["bound"],
                       "achieved": r["achieved"], "unit": r["unit"], "frac": r["frac"]}
                if name == "mfma":
                    row["issued_ops"] = mfma_ops
                    row["dense_equivalent_ops"] = r["dense_equivalent_ops"]
                # step_ms is taken with per-kernel events on, so it includes their cost
                sweep.append(row)
                log("sweep", sweep[-1])
        lbl.free_abstraction(h8)
        out["kernel_sweep"] = sweep

    if not args.no_mall:
        out["beyond_mall"] = bench_mall(args, lbl, torch, gen, Os, n_props, stream)

    if not args.no_configs:
        out["configs"] = bench_configs(args, lbl, torch, gen, stream)

    if not (args.no_batch and args.no_serve):
        log("load the six batch abstractions")
        abss = load_batch_abstractions(lbl, gen)
        if not args.no_batch:
            out["batch"] = bench_batch(args, lbl, torch, gen, abss, stream)
            log("batch", out["batch"])
        if not args.no_serve:
            out["serve"] = bench_serve(args, lbl, torch, gen, abss)
        for _, hb in abss:
            lbl.free_abstraction(hb)

    if not args.no_table1:
        out["table1"] = bench_table1(args, lbl, torch, gen, stream)

    if not args.no_cpu:
        import oracle  # the CPU baseline leg: oracle as it stands, all host threads

        threads = min(os.cpu_count() or 1, 64)
        frames, t0 = 0, time.perf_counter()
        while True:
            oracle.label_csr(a.row_ptr, a.col_idx, a.grid.n_cells, Os_host[frames % len(Os_host)], threads=threads)
            frames += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": frames * pairs / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
                               "sample": f"{frames} full frames of the same workload ({dt:.1f} s)"}
        # the same oracle on one thread, over a bounded sample of rows
        rows = np.arange(0, a.n_traj, 8, dtype=np.uint64)
        n1, t0 = 0, time.perf_counter()
        while True:
            oracle.label_csr(a.row_ptr, a.col_idx, a.grid.n_cells, Os_host[n1 % len(Os_host)], rows=rows, threads=1)
            n1 += 1
            if time.perf_counter() - t0 >= min(3.0, args.cpu_seconds):
                break
        dt1 = time.perf_counter() - t0
        out["cpu_baseline"]["single_thread"] = {
            "value": n1 * len(rows) * n_props / dt1, "unit": "pairs/s", "cores": 1,
            "sample": f"{n1} passes over every 8th row of a frame ({dt1:.1f} s)"}

    lbl.free_abstraction(h)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
