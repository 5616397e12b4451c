"""Benchmark: g3 triplets binned per second on one MI355X.

Workload: N = 65536 Lennard-Jones-like fluid at rho = 0.85 sigma^-3, 50 frames
of jittered FCC (sd 0.15 sigma), rmax = 3.0 sigma, dr = 0.05 sigma (60 bins),
half layout, int32 coordinates at sigma/4096, uint64 counts.  One step is one
pass of the whole hot path (cell build, neighbour lists, triplet binning,
flush) over all 50 frames.

Reported: the batched form (one hipGraph launch per step) as the headline,
the plain per-frame form beside it, the triplet kernel's and the neighbour
build's HIP-event durations against the int32 VALU roofline (and the triplet
kernel against the measured LDS ceilings), the uneven-systems batch, the
served form (open-loop latency, and closed-loop throughput against plain
per-request launches), and the CPU oracle on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-plain]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic int32 operations of the method (see the design notes), per
# candidate pair (centre, unordered {j,k} within rmax of the centre):
#   d_jk = d_ik - d_ij (3 sub), |d_jk|^2 (3 mul + 2 add), compare with R2 (1),
#   exact bin of |d_jk|^2 (table + step: 2), histogram address (1) and the
#   accept decision for the increment (1): 13, within the 12-15 a candidate
#   costs when every candidate is binned and accepted ones are kept.  The
#   histogram increments themselves are LDS operations, priced by the LDS
#   ceiling.  In the default enumeration a candidate pair is one of the
#   centre's neighbours ranked above it, and one increment stands for one
#   triangle (three triplets binned, added by the expansion).
OPS_PER_CANDIDATE = 13
OPS_PER_BINNED = 0
# Neighbour build: per (centre, stencil atom) pair tested, the same 9 (3 sub,
# 3 mul, 2 add, 1 compare); per neighbour written: its bin (table + compare:
# 2), its r12 slab (1) and its list position (1)
BUILD_OPS_PER_CANDIDATE = 9
BUILD_OPS_PER_NEIGHBOUR = 4
# int32 VALU peak of MI355X: 256 CUs x 64 lanes/clk x 2.4 GHz
INT32_VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the library defaults instead of the autotuned configuration")
    ap.add_argument("--tuning", default="",
                    help="fixed tuning, e.g. centres_per_item=1024,lds_hist_bins=25536 (no autotuner run)")
    ap.add_argument("--no-per-centre", action="store_true",
                    help="skip timing the per-centre enumeration beside the default")
    ap.add_argument("--cpu-frames", type=int, default=8,
                    help="frames of the workload the CPU oracle processes (all centres)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests in the served (continuous batching) run; 0 skips it")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--no-paper-shapes", action="store_true",
                    help="skip the replay of the paper's g3 runs (Table 2 shapes)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (HBM counter calibration)")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-systems batch")
    ap.add_argument("--no-lds", action="store_true", help="skip the LDS rate probe")
    ap.add_argument("--saturated-requests", type=int, default=300,
                    help="requests of the closed-loop served run (0 skips it)")
    ap.add_argument("--cpu1-centres", type=int, default=4096,
                    help="centres of one frame the single-thread oracle run takes")
    return ap.parse_args()


def mark(msg: str):
    """Progress marker on stderr, flushed before the GPU work it names."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(frames would shard across GPUs with one uint64 all-reduce of the "
              "histogram; see the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1708_08619_amd import g3, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = synth.lj_large(n_frames=args.frames)
    frames = torch.from_numpy(w.frames).to(dev)
    hist = g3.new_hist(w.nbins, w.layout, dev)
    system = dict(frames=frames, box=w.box, rmax=w.rmax, nbins=w.nbins, layout=w.layout,
                  hist=hist)
    plan = g3.Plan()
    if args.calib_copy_mib:
        src = torch.empty(args.calib_copy_mib << 18, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the autotuner picks the triplet kernel's tiling for this workload (on
    # scratch histograms, outside the timed region) and the plan keeps it
    if args.tuning:
        plan.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(","))})
    elif not args.no_autotune:
        mark("autotune")
        plan.autotune([system])
    tuning = plan.get_tuning()

    # triplets binned per step = total of the half histogram of one pass
    mark(f"first batched pass: N={w.n_atoms} frames={w.n_frames}")
    plan.accumulate_batch([system])
    plan.sync()
    binned = int(hist.sum().item())
    hist.zero_()

    def timed(step_fn, steps, warmup):
        for _ in range(warmup):
            step_fn()
        plan.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step_fn()
        plan.sync()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    mark(f"batched: {args.warmup} warm-up + {args.steps} timed steps (graph replays)")
    batched_s = timed(lambda: plan.accumulate_batch([system]), args.steps, args.warmup)
    mark("batched: triplet-kernel timing (direct launches)")

    # triplet-kernel duration: HIP events around the kernel on the plan's stream
    # (direct launches of the same kernels with the same arguments)
    plan.kernel_time_reset(True)
    timed(lambda: plan.accumulate_batch([system]), max(3, args.steps // 2), 0)
    kern_ms, kern_n = plan.kernel_time()
    build_ms, build_n = plan.stage_time(g3.STAGE_NEIGHBOURS)
    cells_ms, _ = plan.stage_time(g3.STAGE_CELLS)
    cand = plan.candidates() // max(kern_n, 1)
    b_cand, b_nbrs = plan.build_counts()
    b_cand //= max(build_n, 1)
    b_nbrs //= max(build_n, 1)
    plan.kernel_time_reset(False)

    plain = None
    if not args.no_plain:
        mark("plain per-frame form")
        plain_s = timed(lambda: plan.accumulate(frames, w.box, w.rmax, w.nbins, w.layout, hist),
                        max(2, args.steps // 2), 1)
        plan.kernel_time_reset(True)
        timed(lambda: plan.accumulate(frames, w.box, w.rmax, w.nbins, w.layout, hist), 1, 0)
        pk_ms, pk_n = plan.kernel_time()
        plan.kernel_time_reset(False)
        plain = {"value": binned / plain_s / 1e9, "ms_per_step": plain_s * 1e3,
                 "triplet_kernel_ms_per_frame": pk_ms}

    tri_once = plan.get_tuning()["per_centre"] != 1
    increments = binned // 3 if tri_once else binned
    ops = OPS_PER_CANDIDATE * cand + OPS_PER_BINNED * increments
    achieved = ops / (kern_ms * 1e-3) / 1e12 if kern_ms > 0 else None
    roofline = {"bound": "alu", "achieved": achieved, "peak": INT32_VALU_PEAK_TOPS,
                "unit": "Tops/s (int32)", "frac": achieved / INT32_VALU_PEAK_TOPS if achieved else None,
                "traffic": traffic_per_launch(), "traffic_unit": "bytes per launch",
                "kernel": "k_triplet", "kernel_ms": kern_ms,
                "candidates_per_launch": cand, "increments_per_launch": increments,
                "ops_per_candidate": OPS_PER_CANDIDATE, "ops_per_increment": OPS_PER_BINNED}
    if not args.no_lds:
        mark("LDS rate probe")
        roofline["lds"] = lds_ceiling(g3, cand, increments, kern_ms, tuning["lds_hist_bins"])
        roofline["valu_ceiling_ms"] = ops / (INT32_VALU_PEAK_TOPS * 1e12) * 1e3
        lds_ms = roofline["lds"]["ceiling_ms"]
        roofline["binding"] = "lds" if lds_ms > roofline["valu_ceiling_ms"] else "valu"
        roofline["frac_of_binding"] = max(lds_ms, roofline["valu_ceiling_ms"]) / kern_ms
    b_ops = BUILD_OPS_PER_CANDIDATE * b_cand + BUILD_OPS_PER_NEIGHBOUR * b_nbrs
    b_ach = b_ops / (build_ms * 1e-3) / 1e12 if build_ms > 0 else None
    roofline_build = {"bound": "alu", "achieved": b_ach, "peak": INT32_VALU_PEAK_TOPS,
                      "unit": "Tops/s (int32)", "frac": b_ach / INT32_VALU_PEAK_TOPS if b_ach else None,
                      "kernel": "neighbour build (k_nbr_wave + k_nbr_build over its overflow cells)",
                      "kernel_ms": build_ms, "candidates_per_launch": b_cand,
                      "neighbours_per_launch": b_nbrs,
                      "ops_per_candidate": BUILD_OPS_PER_CANDIDATE,
                      "ops_per_neighbour": BUILD_OPS_PER_NEIGHBOUR, "cell_build_ms": cells_ms}

    # the paper's enumeration (every centre's unordered pairs) for comparison
    per_centre = None
    if not args.no_per_centre:
        mark("per-centre enumeration, batched")
        plan.set_tuning(**dict(tuning, per_centre=1))
        pc_s = timed(lambda: plan.accumulate_batch([system]), max(3, args.steps // 2), 1)
        plan.kernel_time_reset(True)
        c0 = plan.candidates()
        timed(lambda: plan.accumulate_batch([system]), 2, 0)
        pc_ms, pc_n = plan.kernel_time()
        pc_cand = (plan.candidates() - c0) // max(pc_n, 1)
        plan.kernel_time_reset(False)
        plan.set_tuning(**tuning)
        per_centre = {"value": binned / pc_s / 1e9, "ms_per_step": pc_s * 1e3,
                      "triplet_kernel_ms": pc_ms, "candidates_per_launch": pc_cand}

    paper_shapes = None
    if not args.no_paper_shapes:
        mark("paper-shape replay: water N = 6720, 13440, 26880, 10 frames, rmax = L/4")
        paper_shapes = paper_shape_replay(torch, dev)

    uneven = None
    if not args.no_uneven:
        mark("uneven-systems batch: 8 systems, N log-uniform 512..32768, 8 frames each")
        uneven = uneven_bench(torch, dev, args.steps)

    served = None
    if args.serve_requests > 0:
        mark(f"served: {args.serve_requests} requests at {args.serve_rate}/s, two budgets")
        served = serve_bench(args.serve_requests, args.serve_rate)
    if args.saturated_requests > 0:
        mark(f"served, closed loop: {args.saturated_requests} requests against plain launches")
        served = served or {}
        served["saturated"] = saturated_bench(torch, dev, args.saturated_requests)

    cpu = None
    if not args.no_cpu:
        mark("cpu baseline (oracle)")
        cpu = cpu_baseline(w, args.cpu_frames, args.cpu1_centres)

    line = {
        "metric": "G triplets binned/s at N=65536 (plain vs batched); p50/p99 served latency",
        "value": binned / batched_s / 1e9,
        "unit": "G triplets binned/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": batched_s * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": "lj65536_jittered_fcc", "n_atoms": w.n_atoms,
                   "n_frames": w.n_frames, "rho_sigma3": 0.85, "jitter_sigma": 0.15,
                   "rmax_sigma": 3.0, "nbins": w.nbins, "layout": "half",
                   "form": "batched (one hipGraph launch per step)",
                   "enumeration": "triangle-once" if tri_once else "per-centre"},
        "triplets_binned_per_step": binned,
        "tuning": tuning,
        "plain": plain,
        "per_centre_enumeration": per_centre,
        "served": served,
        "paper_shapes": paper_shapes,
        "uneven_batch": uneven,
        "roofline": roofline,
        "roofline_neighbour_build": roofline_build,
        "cpu_baseline": cpu,
    }
    plan.close()
    print(json.dumps(line), flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, n_frames: int, centres_1t: int):
    """The oracle (plain C, OpenMP over centres, untuned) on bounded samples
    of the same workload: its first ``n_frames`` frames with every centre on
    all host threads, and the first ``centres_1t`` centres of frame 0 on one
    thread.  Triplets binned of a centre sample = its unordered pairs."""
    import oracle
    oracle.lib()
    nt = oracle.max_threads()
    n_frames = max(1, min(n_frames, w.n_frames))
    t0 = time.perf_counter()
    H = oracle.hist_full(w.frames[:n_frames], w.box, w.rmax, w.nbins, n_threads=nt)
    dt = time.perf_counter() - t0
    binned = int(H.sum()) // 2                  # unordered pairs = half-layout total
    c1 = max(1, min(centres_1t, w.n_atoms))
    t0 = time.perf_counter()
    H1 = oracle.hist_full(w.frames[:1], w.box, w.rmax, w.nbins, n_threads=1,
                          centres=np.arange(c1, dtype=np.int32))
    dt1 = time.perf_counter() - t0
    binned1 = int(H1.sum()) // 2
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"value": binned / dt / 1e9, "unit": "G triplets binned/s", "cores": nt,
            "kind": "oracle", "seconds": dt, "cpu_model": cpu_model(), "cpus_available": avail,
            "sample": f"frames 0..{n_frames - 1} of {w.n_frames}, all {w.n_atoms} centres "
                      f"({binned} triplets binned), {nt} threads",
            "single_thread": {"value": binned1 / dt1 / 1e9, "unit": "G triplets binned/s",
                              "cores": 1, "seconds": dt1,
                              "sample": f"frame 0, centres 0..{c1 - 1} ({binned1} triplets binned)"}}


def lds_ceiling(g3, candidates: int, increments: int, kern_ms: float, slab_words: int):
    """LDS time the triplet kernel cannot go below: per candidate one random
    bin-table read (the step table, 2048 words) and one increment -- at a
    random slab word if the candidate is accepted, at the lane's own trash
    word if not -- priced at the measured rates of each pattern."""
    table_words = 2048
    r = {"add_lane": g3.lds_rate(g3.LDS_ADD_LANE, 16 * 64),
         "add_random": g3.lds_rate(g3.LDS_ADD_RANDOM, slab_words),
         "read_random": g3.lds_rate(g3.LDS_READ_RANDOM, table_words),
         "read_add_random": g3.lds_rate(g3.LDS_READ_ADD, slab_words)}
    rejected = max(candidates - increments, 0)
    t = candidates / r["read_random"] + increments / r["add_random"] + rejected / r["add_lane"]
    return {"rates_lane_ops_per_s": r, "slab_words": slab_words, "table_words": table_words,
            "ceiling_ms": t * 1e3, "frac": t * 1e3 / kern_ms if kern_ms > 0 else None,
            "model": "candidates/read_random + increments/add_random + rejected/add_lane"}


def uneven_bench(torch, dev, steps: int):
    """The batched-systems workload: 8 systems (N log-uniform 512..32768,
    densities 0.7-0.9, jittered FCC, 8 frames each, rmax 2.5 sigma, 50 bins,
    full layout) in one batched call (graph replays) against the plain form
    (per system, per-frame launches), frames resident in HBM."""
    from paper_1708_08619_amd import g3, synth
    ws = synth.uneven_batch()
    systems = [dict(frames=torch.from_numpy(w.frames).to(dev), box=w.box, rmax=w.rmax,
                    nbins=w.nbins, layout=w.layout, hist=g3.new_hist(w.nbins, w.layout, dev))
               for w in ws]
    with g3.Plan() as plan:
        plan.autotune(systems)
        plan.accumulate_batch(systems)
        plan.sync()
        binned = sum(int(s["hist"].sum().item()) // 2 for s in systems)   # full layout: ordered

        def run(fn, reps):
            fn()
            plan.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            plan.sync()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps

        reps = max(5, steps)
        tb = run(lambda: plan.accumulate_batch(systems), reps)

        def plain():
            for s in systems:
                plan.accumulate(s["frames"], s["box"], s["rmax"], s["nbins"], s["layout"], s["hist"])
        tp = run(plain, max(3, reps // 2))
        tuning = plan.get_tuning()
    return {"systems": [int(w.n_atoms) for w in ws], "frames_per_system": 8,
            "triplets_binned": binned, "batched": {"value": binned / tb / 1e9, "ms": tb * 1e3},
            "plain": {"value": binned / tp / 1e9, "ms": tp * 1e3}, "unit": "G triplets binned/s",
            "tuning": tuning}


def saturated_bench(torch, dev, n_requests: int):
    """Served throughput with the server saturated (every request arrives at
    t = 0) against plain per-request launches (g3_accumulate per request, one
    after another on one stream), on the same requests; both copy each
    request's frames from its (pageable) host memory and return its histogram
    to pinned host memory."""
    from paper_1708_08619_amd import g3, serve
    store = serve.TrajectoryStore(n_systems=16, max_frames=20, n_min=1024, n_max=65536)
    reqs0 = serve.poisson_requests(store, n_requests, 1e9)
    out = {"requests": n_requests, "workload": "frames U{1..20}, N log-uniform 1024..65536, "
           "rmax in {2.0, 2.5, 3.0} sigma, dr 0.05 sigma, jittered FCC rho U(0.7,0.9), all at t=0"}
    binned = None
    for fpi in (4, 8):
        reqs = serve.poisson_requests(store, n_requests, 1e9)
        for r in reqs:
            r.arrival = 0.0
        srv = serve.Server(hbm_budget_bytes=16 << 30, frames_per_iter=fpi, max_in_flight=3)
        srv.run_open_loop(serve.poisson_requests(store, 8, 1e9, seed=(1, 2)))   # warm-up
        srv.iterations, srv.peak_used, srv.syncs = 0, 0, 0
        st = srv.run_open_loop(reqs, sample_device=True)
        binned = st["triplets_binned"]
        out[f"served_fpi{fpi}"] = {k: st[k] for k in ("throughput_G_per_s", "requests_per_s", "p50_ms",
                                                      "p99_ms", "iterations", "syncs",
                                                      "device_peak_bytes", "peak_hbm_bytes")}
        del srv
    # plain: per request H2D, g3_accumulate (per-frame launches), D2H
    with g3.Plan() as plan:
        def plain_all():
            res = []
            for r in reqs0:
                fr = torch.from_numpy(np.ascontiguousarray(r.frames)).to(dev, non_blocking=True)
                h = g3.new_hist(r.nbins, r.layout, dev)
                plan.accumulate(fr, r.box, r.rmax, r.nbins, r.layout, h)
                host = torch.empty(h.shape, dtype=h.dtype, pin_memory=True)
                host.copy_(h, non_blocking=True)
                res.append(host)
            plan.sync()
            torch.cuda.synchronize()
            return res
        plain_all()                              # warm-up (scratch, allocator)
        t0 = time.perf_counter()
        res = plain_all()
        tp = time.perf_counter() - t0
        pb = sum(int(h.sum().item()) // (2 if r.layout == g3.FULL else 1) for h, r in zip(res, reqs0))
    out["plain_per_request"] = {"throughput_G_per_s": pb / tp / 1e9, "seconds": tp,
                                "triplets_binned": pb}
    # the same requests as one batched call, frames already on the device:
    # what the GPU sustains on this mix without the server's host work
    systems = [dict(frames=torch.from_numpy(np.ascontiguousarray(r.frames)).to(dev), box=r.box,
                    rmax=r.rmax, nbins=r.nbins, layout=r.layout, hist=g3.new_hist(r.nbins, r.layout, dev))
               for r in reqs0]
    with g3.Plan() as plan:
        plan.accumulate_batch(systems)            # warm-up (scratch)
        plan.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.accumulate_batch(systems)
        plan.sync()
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
    out["one_batch_resident"] = {"throughput_G_per_s": pb / tb / 1e9, "seconds": tb}
    del systems
    out["served_triplets_binned"] = binned
    return out


# The paper's Table 2 (g3, 10 frames, times in seconds including file reading):
# serial CPU, GTX 780 and K40 runs of its per-frame CUDA code.
PAPER_TABLE2_S = {6720: (596, 13, 16), 13440: (2089, 104, 132), 26880: (11515, 860, 1124)}


def paper_shape_replay(torch, dev):
    """The paper's g3 runs at their shapes: water-density systems of 6720,
    13440 and 26880 sites, 10 frames, two sides below L/4 and the third below
    L/2 (80 x 80 x 160 bins, full layout), batched form, frames resident in
    HBM.  The paper's times are quoted for context only: other hardware, its
    own trajectories, and its times include reading the files."""
    from paper_1708_08619_amd import g3, synth
    out = []
    for N in synth.PAPER_SHAPES:
        w = synth.water_replay(N, n_frames=10)
        nc = w.meta["nbins_third"]
        frames = torch.from_numpy(w.frames).to(dev)
        hist = g3.new_hist(w.nbins, w.layout, dev, nbins_third=nc)
        system = dict(frames=frames, box=w.box, rmax=w.rmax, nbins=w.nbins, layout=w.layout,
                      hist=hist, nbins_third=nc)
        with g3.Plan() as plan:
            plan.accumulate_batch([system])
            plan.sync()
            binned = int(hist.sum().item()) // 2      # unordered pairs, as the headline counts
            reps = 3
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                plan.accumulate_batch([system])
            plan.sync()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
        cpu_s, gtx_s, k40_s = PAPER_TABLE2_S[N]
        out.append({"n_atoms": N, "frames": 10, "box_units": w.box[0], "unit": "2^-13 nm",
                    "bins": [w.nbins, w.nbins, nc], "seconds": dt,
                    "triplets_binned": binned, "G_triplets_binned_per_s": binned / dt / 1e9,
                    "paper_cpu_s": cpu_s, "paper_gtx780_s": gtx_s, "paper_k40_s": k40_s,
                    "ratio_vs_paper_gtx780": gtx_s / dt})
        del frames, hist
    return out


def serve_bench(n_requests: int, rate_hz: float):
    """Open-loop Poisson request stream served by continuous batching; p50/p99
    latency (arrival -> histogram in host memory) at two HBM budgets.  The
    budget holds the requests' frames, histograms and neighbour-pool shares
    plus a reserve for the plan's own scratch (partial slots capped to fit
    it, tables, flag log); the device memory actually in use above the
    start is measured after every iteration."""
    from paper_1708_08619_amd import serve
    store = serve.TrajectoryStore(n_systems=16, max_frames=20, n_min=1024, n_max=65536)
    out = {"rate_hz": rate_hz, "workload": "frames U{1..20}, N log-uniform 1024..65536, "
           "rmax in {2.0, 2.5, 3.0} sigma, dr 0.05 sigma, jittered FCC rho U(0.7,0.9)"}
    for name, budget, fpi in (("budget_8GiB", 8 << 30, 2), ("budget_256MiB", 256 << 20, 2)):
        reqs = serve.poisson_requests(store, n_requests, rate_hz)
        warm = serve.poisson_requests(store, 8, 1e6, seed=(1, 2))
        reserve = min(48 << 20, budget // 4)
        srv = serve.Server(hbm_budget_bytes=budget, frames_per_iter=fpi, plan_reserve_bytes=reserve)
        # partial slots: at most 2/3 of the reserve (the rest: tables, flags)
        slot_bytes = 4 * srv.ex.plan.get_tuning()["lds_hist_bins"]
        srv.ex.plan.set_tuning(slot_limit=max(64, (reserve * 2 // 3) // slot_bytes))
        srv.run_open_loop(warm)                 # library scratch and allocator warm-up
        srv.iterations, srv.peak_used, srv.syncs = 0, 0, 0
        st = srv.run_open_loop(reqs, sample_device=True)
        out[name] = {k: st[k] for k in ("requests", "p50_ms", "p99_ms", "mean_ms", "max_ms",
                                        "throughput_G_per_s", "requests_per_s", "iterations",
                                        "peak_hbm_bytes", "device_peak_bytes", "syncs")}
        out[name]["frames_per_iter"] = fpi
        out[name]["plan_reserve_bytes"] = reserve
        del srv
    return out


def traffic_per_launch():
    """HBM bytes per triplet-kernel launch from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary, or None if the kernel source changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_triplet_lj65536_batched_traffic.json")
    src = os.path.join(ROOT, "paper_1708_08619_amd", "csrc", "g3_kernels.hip")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    return rec["bytes_per_launch"] if rec.get("kernel_source_sha256") == h else None


if __name__ == "__main__":
    main()
