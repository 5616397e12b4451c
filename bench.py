"""Benchmark: g3 triplets binned per second on one MI355X.

Workload: N = 65536 Lennard-Jones-like fluid at rho = 0.85 sigma^-3, 50 frames
of jittered FCC (sd 0.15 sigma), rmax = 3.0 sigma, dr = 0.05 sigma (60 bins),
half layout, int32 coordinates at sigma/4096, uint64 counts.  One step is one
pass of the whole hot path (cell build, neighbour lists, triplet binning,
flush) over all 50 frames.

Reported: the batched form (one hipGraph launch per step) as the headline,
the plain per-frame form beside it, the triplet kernel's HIP-event duration
against the int32 VALU roofline, and the CPU oracle on a bounded sample.

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

# Algorithmic int32 operations of the method (see the design notes):
#   per candidate pair (centre, unordered {j,k} within rmax of the centre):
#     d_jk = d_ik - d_ij (3 sub), |d_jk|^2 (3 mul + 2 add), compare with R2 (1)
#   per histogram increment: exact bin of |d_jk|^2 (table + compare: 2),
#     histogram address (1), increment (1)
# In the default enumeration a candidate pair is one of the centre's
# neighbours ranked above it, and one increment stands for one triangle
# (three triplets binned, added by the expansion).
OPS_PER_CANDIDATE = 9
OPS_PER_BINNED = 4
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
    cand = plan.candidates() // max(kern_n, 1)
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
                "candidates_per_launch": cand, "increments_per_launch": increments}

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

    served = None
    if args.serve_requests > 0:
        mark(f"served: {args.serve_requests} requests at {args.serve_rate}/s, two budgets")
        served = serve_bench(args.serve_requests, args.serve_rate)

    cpu = None
    if not args.no_cpu:
        mark("cpu baseline (oracle)")
        cpu = cpu_baseline(w, args.cpu_frames)

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
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    plan.close()
    print(json.dumps(line), flush=True)


def cpu_baseline(w, n_frames: int):
    """The oracle (plain C, OpenMP over centres, untuned) on a bounded
    sample of the same workload: its first ``n_frames`` frames, all centres."""
    import oracle
    oracle.lib()
    nt = oracle.max_threads()
    n_frames = max(1, min(n_frames, w.n_frames))
    t0 = time.perf_counter()
    H = oracle.hist_full(w.frames[:n_frames], w.box, w.rmax, w.nbins, n_threads=nt)
    dt = time.perf_counter() - t0
    binned = int(H.sum()) // 2                  # unordered pairs = half-layout total
    return {"value": binned / dt / 1e9, "unit": "G triplets binned/s", "cores": nt,
            "kind": "oracle", "seconds": dt,
            "sample": f"frames 0..{n_frames - 1} of {w.n_frames}, all {w.n_atoms} centres "
                      f"({binned} triplets binned)"}


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
    latency (arrival -> histogram in host memory) at two HBM budgets."""
    from paper_1708_08619_amd import serve
    store = serve.TrajectoryStore(n_systems=16, max_frames=20, n_min=1024, n_max=65536)
    out = {"rate_hz": rate_hz, "workload": "frames U{1..20}, N log-uniform 1024..65536, "
           "rmax in {2.0, 2.5, 3.0} sigma, dr 0.05 sigma, jittered FCC rho U(0.7,0.9)"}
    for name, budget, fpi in (("budget_8GiB", 8 << 30, 2), ("budget_256MiB", 256 << 20, 2)):
        reqs = serve.poisson_requests(store, n_requests, rate_hz)
        warm = serve.poisson_requests(store, 8, 1e6, seed=(1, 2))
        srv = serve.Server(hbm_budget_bytes=budget, frames_per_iter=fpi)
        srv.run_open_loop(warm)                 # library scratch and allocator warm-up
        srv.iterations, srv.peak_used = 0, 0
        st = srv.run_open_loop(reqs)
        out[name] = {k: st[k] for k in ("requests", "p50_ms", "p99_ms", "mean_ms", "max_ms",
                                        "throughput_G_per_s", "requests_per_s", "iterations",
                                        "peak_hbm_bytes")}
        out[name]["frames_per_iter"] = fpi
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
