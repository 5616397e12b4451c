"""Serving loop for g3 analyses: continuous batching under an HBM budget.

Requests (one system's frames plus rmax, nbins and layout) arrive while
others are on the GPU.  The scheduler works in iterations: every iteration is
one batched accumulate (``g3_accumulate_batch``) over the next
``frames_per_iter`` frames of every active request, so a request that arrives
while the GPU is busy joins the next iteration and leaves as soon as its own
frames are done (iteration-level continuous batching).  Admission is
first-come first-served while the request's device footprint -- its frames,
its histogram and its share of the neighbour pool -- fits the HBM budget; a
request that does not fit waits until finished requests free their memory.
A request's frames and histogram stay resident on the device from admission
to completion; completion is the moment its histogram is visible in host
memory, and latency runs from its arrival to that moment.  Completion is
seen per request, without draining the stream: the histogram is copied to the
host behind the batch that finished it, and the batch's completion ticket
(``g3_ticket_query``) says whether that copy is final; only a request one of
whose frames the library must recompute (``g3_sync``) waits for the device.

The scheduler talks to an executor: :class:`GpuExecutor` drives libg3
through ``g3.Plan`` (all arithmetic runs in the HIP library); tests substitute
a CPU executor to check the scheduling logic.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass

import numpy as np

from . import g3


@dataclass
class Request:
    """One g3 analysis: host int32 frames [F, 3, N] and its parameters."""
    rid: int
    frames: np.ndarray
    box: list
    rmax: float
    nbins: int
    layout: int = g3.HALF
    arrival: float = 0.0            # seconds on the server's clock
    # filled by the server
    admitted: float = math.nan
    done: float = math.nan
    result: np.ndarray | None = None
    status: int = g3.OK
    dev_frames: object = None
    dev_hist: object = None
    next_frame: int = 0
    nbytes: int = 0
    ticket: int = 0
    fetch: object = None
    fetch_ev: object = None

    @property
    def n_frames(self) -> int:
        return int(self.frames.shape[0])

    @property
    def n_atoms(self) -> int:
        return int(self.frames.shape[2])

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def footprint_bytes(req: Request, frames_per_iter: int) -> int:
    """Device bytes a request holds while active: frames, histogram, and the
    neighbour-pool share of one iteration (uniform-density estimate with the
    library's headroom) plus per-frame cell scratch."""
    F, N = req.n_frames, req.n_atoms
    V = float(req.box[0]) * req.box[1] * req.box[2]
    nexp = N / V * 4.0 / 3.0 * math.pi * req.rmax ** 3
    entry = 16 if math.ceil(req.rmax) > 32767 else 8
    k = min(F, frames_per_iter)
    pool = k * N * (1.35 * min(nexp, N) + 16) * entry
    scratch = k * N * 48
    return int(F * 3 * N * 4 + g3.hist_len(req.nbins, req.layout) * 8 + pool + scratch)


class ResultBlocks:
    """Finished histograms are handed out as slices of 16 MiB host blocks
    rather than as arrays of their own.  A new array's pages are touched for
    the first time by the copy (about 0.7 us per 4 KiB page fault); a block
    this large is backed by transparent huge pages where the kernel allows
    them on request, so 300 histograms of 0.9 MB took 61 us each instead of
    166.  A block is freed once no slice of it is referenced (a caller that
    keeps one result keeps at most its block); histograms larger than a
    block get an array of their own."""

    BLOCK_BYTES = 16 << 20

    def __init__(self):
        self._buf = None
        self._off = 0          # in 8-byte words

    def take(self, n: int) -> np.ndarray:
        words = self.BLOCK_BYTES // 8
        if n > words:
            return np.empty(n, dtype=np.uint64)
        if self._buf is None or self._off + n > words:
            self._buf = np.empty(words, dtype=np.uint64)
            self._off = 0
        out = self._buf[self._off:self._off + n]
        self._off += (n + 7) // 8 * 8        # slices start 64-byte steps into the block
        return out


class GpuExecutor:
    """Device side of the server: torch buffers on one HIP stream and a
    libg3 plan on that stream."""

    def __init__(self, device=None):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda:0")
        torch.cuda.set_device(self.device)
        self.plan = g3.Plan()
        self._host = {}
        self._pinned = {}                    # free pinned histogram buffers by length,
                                             # kept for reuse while the executor lives
        self._results = ResultBlocks()

    def upload(self, frames: np.ndarray):
        # Straight from pageable host memory (the runtime stages the copy):
        # pinning every request's frames cost more than the copy itself
        # whenever the pinned-memory cache was cold, as in a burst of new
        # requests.
        t = self.torch
        host = t.from_numpy(np.ascontiguousarray(frames, dtype=np.int32))
        dev = host.to(self.device, non_blocking=True)
        self._host[id(dev)] = host           # the source stays alive until released
        return dev

    def new_hist(self, n: int):
        t = self.torch
        return t.zeros(n, dtype=t.uint64, device=self.device)

    def accumulate_batch(self, systems: list[dict]) -> int:
        """Queue one batched call; returns its completion ticket."""
        self.plan.accumulate_batch(systems)
        return self.plan.last_ticket()

    def ticket_final(self, ticket: int):
        """None while the call runs, then whether its histograms are final."""
        return self.plan.ticket_query(ticket)

    def start_fetch(self, hist):
        t = self.torch
        free = self._pinned.get(int(hist.numel()))
        host = free.pop() if free else t.empty(hist.shape, dtype=t.uint64, pin_memory=True)
        host.copy_(hist, non_blocking=True)
        return host

    def finish_fetch(self, token) -> np.ndarray:
        out = self._results.take(int(token.numel()))
        np.copyto(out, token.numpy())
        # the copy has landed (the caller waited for its event): reuse the buffer
        self._pinned.setdefault(int(token.numel()), []).append(token)
        return out

    def release(self, frames, hist):
        self._host.pop(id(frames), None)

    def sync(self) -> int:
        return self.plan.sync_status()

    def record(self):
        ev = self.torch.cuda.Event()
        ev.record()
        return ev

    def device_used(self) -> int:
        """Device memory in use on the whole device (bytes), measured."""
        free, total = self.torch.cuda.mem_get_info(self.device)
        return int(total - free)


class Server:
    """Iteration-level continuous batching."""

    def __init__(self, hbm_budget_bytes: int = 8 << 30, frames_per_iter: int = 4,
                 max_in_flight: int = 2, executor=None, plan_reserve_bytes: int = 0):
        self.ex = executor if executor is not None else GpuExecutor()
        self.budget = int(hbm_budget_bytes)
        # device memory the plan keeps besides the requests' shares (partial
        # slots, tables, flag log), held back from the budget
        self.reserve = int(plan_reserve_bytes)
        self.frames_per_iter = int(frames_per_iter)
        self.max_in_flight = int(max_in_flight)
        self.queue: collections.deque[Request] = collections.deque()
        self.active: list[Request] = []
        self.in_flight: collections.deque = collections.deque()
        self.finishing: collections.deque[Request] = collections.deque()
        self.used = 0
        self.peak_used = 0
        self.iterations = 0
        self.syncs = 0
        self.completed: list[Request] = []
        self._next_rid = 0
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -- admission -----------------------------------------------------------
    def submit(self, req: Request):
        fr = req.frames
        if fr.ndim != 3 or fr.shape[1] != 3:
            raise ValueError("frames must be [F, 3, N]")
        st = g3.check_args(req.n_atoms, req.box, req.rmax, req.nbins, req.layout)
        if st != g3.OK:
            raise g3.G3Error(st, f"request {req.rid}")
        if req.n_frames == 0:
            raise ValueError("a request needs at least one frame")
        if fr.dtype == np.int32:
            # one pass: a negative coordinate read as uint32 is >= 2^31 > L
            hi = fr.view(np.uint32).max(axis=(0, 2)) if fr.size else np.zeros(3, np.uint32)
            bad = bool(np.any(hi.astype(np.int64) >= np.asarray(req.box, dtype=np.int64)))
        else:
            lo = np.asarray(req.box, dtype=np.int64)[None, :, None]
            bad = bool(fr.size) and (fr.min() < 0 or bool(np.any(fr >= lo)))
        if bad:
            raise g3.G3Error(g3.EDOMAIN, f"request {req.rid}")
        req.nbytes = footprint_bytes(req, self.frames_per_iter)
        if req.nbytes + self.reserve > self.budget:
            raise g3.G3Error(g3.ENOMEM, f"request {req.rid} exceeds the HBM budget")
        self.queue.append(req)

    def request(self, frames: np.ndarray, box, rmax: float, nbins: int,
                layout: int = g3.HALF) -> Request:
        """Submit one analysis now and return its handle (a future): pass it
        to :meth:`result`.  ``frames`` is host int32 [F, 3, N]."""
        req = Request(self._next_rid, frames, list(box), float(rmax), int(nbins), int(layout),
                      arrival=self.now())
        self._next_rid += 1
        self.submit(req)
        return req

    def result(self, req: Request) -> np.ndarray:
        """Serve until ``req`` is complete and return its uint64 histogram
        (other requests keep advancing meanwhile).  On the GPU executor the
        array is a slice of a shared 16 MiB host block (see
        :class:`ResultBlocks`); ``.copy()`` it to hold it on its own."""
        while math.isnan(req.done):
            if not self.step():
                raise RuntimeError(f"request {req.rid} is not queued on this server")
        if req.status != g3.OK:
            raise g3.G3Error(req.status, f"request {req.rid}")
        return req.result

    def _admit(self):
        while self.queue and self.reserve + self.used + self.queue[0].nbytes <= self.budget:
            req = self.queue.popleft()
            req.dev_frames = self.ex.upload(req.frames)
            req.dev_hist = self.ex.new_hist(g3.hist_len(req.nbins, req.layout))
            req.admitted = self.now()
            self.used += req.nbytes
            self.peak_used = max(self.peak_used, self.used)
            self.active.append(req)

    def _release(self, req: Request):
        self.used -= req.nbytes
        self.ex.release(req.dev_frames, req.dev_hist)
        req.dev_frames = req.dev_hist = None
        self.completed.append(req)

    # -- one iteration ---------------------------------------------------------
    def _iterate(self):
        k = self.frames_per_iter
        systems, done_now = [], []
        for req in self.active:
            a, b = req.next_frame, min(req.next_frame + k, req.n_frames)
            systems.append(dict(frames=req.dev_frames[a:b], box=req.box, rmax=req.rmax,
                                nbins=req.nbins, layout=req.layout, hist=req.dev_hist))
            req.next_frame = b
            if b == req.n_frames:
                done_now.append(req)
        try:
            ticket = self.ex.accumulate_batch(systems)
        except Exception:
            for req in list(self.active):     # nothing of this batch was queued
                req.status = g3.EDEVICE
                req.done = self.now()
                self.active.remove(req)
                self._release(req)
            raise
        self.iterations += 1
        # A finishing request's histogram is copied to the host behind this
        # batch (stream order); it is final once the batch's ticket says so.
        for req in done_now:
            self.active.remove(req)
            req.ticket = ticket
            req.fetch = self.ex.start_fetch(req.dev_hist)
            self.finishing.append(req)
        ev = self.ex.record()
        for req in done_now:
            req.fetch_ev = ev
        self.in_flight.append(ev)

    def _complete(self) -> bool:
        """Complete the finishing requests whose copies have landed, in
        stream order; g3_sync runs only for a request with a flagged frame
        (then every finishing copy is taken again after it)."""
        did = False
        while self.finishing and self.finishing[0].fetch_ev.query():
            req = self.finishing[0]
            fin = self.ex.ticket_final(req.ticket)
            if fin is None:       # (its copy landed, so the batch has finished)
                break
            st = g3.OK
            if not fin:
                # a frame of this request is recomputed (or an error is
                # reported) by g3_sync; copies taken before it are stale
                st = self.ex.sync()
                self.syncs += 1
                self.in_flight.clear()
                for r in self.finishing:
                    r.fetch = self.ex.start_fetch(r.dev_hist)
                ev = self.ex.record()
                for r in self.finishing:
                    r.fetch_ev = ev
                ev.synchronize()
            self.finishing.popleft()
            req.status = st
            req.result = self.ex.finish_fetch(req.fetch)
            req.fetch = None
            req.done = self.now()
            self._release(req)
            did = True
            if st != g3.OK:
                raise g3.G3Error(st, f"request {req.rid}")
        return did

    def step(self) -> bool:
        """Complete what has landed, admit what fits and enqueue one
        iteration if there is work and room in flight.  Returns True if it
        did anything."""
        while self.in_flight and self.in_flight[0].query():
            self.in_flight.popleft()
        did = self._complete()
        self._admit()
        if self.active and len(self.in_flight) < self.max_in_flight:
            self._iterate()
            return True
        if self.in_flight:
            self.in_flight[0].synchronize()
            return True
        return did

    def pending(self) -> bool:
        return bool(self.queue or self.active or self.in_flight or self.finishing)

    def drain(self):
        while self.pending():
            if not self.step():
                break
        st = self.ex.sync()
        if st != g3.OK:
            raise g3.G3Error(st, "serving batch")

    # -- open-loop driver --------------------------------------------------------
    def run_open_loop(self, requests: list[Request], sample_device=False) -> dict:
        """Serve requests whose ``arrival`` times (seconds from start) form an
        open-loop schedule.  Returns latency and throughput statistics (with
        ``sample_device``, also the device memory in use, measured after each
        iteration, above what was in use at the start)."""
        pending = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        base = self.ex.device_used() if sample_device else 0
        dev_peak = 0
        i = 0
        while i < len(pending) or self.pending():
            now = self.now()
            while i < len(pending) and pending[i].arrival <= now:
                self.submit(pending[i])
                i += 1
            it = self.iterations
            if self.step():
                if sample_device and self.iterations != it:
                    dev_peak = max(dev_peak, self.ex.device_used() - base)
                continue
            if i < len(pending):
                time.sleep(max(0.0, min(pending[i].arrival - self.now(), 0.001)))
        st = self.ex.sync()
        if st != g3.OK:
            raise g3.G3Error(st, "serving batch")
        out = summarize(requests, self.now(), self.iterations, self.peak_used)
        out["syncs"] = self.syncs
        if sample_device:
            out["device_peak_bytes"] = int(dev_peak)
        return out


def summarize(requests: list[Request], wall: float, iterations: int, peak_used: int = 0) -> dict:
    lat = np.array([r.latency for r in requests]) * 1e3
    binned = sum(int(r.result.sum()) // (2 if r.layout == g3.FULL else 1) for r in requests)
    first = min(r.arrival for r in requests)
    last = max(r.done for r in requests)
    span = max(last - first, 1e-9)
    return {"requests": len(requests), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()), "triplets_binned": binned,
            "throughput_G_per_s": binned / span / 1e9, "requests_per_s": len(requests) / span,
            "iterations": iterations, "wall_s": wall, "peak_hbm_bytes": int(peak_used)}


class TrajectoryStore:
    """Seeded jittered-FCC trajectories that requests draw frames from, so a
    long request stream needs only a few generated systems."""

    def __init__(self, n_systems: int = 16, max_frames: int = 20, n_min: int = 1024,
                 n_max: int = 65536, seed=(20170833, 7)):
        from . import synth
        g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))
        self.max_frames = max_frames
        self.systems = []
        for s in range(n_systems):
            N = int(round(math.exp(g.uniform(math.log(n_min), math.log(n_max)))))
            rho = float(g.uniform(0.7, 0.9))
            frames, box = synth.jittered_fcc(N, rho, 0.1, max_frames, list(seed) + [s])
            self.systems.append((frames, box))

    def request(self, rid: int, g: np.random.Generator, arrival: float) -> Request:
        """frames ~ U{1..max_frames} of a random system, rmax in {2.0, 2.5,
        3.0} sigma with dr = 0.05 sigma, half layout."""
        s = int(g.integers(0, len(self.systems)))
        frames, box = self.systems[s]
        F = int(g.integers(1, frames.shape[0] + 1))
        a = int(g.integers(0, frames.shape[0] - F + 1))
        rm = float(g.choice([2.0, 2.5, 3.0]))
        return Request(rid, frames[a:a + F], list(box), rm * 4096.0, int(round(rm / 0.05)),
                       g3.HALF, arrival)


def poisson_requests(store: TrajectoryStore, n: int, rate_hz: float, seed=(20170833, 9)):
    """Open-loop Poisson arrivals at ``rate_hz``."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))
    t, out = 0.0, []
    for r in range(n):
        t += float(g.exponential(1.0 / rate_hz))
        out.append(store.request(r, g, t))
    return out
