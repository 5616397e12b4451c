"""Scheduler logic of the serving loop on the CPU: a fake executor backed by
the oracle stands in for the GPU, so admission by HBM budget, FIFO order,
frame chunking across iterations, rejection of bad requests and release of
memory after a failure are checked without a device."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1708_08619_amd import g3, serve, synth


class _Done:
    def query(self):
        return True

    def synchronize(self):
        pass


class OracleExecutor:
    """Executes batches with the oracle; device buffers are numpy arrays.

    ``late`` names frames counts (by request frames' identity, see
    ``late_ids``) that a batch leaves out and ``sync`` adds afterwards, the
    way the library recomputes a flagged frame in g3_sync: a batch holding
    such a frame gets a ticket that is not final, and a histogram copied
    before the sync misses those counts."""

    def __init__(self, oracle_mod, fail_on_call=None, late_ids=()):
        self.o = oracle_mod
        self.calls = 0
        self.fail_on_call = fail_on_call
        self.live = 0
        self.late_ids = set(late_ids)
        self.withheld = []          # (hist, counts) added by the next sync
        self.tickets = {}           # ticket -> final
        self.syncs = 0

    def upload(self, frames):
        self.live += 1
        return np.ascontiguousarray(frames, dtype=np.int32)

    def new_hist(self, n):
        return np.zeros(n, dtype=np.uint64)

    def accumulate_batch(self, systems):
        self.calls += 1
        if self.fail_on_call == self.calls:
            raise RuntimeError("injected executor failure")
        final = True
        for s in systems:
            h = self.o.hist(s["frames"], s["box"], s["rmax"], s["nbins"], s["layout"])
            if s.get("tag") in self.late_ids:
                self.withheld.append((s["hist"], h))
                final = False
            else:
                s["hist"] += h
        self.tickets[self.calls] = final
        return self.calls

    def ticket_final(self, ticket):
        return self.tickets[ticket]

    def start_fetch(self, hist):
        return hist.copy()

    def finish_fetch(self, tok):
        return tok

    def release(self, frames, hist):
        self.live -= 1

    def sync(self):
        self.syncs += 1
        for h, add in self.withheld:
            h += add
        self.withheld.clear()
        for t in self.tickets:
            self.tickets[t] = True
        return g3.OK

    def record(self):
        return _Done()


def _requests(n, seed=3):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n):
        N = int(rng.integers(150, 260))
        F = int(rng.integers(1, 7))
        fr, box = synth.jittered_fcc(N, 0.8, 0.1, F, [seed, r])
        rm = float(rng.choice([2.0, 2.5]))
        out.append(serve.Request(r, fr, box, rm * 4096, int(round(rm / 0.05)),
                                 int(rng.integers(0, 2)), arrival=0.0))
    return out


def test_results_and_budget(oracle_mod):
    reqs = _requests(10)
    fp = [serve.footprint_bytes(r, 2) for r in reqs]
    budget = 2 * max(fp)                      # at most two requests fit at once
    ex = OracleExecutor(oracle_mod)
    srv = serve.Server(budget, frames_per_iter=2, executor=ex)
    for r in reqs:
        srv.submit(r)
    srv.drain()
    assert srv.peak_used <= budget
    assert srv.used == 0 and ex.live == 0
    for r in reqs:
        want = oracle_mod.hist(r.frames, r.box, r.rmax, r.nbins, r.layout)
        assert np.array_equal(r.result, want), r.rid
    # FIFO admission, and queueing happened: someone was admitted after
    # another finished
    adm = [r.admitted for r in reqs]
    assert adm == sorted(adm)
    assert any(r.admitted >= min(q.done for q in reqs) for r in reqs)
    assert srv.iterations >= max(r.n_frames for r in reqs) / 2


def test_rejections(oracle_mod):
    srv = serve.Server(1 << 20, frames_per_iter=2, executor=OracleExecutor(oracle_mod))
    fr, box = synth.jittered_fcc(64, 0.8, 0.1, 2, [5, 0])
    bad = fr.copy()
    bad[0, 0, 0] = box[0]
    with pytest.raises(g3.G3Error) as e:
        srv.submit(serve.Request(0, bad, box, 2.0 * 4096, 40))
    assert e.value.status == g3.EDOMAIN
    # a negative coordinate, on each axis, in int32 and in a wider type
    for ax in range(3):
        for dt in (np.int32, np.int64):
            neg = fr.astype(dt)
            neg[-1, ax, -1] = -1
            with pytest.raises(g3.G3Error) as e:
                srv.submit(serve.Request(0, neg, box, 2.0 * 4096, 40))
            assert e.value.status == g3.EDOMAIN
            hi = fr.astype(dt)
            hi[0, ax, 1] = box[ax]
            with pytest.raises(g3.G3Error) as e:
                srv.submit(serve.Request(0, hi, box, 2.0 * 4096, 40))
            assert e.value.status == g3.EDOMAIN
    edge = fr.copy()
    edge[0, :, 0] = np.asarray(box) - 1            # the largest valid coordinates
    edge[0, :, 1] = 0
    srv.submit(serve.Request(9, edge, box, 2.0 * 4096, 40))
    srv.queue.clear()
    with pytest.raises(g3.G3Error) as e:
        srv.submit(serve.Request(1, fr, box, 0.5, 40))
    assert e.value.status == g3.EINVAL
    big = np.zeros((20, 3, 70000), dtype=np.int32)
    with pytest.raises(g3.G3Error) as e:
        srv.submit(serve.Request(2, big, [500000] * 3, 3.0 * 4096, 60))
    assert e.value.status == g3.ENOMEM
    assert not srv.queue


def test_failure_releases_memory(oracle_mod):
    reqs = _requests(4, seed=7)
    ex = OracleExecutor(oracle_mod, fail_on_call=2)
    srv = serve.Server(1 << 30, frames_per_iter=1, executor=ex)
    for r in reqs:
        srv.submit(r)
    with pytest.raises(RuntimeError):
        srv.drain()
    assert srv.used == 0 and not srv.active and ex.live == 0
    failed = [r for r in reqs if r.status == g3.EDEVICE]
    assert failed


def test_future_api(oracle_mod):
    """submit -> handle, result(handle) -> histogram; a later request can be
    collected first and an earlier one still completes."""
    srv = serve.Server(1 << 30, frames_per_iter=1, executor=OracleExecutor(oracle_mod))
    a_fr, a_box = synth.jittered_fcc(200, 0.8, 0.1, 3, [9, 0])
    b_fr, b_box = synth.jittered_fcc(180, 0.8, 0.1, 1, [9, 1])
    fa = srv.request(a_fr, a_box, 2.0 * 4096, 40)
    fb = srv.request(b_fr, b_box, 2.5 * 4096, 50, g3.FULL)
    hb = srv.result(fb)
    assert np.array_equal(hb, oracle_mod.hist(b_fr, b_box, 2.5 * 4096, 50, g3.FULL))
    ha = srv.result(fa)
    assert np.array_equal(ha, oracle_mod.hist(a_fr, a_box, 2.0 * 4096, 40, g3.HALF))
    assert fa.rid != fb.rid and srv.used == 0


def test_recomputed_frames_are_in_the_result(oracle_mod, monkeypatch):
    """A batch whose ticket is not final (a frame the library recomputes in
    g3_sync) must not complete a request from a copy taken before the sync:
    the server syncs, copies again, and every result equals the oracle."""
    reqs = _requests(6, seed=11)
    late = {reqs[2].rid, reqs[4].rid}
    ex = OracleExecutor(oracle_mod, late_ids=late)
    srv = serve.Server(1 << 30, frames_per_iter=2, executor=ex)
    orig = srv._iterate

    def tagged():
        # tag each system with its request so the executor can hold it back
        real = ex.accumulate_batch

        def acc(systems):
            for s, r in zip(systems, list(srv.active)):
                s["tag"] = r.rid
            return real(systems)
        ex.accumulate_batch = acc
        try:
            orig()
        finally:
            ex.accumulate_batch = real
    monkeypatch.setattr(srv, "_iterate", tagged)
    for r in reqs:
        srv.submit(r)
    srv.drain()
    assert ex.syncs >= 1 and srv.syncs >= 1
    for r in reqs:
        want = oracle_mod.hist(r.frames, r.box, r.rmax, r.nbins, r.layout)
        assert np.array_equal(r.result, want), r.rid
    assert srv.used == 0 and ex.live == 0


def test_result_blocks_hand_out_disjoint_slices():
    """Histograms copied out of the device land in slices of shared host
    blocks: every slice has its length, slices never overlap (each keeps its
    own values), a full block is followed by a new one, and a histogram
    larger than a block gets an array of its own."""
    rb = serve.ResultBlocks()
    words = rb.BLOCK_BYTES // 8
    rng = np.random.default_rng(5)
    sizes = [int(x) for x in rng.integers(1, words // 7, size=40)] + [words, words + 1, 3]
    outs = []
    for k, n in enumerate(sizes):
        o = rb.take(n)
        assert o.shape == (n,) and o.dtype == np.uint64
        if o.base is not None:
            assert (o.ctypes.data - o.base.ctypes.data) % 64 == 0
        o[:] = k
        outs.append(o)
    for k, o in enumerate(outs):
        assert np.all(o == k), k
    spans = sorted((o.ctypes.data, o.ctypes.data + 8 * o.size) for o in outs)
    assert all(a[1] <= b[0] for a, b in zip(spans, spans[1:]))
    assert outs[-2].base is None or outs[-2].base.size == words + 1   # its own array
