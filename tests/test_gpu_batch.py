"""GPU: the batched form on the uneven-systems workload at its configured
size against the oracle, the autotuner, per-call completion tickets, many
small systems in runs of items, mixed features in one batch, and bin tables
shared only between systems with equal parameters."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1708_08619_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def g3mod():
    from paper_1708_08619_amd import g3
    g3.lib()
    return g3


def _dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(dev)


def _systems(g3, ws, dev):
    return [dict(frames=_dev(w.frames, dev), box=w.box, rmax=w.rmax, nbins=w.nbins,
                 layout=w.layout, hist=g3.new_hist(w.nbins, w.layout, dev)) for w in ws]


def test_uneven_batch_full_size_matches_oracle(g3mod, torch_dev, oracle_mod):
    """8 systems, N log-uniform in 512..32768, densities 0.7-0.9, 8 jittered
    FCC frames each, rmax 2.5 sigma, 50 bins, full layout: one batched call
    (the frame x atom flattening of Sec. 3.2 applied to g3), every system's
    histogram equal to the oracle's, bin for bin."""
    ws = synth.uneven_batch()
    assert len(ws) == 8 and all(w.frames.shape[0] == 8 for w in ws)
    with g3mod.Plan() as plan:
        systems = _systems(g3mod, ws, torch_dev)
        plan.accumulate_batch(systems)
        plan.sync()
        for w, s in zip(ws, systems):
            got = s["hist"].cpu().numpy().astype(np.uint64)
            want = oracle_mod.hist(w.frames, w.box, w.rmax, w.nbins, w.layout)
            assert np.array_equal(got, want), w.name


def test_autotune_picks_from_grid_and_stays_exact(g3mod, torch_dev, oracle_mod):
    """The autotuner returns a tuning from its grid (workgroups per CU,
    centres per item, all or 3/4 of the LDS histogram), never writes the
    callers' histograms, and the chosen tuning reproduces the oracle."""
    rng = np.random.default_rng(31)
    ws = []
    for s in range(4):
        N = int(round(np.exp(rng.uniform(np.log(400), np.log(3000)))))
        fr, box = synth.jittered_fcc(N, float(rng.uniform(0.7, 0.9)), 0.1, 2, [91, s])
        ws.append(synth.Workload(f"t{s}", fr, box, 2.5 * 4096, 50, s % 2))
    with g3mod.Plan() as plan:
        systems = _systems(g3mod, ws, torch_dev)
        best = plan.autotune(systems)
        for s in systems:
            assert int(s["hist"].count_nonzero().item()) == 0
        assert best["wg_per_cu"] in (1, 2)
        assert best["centres_per_item"] in (256, 512, 1024, 2048)
        # the LDS sizes on the grid: all of what fits beside the item arrays, or 3/4
        probe = g3mod.Plan()
        probe.set_tuning(wg_per_cu=best["wg_per_cu"], centres_per_item=best["centres_per_item"])
        full = probe.get_tuning()["lds_hist_bins"]
        probe.close()
        assert best["lds_hist_bins"] in (full, (full * 3 // 4) & ~63), (best, full)
        assert plan.get_tuning()["lds_hist_bins"] == best["lds_hist_bins"]
        # a second call with the same workload returns the cached tuning
        assert plan.autotune(systems) == best
        plan.accumulate_batch(systems)
        plan.sync()
        for w, s in zip(ws, systems):
            got = s["hist"].cpu().numpy().astype(np.uint64)
            assert np.array_equal(got, oracle_mod.hist(w.frames, w.box, w.rmax, w.nbins, w.layout))


def test_tickets(g3mod, torch_dev, oracle_mod):
    """g3_ticket_query: final once an ordinary call has run; not final for a
    call with a frame to recompute until g3_sync has run; unknown tickets are
    rejected.  The frame to recompute: 2200 atoms in a 50-unit cube with
    2048-centre items, so some lists are longer than such items allow (their
    candidate pairs could pass 2^32); every side is in bin 0, so the half
    histogram is N (N-1) (N-2) / 2 at bin 0."""
    import torch
    w = synth.lj_small("fcc", n_frames=2)
    rng = np.random.default_rng(4)
    box = [200000] * 3
    Nd = 2200
    dense = (100000 + rng.integers(0, 50, size=(1, 3, Nd))).astype(np.int32)
    want_dense = np.zeros(g3mod.hist_len(10, 0), np.uint64)
    want_dense[0] = Nd * (Nd - 1) * (Nd - 2) // 2
    with g3mod.Plan() as plan:
        plan.set_tuning(centres_per_item=2048)
        assert plan.last_ticket() == 0
        h = g3mod.new_hist(w.nbins, w.layout, torch_dev)
        plan.accumulate_batch([dict(frames=_dev(w.frames, torch_dev), box=w.box, rmax=w.rmax,
                                    nbins=w.nbins, layout=w.layout, hist=h)])
        t1 = plan.last_ticket()
        assert t1 == 1
        torch.cuda.synchronize()
        assert plan.ticket_query(t1) is True
        assert np.array_equal(h.cpu().numpy().astype(np.uint64),
                              oracle_mod.hist(w.frames, w.box, w.rmax, w.nbins, w.layout))
        hd = g3mod.new_hist(10, 0, torch_dev)
        plan.accumulate_batch([dict(frames=_dev(dense, torch_dev), box=box, rmax=5000.0, nbins=10,
                                    layout=0, hist=hd)])
        t2 = plan.last_ticket()
        assert t2 == 2
        torch.cuda.synchronize()
        assert plan.ticket_query(t2) is False      # the frame awaits g3_sync's recomputation
        assert plan.ticket_query(t1) is True
        plan.sync()
        assert plan.ticket_query(t2) is True
        assert np.array_equal(hd.cpu().numpy().astype(np.uint64), want_dense)
        with pytest.raises(g3mod.G3Error):
            plan.ticket_query(3)
        with pytest.raises(g3mod.G3Error):
            plan.ticket_query(0)


def test_many_small_systems_in_runs(g3mod, torch_dev, oracle_mod):
    """120 small systems (N 200..800, 3 frames, both layouts) at 64 centres
    per item: about 10^4 items, so the work counter hands out runs of
    several consecutive items of each small segment; every system equals the
    oracle bin for bin."""
    rng = np.random.default_rng(47)
    ws = []
    for k in range(120):
        N = int(rng.integers(200, 801))
        fr, box = synth.jittered_fcc(N, float(rng.uniform(0.7, 0.9)), 0.1, 3, [47, k])
        ws.append(synth.Workload(f"small{k}", fr, box, 2.5 * 4096, 50, int(rng.integers(0, 2)), {}))
    with g3mod.Plan() as plan:
        plan.set_tuning(centres_per_item=64)
        systems = _systems(g3mod, ws, torch_dev)
        plan.accumulate_batch(systems)
        plan.sync()
        for w, s in zip(ws, systems):
            got = s["hist"].cpu().numpy().astype(np.uint64)
            assert np.array_equal(got, oracle_mod.hist(w.frames, w.box, w.rmax, w.nbins, w.layout)), w.name


def test_mixed_features_in_one_batch(g3mod, torch_dev, oracle_mod):
    """72 small systems in one batch at 64 centres per item (runs of several
    items): cutoffs 2.0-2.5 sigma, 30-50 bins, both layouts, every third
    system with the pair histogram (the launch's build then keeps pair
    counters), every fourth with a doubled third axis (the per-centre
    enumeration beside triangle-once systems); every histogram and pair
    histogram equals the oracle's."""
    rng = np.random.default_rng(53)
    cases, systems = [], []
    for k in range(72):
        N = int(rng.integers(200, 701))
        rho = float(rng.uniform(0.7, 0.9))
        fr, box = synth.jittered_fcc(N, rho, 0.1, 2, [53, k])
        rmax = float(rng.uniform(2.0, 2.5)) * 4096
        nb = int(rng.integers(30, 51))
        layout = int(rng.integers(0, 2))
        nc = 2 * nb if k % 4 == 3 else nb
        if nc > nb:                 # the third cutoff (2 rmax) must stay below L/2
            rmax = min(rmax, (min(box) / 2 - 2) / 2)
        h = g3mod.new_hist(nb, layout, torch_dev, nbins_third=nc)
        p = g3mod.new_pair_hist(nb, torch_dev) if k % 3 == 0 else None
        s = dict(frames=_dev(fr, torch_dev), box=box, rmax=rmax, nbins=nb, layout=layout, hist=h,
                 nbins_third=nc)
        if p is not None:
            s["pair_hist"] = p
        systems.append(s)
        cases.append((fr, box, rmax, nb, layout, nc))
    with g3mod.Plan() as plan:
        plan.set_tuning(centres_per_item=64)
        plan.accumulate_batch(systems)
        plan.sync()
        for k, ((fr, box, rmax, nb, layout, nc), s) in enumerate(zip(cases, systems)):
            got = s["hist"].cpu().numpy().astype(np.uint64)
            assert np.array_equal(got, oracle_mod.hist(fr, box, rmax, nb, layout, nbins_third=nc)), k
            if "pair_hist" in s:
                gp = s["pair_hist"].cpu().numpy().astype(np.uint64)
                assert np.array_equal(gp, oracle_mod.pair_hist(fr, box, rmax, nb)), k


def test_bin_tables_shared_only_between_equal_parameters(g3mod, torch_dev, oracle_mod):
    """A batch keeps one copy of the bin tables per (rmax, nbins,
    nbins_third).  Systems whose cutoffs differ by half a unit or one unit
    (thresholds differ in a few bins), one with the same cutoff and a
    doubled third axis, and exact repeats, interleaved in one batch: each
    equals the oracle bin for bin, so no system read another's tables."""
    base = 1.5 * 4096
    params = [(base, 30, 30), (base + 0.5, 30, 30), (base, 30, 60), (base + 1.0, 30, 30),
              (base, 30, 30), (base + 0.5, 30, 30), (base, 29, 29), (base, 30, 60)]
    cases, systems = [], []
    for k, (rmax, nb, nc) in enumerate(params):
        fr, box = synth.jittered_fcc(400 + 37 * k, 0.85, 0.1, 2, [59, k])
        if nc > nb:                 # the third cutoff (2 rmax) must stay below L/2
            assert 2 * rmax < min(box) / 2
        layout = k % 2
        h = g3mod.new_hist(nb, layout, torch_dev, nbins_third=nc)
        systems.append(dict(frames=_dev(fr, torch_dev), box=box, rmax=rmax, nbins=nb, layout=layout,
                            hist=h, nbins_third=nc))
        cases.append((fr, box, rmax, nb, layout, nc))
    with g3mod.Plan() as plan:
        plan.accumulate_batch(systems)
        plan.sync()
        for k, ((fr, box, rmax, nb, layout, nc), s) in enumerate(zip(cases, systems)):
            got = s["hist"].cpu().numpy().astype(np.uint64)
            assert np.array_equal(got, oracle_mod.hist(fr, box, rmax, nb, layout, nbins_third=nc)), k
