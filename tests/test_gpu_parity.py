"""GPU parity: the HIP library (through the C ABI) against the CPU oracle,
bin for bin (integer histograms, tolerance 0)."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import refs
from paper_1708_08619_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


@pytest.fixture()
def plan(g3mod, torch_dev):
    p = g3mod.Plan()
    yield p
    p.close()


def _dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def run_plain(g3, plan, dev, frames, box, rmax, nbins, layout):
    h = g3.new_hist(nbins, layout, dev)
    plan.accumulate(_dev(frames.astype(np.int32), dev), box, rmax, nbins, layout, h)
    plan.sync()
    return h.cpu().numpy().astype(np.uint64)


def run_batch(g3, plan, dev, systems):
    """systems: list of (frames, box, rmax, nbins, layout)."""
    hs, args = [], []
    for fr, box, rmax, nbins, layout in systems:
        h = g3.new_hist(nbins, layout, dev)
        hs.append(h)
        args.append(dict(frames=_dev(fr.astype(np.int32), dev), box=box, rmax=rmax, nbins=nbins,
                         layout=layout, hist=h))
    plan.accumulate_batch(args)
    plan.sync()
    return [h.cpu().numpy().astype(np.uint64) for h in hs]


def both(g3, plan, dev, frames, box, rmax, nbins, layout):
    a = run_plain(g3, plan, dev, frames, box, rmax, nbins, layout)
    (b,) = run_batch(g3, plan, dev, [(frames, box, rmax, nbins, layout)])
    return a, b


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"{what}: {len(bad)} bins differ, first {bad[:5]}: "
                             f"got {got[bad[:5]]} want {want[bad[:5]]}")


# ------------------------------------------------------------------ worked cases
def _cases():
    with open(os.path.join(GOLDEN, "worked_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
@pytest.mark.parametrize("layout", [0, 1])
def test_worked_cases(g3mod, plan, torch_dev, oracle_mod, case, layout):
    pos = np.array(case["positions"], dtype=np.int64)
    fr = pos.T[None].astype(np.int32)
    want = oracle_mod.hist(fr, case["box"], case["rmax"], case["nbins"], layout)
    a, b = both(g3mod, plan, torch_dev, fr, case["box"], case["rmax"], case["nbins"], layout)
    assert_same(a, want, "plain")
    assert_same(b, want, "batched")


# ------------------------------------------------------------------ small LJ (N=256)
@pytest.mark.parametrize("kind", ["gas", "fcc"])
@pytest.mark.parametrize("layout", [0, 1])
def test_lj256(g3mod, plan, torch_dev, oracle_mod, kind, layout):
    w = synth.lj_small(kind, n_frames=10)
    want = oracle_mod.hist(w.frames, w.box, w.rmax, w.nbins, layout)
    a, b = both(g3mod, plan, torch_dev, w.frames, w.box, w.rmax, w.nbins, layout)
    assert_same(a, want, "plain")
    assert_same(b, want, "batched")
    assert want.sum() > 0


# ------------------------------------------------------------------ water (wide entries)
def test_water4096_wide_entries(g3mod, plan, torch_dev, oracle_mod):
    w = synth.water_like(n_frames=100)
    assert np.ceil(w.rmax) > 32767             # exercises the int32 entry path
    want = oracle_mod.hist(w.frames, w.box, w.rmax, w.nbins, w.layout)
    a, b = both(g3mod, plan, torch_dev, w.frames, w.box, w.rmax, w.nbins, w.layout)
    assert_same(a, want, "plain")
    assert_same(b, want, "batched")


# ------------------------------------------------------------------ random boxes
@pytest.mark.parametrize("seed", range(5))
def test_random_boxes(g3mod, plan, torch_dev, oracle_mod, seed):
    """Non-cubic boxes, ragged N (not a multiple of the centre block), rmax
    from L/5 up to just below L/2 of the smallest side, random nbins."""
    rng = np.random.default_rng(1000 + seed)
    box = [int(x) for x in rng.integers(20000, 60000, size=3)]
    rmax = float(rng.uniform(min(box) / 5, min(box) / 2 - 2))
    nbins = int(rng.integers(5, 64))
    N = int(rng.integers(300, 1500))
    F = 3
    fr = np.stack([np.stack([rng.integers(0, L, size=N) for L in box]) for _ in range(F)]
                  ).astype(np.int32)
    for layout in (0, 1):
        want = oracle_mod.hist(fr, box, rmax, nbins, layout)
        a, b = both(g3mod, plan, torch_dev, fr, box, rmax, nbins, layout)
        assert_same(a, want, f"plain layout {layout}")
        assert_same(b, want, f"batched layout {layout}")


def test_coincident_and_boundary_atoms(g3mod, plan, torch_dev, oracle_mod):
    """Atoms at the same point (r = 0, bin 0), on x = 0 and x = L - 1."""
    rng = np.random.default_rng(9)
    box = [30000, 31000, 32000]
    N = 400
    fr = np.stack([rng.integers(0, L, size=N) for L in box])[None].astype(np.int32)
    fr[0, :, 1] = fr[0, :, 0]
    fr[0, :, 2] = fr[0, :, 0]
    fr[0, 0, 3], fr[0, 0, 4] = 0, box[0] - 1
    fr[0, 1, 4] = fr[0, 1, 3]
    fr[0, 2, 4] = fr[0, 2, 3]
    for layout in (0, 1):
        want = oracle_mod.hist(fr, box, 9000.0, 30, layout)
        a, b = both(g3mod, plan, torch_dev, fr, box, 9000.0, 30, layout)
        assert_same(a, want, "plain")
        assert_same(b, want, "batched")


# ------------------------------------------------------------------ batching
def test_uneven_batch_matches_oracle(g3mod, plan, torch_dev, oracle_mod):
    """Eight systems of uneven size (smaller stand-in for the batched case so
    the oracle finishes quickly), mixed layouts, one graph launch."""
    rng = np.random.default_rng(21)
    systems = []
    for s in range(8):
        N = int(round(np.exp(rng.uniform(np.log(256), np.log(2048)))))
        rho = float(rng.uniform(0.7, 0.9))
        fr, box = synth.jittered_fcc(N, rho, 0.1, 2, [77, s])
        systems.append((fr, box, 2.5 * 4096, 50, s % 2))
    got = run_batch(g3mod, plan, torch_dev, systems)
    for (fr, box, rmax, nb, lay), h in zip(systems, got):
        assert_same(h, oracle_mod.hist(fr, box, rmax, nb, lay), f"N={fr.shape[2]}")


def test_batched_equals_sum_of_plain(g3mod, plan, torch_dev):
    ws = synth.uneven_batch()
    systems = [(w.frames, w.box, w.rmax, w.nbins, w.layout) for w in ws]
    got = run_batch(g3mod, plan, torch_dev, systems)
    for (fr, box, rmax, nb, lay), h in zip(systems, got):
        acc = np.zeros_like(h)
        for f in range(fr.shape[0]):
            acc += run_plain(g3mod, plan, torch_dev, fr[f:f + 1], box, rmax, nb, lay)
        assert_same(h, acc, f"N={fr.shape[2]}")


def test_mixed_entry_formats_in_one_batch(g3mod, plan, torch_dev, oracle_mod):
    w = synth.water_like(n_frames=3)
    s = synth.lj_small("fcc", n_frames=3)
    got = run_batch(g3mod, plan, torch_dev, [(w.frames, w.box, w.rmax, w.nbins, 0),
                                             (s.frames, s.box, s.rmax, s.nbins, 1)])
    assert_same(got[0], oracle_mod.hist(w.frames, w.box, w.rmax, w.nbins, 0), "water")
    assert_same(got[1], oracle_mod.hist(s.frames, s.box, s.rmax, s.nbins, 1), "lj")


def test_accumulate_adds(g3mod, plan, torch_dev, oracle_mod):
    w = synth.lj_small("fcc", n_frames=2)
    h = g3mod.new_hist(w.nbins, 0, torch_dev)
    fr = _dev(w.frames, torch_dev)
    plan.accumulate(fr, w.box, w.rmax, w.nbins, 0, h)
    plan.accumulate_batch([dict(frames=fr, box=w.box, rmax=w.rmax, nbins=w.nbins, layout=0,
                                hist=h)])
    plan.sync()
    want = oracle_mod.hist(w.frames, w.box, w.rmax, w.nbins, 0)
    assert_same(h.cpu().numpy().astype(np.uint64), 2 * want, "accumulated")


# ------------------------------------------------------------------ tuning invariance
@pytest.mark.parametrize("tun", [
    dict(lds_hist_bins=4096),                          # many thin slabs
    dict(centres_per_item=64),
    dict(centres_per_item=1024),
    dict(wg_per_cu=2),
    dict(per_centre=1),
    dict(per_centre=1, lds_hist_bins=4096, centres_per_item=64),
])
def test_tuning_does_not_change_results(g3mod, plan, torch_dev, oracle_mod, tun):
    w = synth.lj_small("fcc", n_frames=4)
    want = oracle_mod.hist(w.frames, w.box, w.rmax, w.nbins, 0)
    plan.set_tuning(**tun)
    a, b = both(g3mod, plan, torch_dev, w.frames, w.box, w.rmax, w.nbins, 0)
    assert_same(a, want, f"plain {tun}")
    assert_same(b, want, f"batched {tun}")


@pytest.mark.parametrize("per_centre", [0, 1])
@pytest.mark.parametrize("cb", [1024, 2048])
def test_item_over_2_32_candidates(g3mod, plan, torch_dev, per_centre, cb):
    """4000 atoms inside a 50-unit cube (rmax 5000, 10 bins): every side of
    every triplet is in bin 0, so the half histogram is N (N-1) (N-2) / 2 at
    bin 0 and zero elsewhere.  With 1024 or 2048 centres per item one item
    holds more than 2^32 candidate pairs, all aimed at one LDS counter; the
    kernel must split it into exact passes."""
    rng = np.random.default_rng(3)
    N = 4000
    box = [200000, 200000, 200000]
    fr = (100000 + rng.integers(0, 50, size=(1, 3, N))).astype(np.int32)
    plan.set_tuning(centres_per_item=cb, per_centre=per_centre)
    want = np.zeros(g3mod.hist_len(10, 0), np.uint64)
    want[0] = N * (N - 1) * (N - 2) // 2
    a, b = both(g3mod, plan, torch_dev, fr, box, 5000.0, 10, 0)
    assert_same(a, want, "plain")
    assert_same(b, want, "batched")


@pytest.mark.parametrize("per_centre", [0, 1])
def test_two_centres_per_thread_items(g3mod, plan, torch_dev, oracle_mod, per_centre):
    """2048 centres per work item: each thread of the triplet workgroup sets
    up two centres (3000 atoms, so both halves hold centres); both forms
    equal the oracle."""
    fr, box = synth.jittered_fcc(3000, 0.8, 0.1, 2, [41, 0])
    rmax, nb = 2.5 * 4096, 40
    plan.set_tuning(centres_per_item=2048, per_centre=per_centre)
    assert plan.get_tuning()["centres_per_item"] == 2048
    for layout in (0, 1):
        want = oracle_mod.hist(fr, box, rmax, nb, layout)
        a, b = both(g3mod, plan, torch_dev, fr, box, rmax, nb, layout)
        assert_same(a, want, f"plain layout {layout}")
        assert_same(b, want, f"batched layout {layout}")


@pytest.mark.parametrize("per_centre", [0, 1])
@pytest.mark.parametrize("layout", [0, 1])
def test_atomic_flush_fallback(g3mod, plan, torch_dev, oracle_mod, per_centre, layout):
    """One partial slot per launch: nearly every slab flush takes the 64-bit
    atomic path (mirror writes of the full layout, the triangle buffer of
    the default enumeration, a longer third axis); results are unchanged in
    both forms."""
    w = synth.lj_small("fcc", n_frames=3)
    plan.set_tuning(slot_limit=1, lds_hist_bins=4096, per_centre=per_centre)
    assert plan.get_tuning()["slot_limit"] == 1
    want = oracle_mod.hist(w.frames, w.box, w.rmax, w.nbins, layout)
    a, b = both(g3mod, plan, torch_dev, w.frames, w.box, w.rmax, w.nbins, layout)
    assert_same(a, want, "plain")
    assert_same(b, want, "batched")
    L = w.box[0]
    want3 = oracle_mod.hist(w.frames, w.box, L / 4.0, 16, layout, nbins_third=32)
    h = g3mod.new_hist(16, layout, torch_dev, nbins_third=32)
    plan.accumulate(_dev(w.frames.astype(np.int32), torch_dev), w.box, L / 4.0, 16, layout, h,
                    nbins_third=32)
    plan.sync()
    assert_same(h.cpu().numpy().astype(np.uint64), want3, "third axis")


@pytest.mark.parametrize("per_centre", [0, 1])
def test_narrow_components_beyond_int16(g3mod, plan, torch_dev, oracle_mod, per_centre):
    """rmax = 30000 units in a 100000-unit box: 3 cells of 33333 units per
    axis, so stencil components reach +-66666 while entries stay narrow
    (C <= 32767).  The neighbour test saturates components to int16; every
    saturated candidate must be rejected, every accepted one exact."""
    rng = np.random.default_rng(77)
    box = [100000, 100000, 100000]
    fr = np.stack([np.stack([rng.integers(0, L, size=500) for L in box]) for _ in range(2)])
    plan.set_tuning(per_centre=per_centre)
    for layout in (0, 1):
        want = oracle_mod.hist(fr, box, 30000.0, 20, layout)
        a, b = both(g3mod, plan, torch_dev, fr, box, 30000.0, 20, layout)
        assert_same(a, want, f"plain layout {layout}")
        assert_same(b, want, f"batched layout {layout}")


@pytest.mark.parametrize("per_centre", [0, 1])
def test_pad_entries_near_their_bound(g3mod, plan, torch_dev, oracle_mod, per_centre):
    """Neighbour lists end in pad entries that every row must reject: with
    rmax = 15000 units and a third axis of twice the bins (third side up to
    30000), the narrow pads (components -32768) sit close to the bound the
    host checks, 3 (32769 - C)^2 >= R3, so the triplet kernel runs its
    padded form on rows with large components."""
    rng = np.random.default_rng(91)
    box = [64000, 64000, 64000]
    fr = np.stack([np.stack([rng.integers(0, L, size=700) for L in box]) for _ in range(2)])
    plan.set_tuning(per_centre=per_centre)
    for layout in (0, 1):
        want = oracle_mod.hist(fr, box, 15000.0, 12, layout, nbins_third=24)
        h = g3mod.new_hist(12, layout, torch_dev, nbins_third=24)
        plan.accumulate(_dev(fr.astype(np.int32), torch_dev), box, 15000.0, 12, layout, h,
                        nbins_third=24)
        plan.sync()
        assert_same(h.cpu().numpy().astype(np.uint64), want, f"layout {layout}")
        a, b = both(g3mod, plan, torch_dev, fr, box, 15000.0, 12, layout)
        assert_same(a, oracle_mod.hist(fr, box, 15000.0, 12, layout), f"plain layout {layout}")
        assert_same(b, oracle_mod.hist(fr, box, 15000.0, 12, layout), f"batched layout {layout}")


# ------------------------------------------------------------------ edge cases
def test_empty_and_tiny(g3mod, plan, torch_dev):
    import torch
    box = [50000] * 3
    for N in (0, 1, 2):
        fr = torch.zeros((2, 3, N), dtype=torch.int32, device=torch_dev)
        h = g3mod.new_hist(10, 0, torch_dev)
        plan.accumulate(fr, box, 1000.0, 10, 0, h)
        plan.accumulate_batch([dict(frames=fr, box=box, rmax=1000.0, nbins=10, layout=0, hist=h)])
        plan.sync()
        assert int(h.sum().item()) == 0
    fr = torch.zeros((0, 3, 10), dtype=torch.int32, device=torch_dev)
    h = g3mod.new_hist(10, 0, torch_dev)
    plan.accumulate(fr, box, 1000.0, 10, 0, h)
    plan.sync()


def test_domain_error(g3mod, plan, torch_dev, oracle_mod):
    """A coordinate equal to L is outside [0, L): that frame adds nothing and
    g3_sync reports G3_EDOMAIN; the other frames still count."""
    w = synth.lj_small("gas", n_frames=3)
    fr = w.frames.copy()
    fr[1, 0, 7] = w.box[0]
    h = g3mod.new_hist(w.nbins, 0, torch_dev)
    plan.accumulate(_dev(fr, torch_dev), w.box, w.rmax, w.nbins, 0, h)
    assert plan.sync_status() == g3mod.EDOMAIN
    want = oracle_mod.hist(fr[[0, 2]], w.box, w.rmax, w.nbins, 0)
    assert_same(h.cpu().numpy().astype(np.uint64), want, "valid frames")
    h2 = g3mod.new_hist(w.nbins, 0, torch_dev)
    fr[1, 0, 7] = -1
    plan.accumulate_batch([dict(frames=_dev(fr, torch_dev), box=w.box, rmax=w.rmax,
                                nbins=w.nbins, layout=0, hist=h2)])
    assert plan.sync_status() == g3mod.EDOMAIN
    assert_same(h2.cpu().numpy().astype(np.uint64), want, "valid frames (batched)")
    plan.sync()                         # the error was reported once


def test_pool_overflow_is_recomputed(g3mod, plan, torch_dev, oracle_mod):
    """A dense cluster far above the uniform-density neighbour estimate: the
    batched scratch overflows, g3_sync recomputes the frame, result exact."""
    rng = np.random.default_rng(4)
    box = [200000] * 3
    N = 1200
    pos = np.stack([rng.integers(0, L, size=N) for L in box])
    c = np.array(box) // 2
    pos[:, :600] = (c[:, None] + rng.integers(-900, 900, size=(3, 600)))
    fr = pos[None].astype(np.int32)
    rmax, nb = 2500.0, 20
    want = oracle_mod.hist(fr, box, rmax, nb, 0)
    (b,) = run_batch(g3mod, plan, torch_dev, [(fr, box, rmax, nb, 0)])
    assert_same(b, want, "batched after recompute")


def test_too_many_neighbours_reports_enomem(g3mod, plan, torch_dev):
    rng = np.random.default_rng(5)
    box = [200000] * 3
    N = 4200                      # more neighbours than the per-centre capacity (4096)
    c = np.array(box) // 2
    fr = (c[:, None] + rng.integers(-500, 500, size=(3, N)))[None].astype(np.int32)
    h = g3mod.new_hist(10, 0, torch_dev)
    plan.accumulate(_dev(fr, torch_dev), box, 5000.0, 10, 0, h)
    assert plan.sync_status() == g3mod.ENOMEM
    assert int(h.sum().item()) == 0


def test_invalid_arguments_queue_nothing(g3mod, plan, torch_dev):
    w = synth.lj_small("gas", n_frames=1)
    h = g3mod.new_hist(w.nbins, 0, torch_dev)
    with pytest.raises(g3mod.G3Error):
        plan.accumulate(_dev(w.frames, torch_dev), [20000] * 3, w.rmax, w.nbins, 0, h)
    plan.sync()
    assert int(h.sum().item()) == 0


# ------------------------------------------------------------------ full size
def test_perfect_fcc_65536(g3mod, plan, torch_dev):
    """N = 65536 exactly as a 32x32x16 FCC crystal at the large-system
    density and cutoff: every site sees the same neighbour vectors, so the
    expected histogram follows from lattice vectors alone."""
    a = 6708                                   # ~1.638 sigma at 4096/sigma: rho ~ 0.91
    n = (32, 32, 16)
    box = [a * n[0], a * n[1], a * n[2]]
    h = a // 2
    basis = np.array([[0, 0, 0], [0, h, h], [h, 0, h], [h, h, 0]])
    g = np.stack(np.meshgrid(*[np.arange(k) * a for k in n], indexing="ij"), -1).reshape(-1, 3)
    sites = (g[:, None, :] + basis[None]).reshape(-1, 3)
    assert len(sites) == 65536
    fr = sites.T[None].astype(np.int32)
    rmax, nb = 3.0 * 4096, 60
    want_full = refs.lattice_full(refs.fcc_vectors(a, rmax), 65536, rmax, nb)
    for layout in (0, 1):
        if layout == 1:
            want = want_full.reshape(-1)
        else:
            import oracle
            want, bad = oracle.fold_half(want_full)
            assert bad == 0
        a_, b_ = both(g3mod, plan, torch_dev, fr, box, rmax, nb, layout)
        assert_same(a_, want, "plain")
        assert_same(b_, want, "batched")


def test_large_system_sampled_frames(g3mod, plan, torch_dev, oracle_mod):
    """The N=65536 workload in the benchmark's batched launch over all 50
    frames equals the sum of per-frame plain runs, and two sampled frames
    equal the oracle exactly."""
    w = synth.lj_large(n_frames=50)
    (batched,) = run_batch(g3mod, plan, torch_dev, [(w.frames, w.box, w.rmax, w.nbins, w.layout)])
    per = [run_plain(g3mod, plan, torch_dev, w.frames[f:f + 1], w.box, w.rmax, w.nbins, w.layout)
           for f in range(w.n_frames)]
    assert_same(batched, np.sum(per, axis=0, dtype=np.uint64), "batched vs sum of plain")
    for f in (0, 37):
        want = oracle_mod.hist(w.frames[f:f + 1], w.box, w.rmax, w.nbins, w.layout)
        assert_same(per[f], want, f"frame {f}")


# ------------------------------------------------------------------ enumeration modes
def _mode_workloads():
    out = []
    for kind in ("gas", "fcc"):
        w = synth.lj_small(kind, n_frames=3)
        for layout in (0, 1):
            out.append((f"lj256_{kind}_L{layout}", w.frames, w.box, w.rmax, w.nbins, layout))
    w = synth.water_like(n_frames=2)
    out.append(("water4096_wide", w.frames, w.box, w.rmax, w.nbins, 1))
    for seed in range(2):
        rng = np.random.default_rng(60 + seed)
        box = [int(x) for x in rng.integers(20000, 60000, size=3)]
        N = int(rng.integers(200, 1200))
        fr = np.stack([np.stack([rng.integers(0, L, size=N) for L in box]) for _ in range(2)])
        rmax = float(rng.uniform(0.3, 0.49) * min(box))     # past L/4 and L/3
        out.append((f"random{seed}", fr.astype(np.int32), box, rmax, int(rng.integers(5, 41)),
                    seed % 2))
    return out


@pytest.mark.parametrize("wl", _mode_workloads(), ids=lambda w: w[0])
@pytest.mark.parametrize("per_centre", [0, 1])
def test_enumeration_modes_match_oracle(g3mod, plan, torch_dev, oracle_mod, wl, per_centre):
    """Both enumerations (each triangle once and expanded, or every centre's
    pairs) give the oracle's histogram, in both forms."""
    _, fr, box, rmax, nbins, layout = wl
    plan.set_tuning(per_centre=per_centre)
    want = oracle_mod.hist(fr, box, rmax, nbins, layout)
    a, b = both(g3mod, plan, torch_dev, fr, box, rmax, nbins, layout)
    assert_same(a, want, "plain")
    assert_same(b, want, "batched")


def test_large_system_per_centre_mode(g3mod, plan, torch_dev, oracle_mod):
    """The N = 65536 workload with every centre's pairs evaluated (the
    paper's loop), two frames batched, equals the oracle."""
    w = synth.lj_large(n_frames=50)
    fr = w.frames[[3, 44]]
    plan.set_tuning(per_centre=1)
    (b,) = run_batch(g3mod, plan, torch_dev, [(fr, w.box, w.rmax, w.nbins, w.layout)])
    assert_same(b, oracle_mod.hist(fr, w.box, w.rmax, w.nbins, w.layout), "per-centre batched")
