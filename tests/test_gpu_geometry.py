"""GPU parity of the longer third axis (nbins_third bins of the pair-bin
width; with rmax = L/4 and 2 nbins this is the paper's geometry: two sides
below L/4, the third below L/2), against the oracle, bin for bin."""
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


@pytest.fixture()
def plan(g3mod, torch_dev):
    p = g3mod.Plan()
    yield p
    p.close()


def _dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(dev)


def _np(t):
    return t.cpu().numpy().astype(np.uint64)


def _workloads():
    out = []
    for kind in ("fcc", "gas"):
        w = synth.lj_small(kind, n_frames=3)
        L = w.box[0]
        out.append((f"lj256_{kind}_quarter_box", w.frames, w.box, L / 4.0, 20, 40))
    for seed in range(3):
        rng = np.random.default_rng(80 + seed)
        box = [int(x) for x in rng.integers(30000, 60000, size=3)]
        N = int(rng.integers(300, 1500))
        fr = np.stack([np.stack([rng.integers(0, L, size=N) for L in box]) for _ in range(2)])
        nb = int(rng.integers(5, 30))
        out.append((f"random{seed}", fr.astype(np.int32), box, float(rng.uniform(0.1, 0.25) * min(box)),
                    nb, nb + int(rng.integers(1, nb + 1))))
    # third cutoff 40000 units: 32-bit entries
    rng = np.random.default_rng(90)
    box = [80000] * 3
    fr = np.stack([np.stack([rng.integers(0, L, size=1500) for L in box]) for _ in range(2)])
    out.append(("wide_third", fr.astype(np.int32), box, 20000.0, 25, 50))
    return out


@pytest.mark.parametrize("wl", _workloads(), ids=lambda w: w[0])
@pytest.mark.parametrize("layout", [0, 1])
def test_third_axis_matches_oracle(g3mod, plan, torch_dev, oracle_mod, wl, layout):
    _, fr, box, rmax, nb, nc = wl
    want = oracle_mod.hist(fr, box, rmax, nb, layout, nbins_third=nc)
    want_p = oracle_mod.pair_hist(fr, box, rmax, nb)
    h = g3mod.new_hist(nb, layout, torch_dev, nbins_third=nc)
    p = g3mod.new_pair_hist(nb, torch_dev)
    plan.accumulate(_dev(fr, torch_dev), box, rmax, nb, layout, h, pair_hist=p, nbins_third=nc)
    plan.sync()
    assert np.array_equal(_np(h), want) and np.array_equal(_np(p), want_p)
    hb = g3mod.new_hist(nb, layout, torch_dev, nbins_third=nc)
    plan.accumulate_batch([dict(frames=_dev(fr, torch_dev), box=box, rmax=rmax, nbins=nb,
                                layout=layout, hist=hb, nbins_third=nc)])
    plan.sync()
    assert np.array_equal(_np(hb), want)


def test_mixed_batch_of_both_axes(g3mod, plan, torch_dev, oracle_mod):
    """One batch: a system with the one-cutoff axis (triangle-once) beside one
    with the paper's geometry (per-centre); both exact."""
    w = synth.lj_small("fcc", n_frames=2)
    L = w.box[0]
    g = synth.lj_small("gas", n_frames=2)
    want_a = oracle_mod.hist(w.frames, w.box, w.rmax, w.nbins, 0)
    want_b = oracle_mod.hist(g.frames, g.box, L / 4.0, 16, 1, nbins_third=32)
    ha = g3mod.new_hist(w.nbins, 0, torch_dev)
    hb = g3mod.new_hist(16, 1, torch_dev, nbins_third=32)
    plan.accumulate_batch([
        dict(frames=_dev(w.frames, torch_dev), box=w.box, rmax=w.rmax, nbins=w.nbins, layout=0, hist=ha),
        dict(frames=_dev(g.frames, torch_dev), box=g.box, rmax=L / 4.0, nbins=16, layout=1, hist=hb,
             nbins_third=32)])
    plan.sync()
    assert np.array_equal(_np(ha), want_a) and np.array_equal(_np(hb), want_b)


def test_third_axis_arguments(g3mod, plan, torch_dev):
    w = synth.lj_small("gas", n_frames=1)
    fr = _dev(w.frames, torch_dev)
    for nc in (19, 41):                     # below nbins, above 2 nbins
        with pytest.raises((g3mod.G3Error, ValueError)):
            h = g3mod.new_hist(20, 0, torch_dev, nbins_third=max(nc, 20))
            plan.accumulate(fr, w.box, w.rmax, 20, 0, h, nbins_third=nc)
    big = [200000] * 3
    h = g3mod.new_hist(10, 0, torch_dev, nbins_third=20)
    with pytest.raises(g3mod.G3Error):      # third cutoff 2 x 30000 > 46340 units
        plan.accumulate(_dev(np.zeros((1, 3, 8), np.int32), torch_dev), big, 30000.0, 10, 0, h,
                        nbins_third=20)
    plan.sync()


def test_paper_shape_replay_frame(g3mod, plan, torch_dev, oracle_mod):
    """One frame of the N = 6720 water-density replay (two sides below L/4,
    the third below L/2, 80 x 80 x 160 bins, full layout), batched, equals the
    oracle bin for bin."""
    w = synth.water_replay(6720, n_frames=1)
    nc = w.meta["nbins_third"]
    want = oracle_mod.hist(w.frames, w.box, w.rmax, w.nbins, w.layout, nbins_third=nc)
    h = g3mod.new_hist(w.nbins, w.layout, torch_dev, nbins_third=nc)
    plan.accumulate_batch([dict(frames=_dev(w.frames, torch_dev), box=w.box, rmax=w.rmax,
                                nbins=w.nbins, layout=w.layout, hist=h, nbins_third=nc)])
    plan.sync()
    got = _np(h)
    assert np.array_equal(got, want)
    assert got.reshape(w.nbins, w.nbins, nc)[:, :, w.nbins:].sum() > 0
