"""GPU parity of the pair histogram (g2 output): the library's pair_hist
against the oracle's ordered-pair count, bin for bin, in the plain and the
batched form, with the triplet histogram checked beside it."""
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


def plain_pairs(g3, plan, dev, fr, box, rmax, nbins, layout):
    h, p = g3.new_hist(nbins, layout, dev), g3.new_pair_hist(nbins, dev)
    plan.accumulate(_dev(fr, dev), box, rmax, nbins, layout, h, pair_hist=p)
    plan.sync()
    return _np(h), _np(p)


def batch_pairs(g3, plan, dev, systems):
    out, args = [], []
    for fr, box, rmax, nbins, layout in systems:
        h, p = g3.new_hist(nbins, layout, dev), g3.new_pair_hist(nbins, dev)
        out.append((h, p))
        args.append(dict(frames=_dev(fr, dev), box=box, rmax=rmax, nbins=nbins, layout=layout,
                         hist=h, pair_hist=p))
    plan.accumulate_batch(args)
    plan.sync()
    return [(_np(h), _np(p)) for h, p in out]


def _workloads():
    out = []
    for kind in ("gas", "fcc"):
        w = synth.lj_small(kind, n_frames=3)
        out.append((f"lj256_{kind}", w.frames, w.box, w.rmax, w.nbins, kind == "gas"))
    w = synth.water_like(n_frames=2)
    out.append(("water4096_wide", w.frames, w.box, w.rmax, w.nbins, 1))
    for seed in range(3):
        rng = np.random.default_rng(40 + seed)
        box = [int(x) for x in rng.integers(20000, 60000, size=3)]
        N = int(rng.integers(200, 1500))
        fr = np.stack([np.stack([rng.integers(0, L, size=N) for L in box]) for _ in range(2)])
        rmax = float(rng.uniform(0.15, 0.45) * min(box))
        out.append((f"random{seed}", fr.astype(np.int32), box, rmax, int(rng.integers(5, 61)),
                    seed % 2))
    return out


@pytest.mark.parametrize("wl", _workloads(), ids=lambda w: w[0])
def test_pairs_match_oracle(g3mod, plan, torch_dev, oracle_mod, wl):
    _, fr, box, rmax, nbins, layout = wl
    want_p = oracle_mod.pair_hist(fr, box, rmax, nbins)
    want_h = oracle_mod.hist(fr, box, rmax, nbins, layout)
    h, p = plain_pairs(g3mod, plan, torch_dev, fr, box, rmax, nbins, layout)
    assert np.array_equal(p, want_p) and np.array_equal(h, want_h)
    ((h, p),) = batch_pairs(g3mod, plan, torch_dev, [(fr, box, rmax, nbins, layout)])
    assert np.array_equal(p, want_p) and np.array_equal(h, want_h)


def test_pairs_shared_by_systems_of_a_batch(g3mod, plan, torch_dev, oracle_mod):
    ws = synth.uneven_batch(n_systems=3, frames_per_system=2)
    nb = ws[0].nbins
    assert all(w.nbins == nb for w in ws)
    shared = g3mod.new_pair_hist(nb, torch_dev)
    args = [dict(frames=_dev(w.frames, torch_dev), box=w.box, rmax=w.rmax, nbins=w.nbins,
                 layout=w.layout, hist=g3mod.new_hist(w.nbins, w.layout, torch_dev),
                 pair_hist=shared) for w in ws]
    plan.accumulate_batch(args)
    plan.sync()
    want = sum(oracle_mod.pair_hist(w.frames, w.box, w.rmax, w.nbins) for w in ws)
    assert np.array_equal(_np(shared), want)


def test_two_atoms_count_pairs_only(g3mod, plan, torch_dev, oracle_mod):
    box = [40000] * 3
    fr = np.array([[[100, 3000]], [[100, 100]], [[100, 39900]]], dtype=np.int32)
    fr = np.transpose(fr, (1, 0, 2)).copy()            # [1][3][2]
    fr = np.concatenate([fr, fr + 7])
    h, p = plain_pairs(g3mod, plan, torch_dev, fr, box, 5000.0, 10, 0)
    assert int(h.sum()) == 0
    assert np.array_equal(p, oracle_mod.pair_hist(fr, box, 5000.0, 10)) and p.sum() == 4
    ((h, p),) = batch_pairs(g3mod, plan, torch_dev, [(fr, box, 5000.0, 10, 0)])
    assert int(h.sum()) == 0 and p.sum() == 4


def test_pool_overflow_counts_pairs_once(g3mod, plan, torch_dev, oracle_mod):
    """The frame whose batched scratch overflows is recomputed by g3_sync; its
    pairs were already counted in full and are not added again."""
    rng = np.random.default_rng(4)
    box = [200000] * 3
    N = 1200
    pos = np.stack([rng.integers(0, L, size=N) for L in box])
    c = np.array(box) // 2
    pos[:, :600] = (c[:, None] + rng.integers(-900, 900, size=(3, 600)))
    fr = pos[None].astype(np.int32)
    ((h, p),) = batch_pairs(g3mod, plan, torch_dev, [(fr, box, 2500.0, 20, 0)])
    assert np.array_equal(h, oracle_mod.hist(fr, box, 2500.0, 20, 0))
    assert np.array_equal(p, oracle_mod.pair_hist(fr, box, 2500.0, 20))


def test_capacity_error_still_counts_pairs(g3mod, plan, torch_dev, oracle_mod):
    rng = np.random.default_rng(5)
    box = [200000] * 3
    c = np.array(box) // 2
    fr = (c[:, None] + rng.integers(-500, 500, size=(3, 4200)))[None].astype(np.int32)
    h, p = g3mod.new_hist(10, 0, torch_dev), g3mod.new_pair_hist(10, torch_dev)
    plan.accumulate(_dev(fr, torch_dev), box, 5000.0, 10, 0, h, pair_hist=p)
    assert plan.sync_status() == g3mod.ENOMEM
    assert int(h.sum().item()) == 0
    assert np.array_equal(_np(p), oracle_mod.pair_hist(fr, box, 5000.0, 10))


def test_domain_error_frame_adds_no_pairs(g3mod, plan, torch_dev, oracle_mod):
    w = synth.lj_small("gas", n_frames=3)
    fr = w.frames.copy()
    fr[1, 2, 5] = w.box[2]
    h, p = g3mod.new_hist(w.nbins, 0, torch_dev), g3mod.new_pair_hist(w.nbins, torch_dev)
    plan.accumulate(_dev(fr, torch_dev), w.box, w.rmax, w.nbins, 0, h, pair_hist=p)
    assert plan.sync_status() == g3mod.EDOMAIN
    assert np.array_equal(_np(p), oracle_mod.pair_hist(fr[[0, 2]], w.box, w.rmax, w.nbins))


def test_pair_hist_overlapping_hist_is_rejected(g3mod, plan, torch_dev):
    w = synth.lj_small("gas", n_frames=1)
    h = g3mod.new_hist(w.nbins, 0, torch_dev)
    with pytest.raises(g3mod.G3Error) as e:
        plan.accumulate(_dev(w.frames, torch_dev), w.box, w.rmax, w.nbins, 0, h,
                        pair_hist=h[5:5 + w.nbins])
    assert e.value.status == g3mod.EINVAL
    with pytest.raises(g3mod.G3Error):
        plan.accumulate_batch([dict(frames=_dev(w.frames, torch_dev), box=w.box, rmax=w.rmax,
                                    nbins=w.nbins, layout=0, hist=h, pair_hist=h[:w.nbins])])
    plan.sync()
    assert int(h.sum().item()) == 0


def test_large_system_pairs(g3mod, plan, torch_dev, oracle_mod):
    """N = 65536 (the large-system workload), frames 0 and 37 batched with
    the pair output on: both histograms equal the oracle."""
    w = synth.lj_large(n_frames=50)
    fr = w.frames[[0, 37]]
    ((h, p),) = batch_pairs(g3mod, plan, torch_dev, [(fr, w.box, w.rmax, w.nbins, w.layout)])
    assert np.array_equal(p, oracle_mod.pair_hist(fr, w.box, w.rmax, w.nbins))
    assert np.array_equal(h, oracle_mod.hist(fr, w.box, w.rmax, w.nbins, w.layout))


def test_superposition_chain_matches_oracle(g3mod, plan, torch_dev, oracle_mod):
    """Histograms from the GPU, normalised and turned into the superposition
    ratio and an isosceles slice by the library, equal the same chain run on
    the oracle's histograms with the oracle's definitions."""
    w = synth.lj_small("fcc", n_frames=4)
    h, p = plain_pairs(g3mod, plan, torch_dev, w.frames, w.box, w.rmax, w.nbins, 1)
    F, N, nb = w.frames.shape[0], w.frames.shape[2], w.nbins
    g3v = g3mod.normalize(h, 1, nb, w.rmax, F, N, w.box)
    g2v = g3mod.normalize_pairs(p, nb, w.rmax, F, N, w.box)
    got = g3mod.superposition(g3v, 1, nb, g2v).reshape(nb, nb, nb)
    Ho = oracle_mod.hist(w.frames, w.box, w.rmax, nb, 1)
    Po = oracle_mod.pair_hist(w.frames, w.box, w.rmax, nb)
    g3o = oracle_mod.normalize(Ho, 1, nb, w.rmax, F, N, w.box).reshape(nb, nb, nb)
    g2o = oracle_mod.normalize_pairs(Po, nb, w.rmax, F, N, w.box)
    want = oracle_mod.superposition_full(g3o, g2o)
    assert np.allclose(got, want, rtol=1e-10, atol=0)
    a = 20
    th, val = g3mod.isosceles(g3v, 1, nb, a)
    assert np.allclose(val, g3o[a, a, :], rtol=1e-10, atol=0)
    assert np.allclose(th, [oracle_mod.isosceles_angle(a, c) for c in range(nb)], rtol=1e-12)
