"""GPU parity at the limits of the arguments: the largest nbins the LDS slabs
take (at most 63 slabs of whole rows per system, the bound the header states
for the default tuning and for 2048 centres per item) bit for bit against the
oracle, one more bin rejected with G3_EINVAL before anything is queued; the
largest and the smallest cutoff (rmax = 46340 and 1 unit); one bin; the
largest number of atoms (2^22, a perfect crystal with a closed-form
histogram)."""
from __future__ import annotations

import numpy as np
import pytest

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


def _gas(seed, N, box, F=2):
    rng = np.random.default_rng(seed)
    return np.stack([np.stack([rng.integers(0, L, size=N) for L in box]) for _ in range(F)]
                    ).astype(np.int32)


def _check(g3, plan, dev, oracle_mod, fr, box, rmax, nb, nc, layout):
    want = oracle_mod.hist(fr, box, rmax, nb, layout, nbins_third=nc)
    h = g3.new_hist(nb, layout, dev, nbins_third=nc)
    plan.accumulate(_dev(fr, dev), box, rmax, nb, layout, h, nbins_third=nc)
    plan.sync()
    assert np.array_equal(_np(h), want), "plain"
    hb = g3.new_hist(nb, layout, dev, nbins_third=nc)
    plan.accumulate_batch([dict(frames=_dev(fr, dev), box=box, rmax=rmax, nbins=nb, layout=layout,
                                hist=hb, nbins_third=nc)])
    plan.sync()
    assert np.array_equal(_np(hb), want), "batched"
    return want


def _rejected(g3, plan, dev, fr, box, rmax, nb, nc):
    h = g3.new_hist(nb, 0, dev, nbins_third=nc)
    with pytest.raises(g3.G3Error) as e:
        plan.accumulate(_dev(fr, dev), box, rmax, nb, 0, h, nbins_third=nc)
    assert e.value.status == g3.EINVAL
    with pytest.raises(g3.G3Error) as e:
        plan.accumulate_batch([dict(frames=_dev(fr, dev), box=box, rmax=rmax, nbins=nb, layout=0,
                                    hist=h, nbins_third=nc)])
    assert e.value.status == g3.EINVAL
    plan.sync()
    assert int(h.sum().item()) == 0


# (centres per item, largest nbins with one cutoff, with a doubled third axis)
_SLAB_LIMITS = [(0, 147, 116), (2048, 139, 110)]


@pytest.mark.parametrize("cb,nb1,nb2", _SLAB_LIMITS, ids=["default", "cb2048"])
@pytest.mark.parametrize("doubled", [False, True], ids=["one_cutoff", "doubled_third"])
def test_largest_nbins(g3mod, plan, torch_dev, oracle_mod, cb, nb1, nb2, doubled):
    if cb:
        plan.set_tuning(centres_per_item=cb)
    box = [40000] * 3
    fr = _gas(500 + cb, 400, box)
    nb = nb2 if doubled else nb1
    nc = 2 * nb if doubled else nb
    rmax = 9000.0 if doubled else 15000.0
    for layout in (0, 1):
        want = _check(g3mod, plan, torch_dev, oracle_mod, fr, box, rmax, nb, nc, layout)
        assert want.sum() > 0
    _rejected(g3mod, plan, torch_dev, fr, box, rmax, nb + 1, 2 * (nb + 1) if doubled else nb + 1)


def test_largest_cutoff(g3mod, plan, torch_dev, oracle_mod):
    """rmax = 46340 units: squared distances up to 2^31 - 1, 32-bit entries."""
    box = [100000, 96000, 120000]
    fr = _gas(610, 500, box)
    for layout in (0, 1):
        want = _check(g3mod, plan, torch_dev, oracle_mod, fr, box, 46340.0, 30, 30, layout)
        assert want.sum() > 0


def test_smallest_cutoff_and_one_bin(g3mod, plan, torch_dev, oracle_mod):
    """rmax = 1 unit: only coincident atoms are neighbours (r = 0); many atoms
    share a handful of sites.  Then the same points with one bin per axis."""
    rng = np.random.default_rng(620)
    box = [1000, 1200, 900]
    sites = np.stack([rng.integers(0, L, size=12) for L in box])
    fr = np.stack([sites[:, rng.integers(0, 12, size=300)] for _ in range(2)]).astype(np.int32)
    for layout in (0, 1):
        want = _check(g3mod, plan, torch_dev, oracle_mod, fr, box, 1.0, 3, 3, layout)
        assert want.sum() > 0
        want = _check(g3mod, plan, torch_dev, oracle_mod, fr, box, 300.0, 1, 1, layout)
        assert want.sum() > 0


def test_perfect_fcc_at_the_atom_limit(g3mod, plan, torch_dev):
    """N = 2^22 atoms, the largest N, as a 128 x 128 x 64 FCC crystal at the
    large-system density and cutoff: every site sees the same neighbour
    vectors, so the expected histogram is N times the lattice-vector count.
    Cell, list and pool offsets reach their largest sizes here."""
    import oracle
    import refs
    a = 6708                                   # ~1.638 sigma at 4096/sigma: rho ~ 0.91
    n = (128, 128, 64)
    box = [a * k for k in n]
    h = a // 2
    basis = np.array([[0, 0, 0], [0, h, h], [h, 0, h], [h, h, 0]], dtype=np.int32)
    g = np.stack(np.meshgrid(*[np.arange(k, dtype=np.int32) * a for k in n], indexing="ij"),
                 -1).reshape(-1, 3)
    sites = (g[:, None, :] + basis[None]).reshape(-1, 3)
    N = len(sites)
    assert N == 1 << 22
    fr = np.ascontiguousarray(sites.T[None])
    del g, sites
    rmax, nb = 3.0 * 4096, 60
    want_full = refs.lattice_full(refs.fcc_vectors(a, rmax), N, rmax, nb)
    want_half, bad = oracle.fold_half(want_full)
    assert bad == 0
    d = _dev(fr, torch_dev)
    for layout, want in ((0, want_half), (1, want_full.reshape(-1))):
        h1 = g3mod.new_hist(nb, layout, torch_dev)
        plan.accumulate(d, box, rmax, nb, layout, h1)
        plan.sync()
        assert np.array_equal(_np(h1), want), f"plain layout {layout}"
        h2 = g3mod.new_hist(nb, layout, torch_dev)
        plan.accumulate_batch([dict(frames=d, box=box, rmax=rmax, nbins=nb, layout=layout, hist=h2)])
        plan.sync()
        assert np.array_equal(_np(h2), want), f"batched layout {layout}"
