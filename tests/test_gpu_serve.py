"""Serving on the GPU: requests of mixed size, frames and cutoff batched
together give, each, exactly the histogram they give alone."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1708_08619_amd import serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_alone_equals_in_the_mix(torch_dev, oracle_mod):
    import torch
    from paper_1708_08619_amd import g3
    store = serve.TrajectoryStore(n_systems=5, max_frames=6, n_min=600, n_max=6000, seed=(11, 1))
    g = np.random.Generator(np.random.PCG64(5))
    reqs = [store.request(r, g, arrival=0.0005 * r) for r in range(24)]
    fp = [serve.footprint_bytes(r, 2) for r in reqs]
    srv = serve.Server(hbm_budget_bytes=4 * max(fp), frames_per_iter=2)   # forces queueing
    stats = srv.run_open_loop(reqs)
    assert stats["requests"] == 24 and srv.used == 0
    assert srv.peak_used <= 4 * max(fp)
    assert srv.iterations > 1
    with g3.Plan() as plan:
        for r in reqs:
            h = g3.new_hist(r.nbins, r.layout, torch_dev)
            plan.accumulate(torch.from_numpy(np.ascontiguousarray(r.frames)).to(torch_dev), r.box,
                            r.rmax, r.nbins, r.layout, h)
            plan.sync()
            alone = h.cpu().numpy().astype(np.uint64)
            assert np.array_equal(r.result, alone), r.rid
    for r in reqs:
        assert np.array_equal(r.result, oracle_mod.hist(r.frames, r.box, r.rmax, r.nbins, r.layout)), r.rid


def test_flagged_request_in_the_mix(torch_dev, oracle_mod):
    """A request whose frames the library must recompute in g3_sync (2200
    atoms in a 50-unit cube: with 2048-centre items some lists are longer
    than such items allow) served among ordinary ones: it completes only
    after g3_sync has added its recomputed frames, and every request --
    flagged or not -- is exact (the cube by its closed form, every side in
    bin 0: N (N-1) (N-2) / 2 per frame at half bin 0; the others against the
    oracle)."""
    from paper_1708_08619_amd import g3
    store = serve.TrajectoryStore(n_systems=3, max_frames=4, n_min=500, n_max=2000, seed=(12, 3))
    g = np.random.Generator(np.random.PCG64(8))
    reqs = [store.request(r, g, arrival=0.0) for r in range(8)]
    rng = np.random.default_rng(4)
    Nd, Fd = 2200, 2
    dense_fr = (100000 + rng.integers(0, 50, size=(Fd, 3, Nd))).astype(np.int32)
    dense = serve.Request(100, dense_fr, [200000] * 3, 5000.0, 10, 0, arrival=0.0)
    mix = reqs[:3] + [dense] + reqs[3:]
    srv = serve.Server(hbm_budget_bytes=4 << 30, frames_per_iter=2)
    srv.ex.plan.set_tuning(centres_per_item=2048)
    stats = srv.run_open_loop(mix)
    assert stats["requests"] == len(mix) and srv.used == 0
    assert srv.syncs >= 1                 # the dense request went through g3_sync
    want = np.zeros(g3.hist_len(10, 0), np.uint64)
    want[0] = Fd * (Nd * (Nd - 1) * (Nd - 2) // 2)
    assert np.array_equal(dense.result, want)
    for r in reqs:
        want = oracle_mod.hist(r.frames, r.box, r.rmax, r.nbins, r.layout)
        assert np.array_equal(r.result, want), r.rid
