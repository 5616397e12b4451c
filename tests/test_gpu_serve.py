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


def _dense_cluster_frames(n_frames, seed):
    """Half the atoms in a small cluster far above the uniform-density
    neighbour estimate: the batched neighbour pool overflows and the library
    recomputes such a frame in g3_sync."""
    rng = np.random.default_rng(seed)
    box = [200000] * 3
    N = 1200
    out = []
    for _ in range(n_frames):
        pos = np.stack([rng.integers(0, L, size=N) for L in box])
        c = np.array(box) // 2
        pos[:, :600] = c[:, None] + rng.integers(-900, 900, size=(3, 600))
        out.append(pos)
    return np.stack(out).astype(np.int32), box


def test_flagged_request_in_the_mix(torch_dev, oracle_mod):
    """A request whose frames must be recomputed (pool overflow) served among
    ordinary ones: it completes only after g3_sync has added its recomputed
    frames, and every request -- flagged or not -- equals the oracle."""
    store = serve.TrajectoryStore(n_systems=3, max_frames=4, n_min=500, n_max=2000, seed=(12, 3))
    g = np.random.Generator(np.random.PCG64(8))
    reqs = [store.request(r, g, arrival=0.0) for r in range(8)]
    fr, box = _dense_cluster_frames(3, 4)
    dense = serve.Request(100, fr, box, 2500.0, 20, 0, arrival=0.0)
    mix = reqs[:3] + [dense] + reqs[3:]
    srv = serve.Server(hbm_budget_bytes=1 << 30, frames_per_iter=2)
    stats = srv.run_open_loop(mix)
    assert stats["requests"] == len(mix) and srv.used == 0
    assert srv.syncs >= 1                 # the dense request went through g3_sync
    for r in mix:
        want = oracle_mod.hist(r.frames, r.box, r.rmax, r.nbins, r.layout)
        assert np.array_equal(r.result, want), r.rid
