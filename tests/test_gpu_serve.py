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
    small = sorted(reqs, key=lambda r: r.n_atoms * r.n_frames)[:2]
    for r in small:
        assert np.array_equal(r.result, oracle_mod.hist(r.frames, r.box, r.rmax, r.nbins, r.layout))
