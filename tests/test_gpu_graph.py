"""One Algorithm-1 iteration captured into a HIP graph and replayed: every
replay must reproduce the eagerly computed iterate bit for bit, with eager
work and synchronisations between replays."""
import numpy as np
import pytest

import pd_inputs as P

pytestmark = pytest.mark.gpu


def test_graph_replay_matches_eager():
    import torch
    from paper_2008_01541_amd.driver import Alg1Runner
    sc = P.scene_small(16, 15, 8, h=1.0, region_top_layers=2, seed=5, depth_frac=0.05)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        run_e = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, sc.proxies, sc.k_pen)
        run_g = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, sc.proxies, sc.k_pen)
        for r in (run_e, run_g):
            r.set_spheres(sc.spheres.centers(2), sc.spheres.radii)
            r.outer_iteration(n_inner=2)            # allocations happen here, outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        run_g.outer_iteration(n_inner=2)
    torch.cuda.synchronize()
    # the capture did not execute; run_g is still one iteration behind run_e's next step
    for rep in range(4):
        with torch.cuda.stream(s):
            run_e.outer_iteration(n_inner=2)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        xe = run_e.positions()
        xg = run_g.positions()
        assert np.array_equal(xe, xg), f"replay {rep} differs: {np.abs(xe - xg).max()}"
        with torch.cuda.stream(s):                  # unrelated eager work between replays
            _ = torch.ones(1000, device="cuda").sum()
        torch.cuda.synchronize()
