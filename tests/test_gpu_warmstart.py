"""Learned warm start on a small slab: the network is trained on frames the
method generates, then compared with the cold start (previous frame) on a
held-out trajectory.  The plain iteration converged to 1e-9 judges every
warm result (accepted within 1e-6 relative, else charged the cold solve)."""
import numpy as np
import pytest

import pd_inputs as P

pytestmark = pytest.mark.gpu


def test_warm_start_gains_iterations():
    import torch
    from paper_2008_01541_amd.driver import Alg1Runner
    from paper_2008_01541_amd.warmstart import WarmStart, evaluate, generate_trajectory, summarize
    sc = P.scene_small(16, 15, 8, h=1.0, region_top_layers=2, seed=5, n_spheres=3,
                       depth_frac=0.02)
    run = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, sc.proxies, sc.k_pen)
    rng = np.random.default_rng(40)

    def traj(seed):
        r = np.random.default_rng(seed)
        xy = np.vstack([r.uniform(4, 12, 3), r.uniform(4, 11, 3)])
        drift = r.uniform(-0.05, 0.05, size=(2, 3))
        rad = r.uniform(1.0, 2.0, 3)
        depth = r.uniform(0.004, 0.01, 3)
        return (lambda fr: np.vstack([xy + drift * fr, (sc.nz + rad - depth * fr)[None, :]])), rad

    Xs, Ys, cold = [], [], []
    for s in range(3):
        fn, rad = traj(100 + s)
        X, Y, it = generate_trajectory(run, fn, rad, n_frames=24, tol=1e-6)
        Xs.append(X); Ys.append(Y); cold += it
    X = torch.cat(Xs); Y = torch.cat(Ys)
    ws = WarmStart(run.ctx.m, hidden=256, seed=4, max_batch=32)
    hist = ws.train(X, Y, epochs=60, lr=1e-3)
    assert hist[-1] < 0.5 * hist[0]
    fn, rad = traj(999)
    sm_ex = summarize(evaluate(run, ws, fn, rad, n_frames=16, tol=1e-8, judge_tol=1e-9,
                               accept=1e-6, predictor="extrapolate"))
    print("extrapolation:", sm_ex)
    rows = evaluate(run, ws, fn, rad, n_frames=16, tol=1e-8, judge_tol=1e-9, accept=1e-6)
    sm = summarize(rows)
    print("learned:", sm)
    warm = [r for r in rows if "warm_iters" in r]
    assert len(warm) == 14                     # frames 3..16 have two previous frames
    for r in rows:
        assert r["cold_rel_diff"] <= 1e-6           # the run tolerance meets the bound
    for r in warm:
        assert r["fell_back"] == (r["rel_diff"] > 1e-6)
        assert r["charged_iters"] == r["warm_iters"] + (r["cold_iters"] if r["fell_back"] else 0)
    assert sm["fell_back"] <= 2
    # what the trained network gains over the method without it
    assert sm["charged_outer_iters_per_frame"] < sm["cold_outer_iters_per_frame"]
    assert sm["warm_start_err_mean"] < sm["cold_start_err_mean"]
    run.close()
    ws.close()
