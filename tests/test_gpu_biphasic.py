"""The biphasic strain-limiting material (Sec. 5.3) on the GPU against the
oracle: local steps with the clamped-SVD projection (forces on E_alpha and
E_beta, FP64 and FP32 rotations), the Schur complement with mu + mu', and
Alg. 1 iterations with spheres pressed in far enough to engage the limit."""
import numpy as np
import pytest

import pd_inputs as P
from gpu_util import dev, host
from oracle import fem, pd as opd

pytestmark = pytest.mark.gpu

SMIN, SMAX = 0.95, 1.05


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _pair(sc):
    from paper_2008_01541_amd.driver import Alg1Runner
    kw = dict(mu_prime=10 * sc.mu, sigma_min=SMIN, sigma_max=SMAX)
    om = opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region, **kw)
    run = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, sc.proxies, sc.k_pen, **kw)
    return om, run


def test_local_steps_biphasic_match_oracle(torch_cuda):
    sc = P.scene_small(16, 15, 8, h=1.0, region_top_layers=2, seed=5)
    om, run = _pair(sc)
    ctx = run.ctx
    rng = np.random.default_rng(3)
    x = sc.rest + 0.12 * rng.normal(size=sc.rest.shape)
    x[:, sc.dirichlet] = sc.rest[:, sc.dirichlet]
    F = fem.deformation_gradients(x, sc.tets, om.B)
    sv = np.linalg.svd(F, compute_uv=False)
    assert ((sv < SMIN) | (sv > SMAX)).any(axis=1).mean() > 0.5      # limit engaged
    f = torch_cuda.empty(3 * sc.n_nodes, dtype=torch_cuda.float64, device="cuda")
    ctx.local_step_full(dev(x), f)
    f_or = om.forces(x, om.rotations(x, om.alpha), om.alpha, om.projections(x, om.alpha))
    assert np.abs(host(f, (3, -1)) - f_or).max() <= 1e-10 * np.abs(f_or).max()
    x2 = x[:, om.i2]
    fb = torch_cuda.empty(3 * ctx.m, dtype=torch_cuda.float64, device="cuda")
    fb_or = om.forces(x, om.rotations(x, om.beta), om.beta, om.projections(x, om.beta))[:, om.i2]
    ctx.local_step_region(dev(x2), fb)
    assert np.abs(host(fb, (3, -1)) - fb_or).max() <= 1e-10 * np.abs(fb_or).max()
    ctx.local_step_region(dev(x2), fb, rot_fp32=True)
    assert np.abs(host(fb, (3, -1)) - fb_or).max() <= 1e-5 * np.abs(fb_or).max()
    run.close()


def test_schur_biphasic_matches_oracle(torch_cuda):
    sc = P.scene_small(9, 7, 6, h=0.5, region_top_layers=2, seed=4)
    om, run = _pair(sc)
    m = run.ctx.m
    S = torch_cuda.empty(m * m, dtype=torch_cuda.float64, device="cuda")
    run.ctx.get_schur(S)
    So = om.schur()
    assert np.abs(host(S, (m, m)).T - So).max() <= 1e-10 * np.abs(So).max()
    run.close()


def test_alg1_biphasic_matches_oracle(torch_cuda):
    sc = P.scene_small(16, 15, 8, h=1.0, region_top_layers=2, seed=5, n_spheres=3,
                       depth_frac=0.12)
    om, run = _pair(sc)
    x_or = sc.rest.copy()
    worst, clamped = 0.0, 0
    for step in range(1, 4):
        cen, rad = sc.spheres.centers(step), sc.spheres.radii
        run.set_spheres(cen, rad)
        det = opd.sphere_detector(om, sc.proxy_local(), cen, rad, sc.k_pen)
        for _ in range(2):
            run.outer_iteration(n_inner=2)
            x_or = opd.alg1_outer_iteration(om, x_or, det, n_inner=2)
            scale = np.abs(x_or - sc.rest).max()
            worst = max(worst, np.abs(run.positions() - x_or).max() / scale)
        F = fem.deformation_gradients(x_or, sc.tets, om.B)
        sv = np.linalg.svd(F, compute_uv=False)
        clamped = max(clamped, int(((sv < SMIN) | (sv > SMAX)).any(axis=1).sum()))
    assert clamped > 20
    assert worst <= 1e-9
    run.close()
