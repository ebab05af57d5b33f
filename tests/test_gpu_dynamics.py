"""Backward-Euler dynamics on the GPU against the oracle: the Schur complement
with the inertia diagonal, Alg. 1 over several time steps with spheres
pressed in (target and velocity advanced by the library), a rigid
translation reproduced exactly, linear momentum conserved without supports,
and the call-order checks."""
import numpy as np
import pytest

import pd_inputs as P
from gpu_util import dev, host
from oracle import pd as opd

pytestmark = pytest.mark.gpu

RHO = 1000.0
DT = 1.0 / 30.0


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _runner(sc, **kw):
    from paper_2008_01541_amd.driver import Alg1Runner
    return Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, sc.proxies, sc.k_pen,
                      density=RHO, dt=DT, **kw)


@pytest.mark.parametrize("name", ["g9x7x6", "g16x15x8"])
def test_schur_with_inertia_matches_oracle(torch_cuda, name):
    from gpu_util import SMALL_SCENES
    sc = SMALL_SCENES[name]()
    om = opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region, density=RHO, dt=DT)
    run = _runner(sc)
    S = torch_cuda.empty(run.ctx.m ** 2, dtype=torch_cuda.float64, device="cuda")
    run.ctx.get_schur(S)
    Sg = host(S, (run.ctx.m, run.ctx.m)).T
    So = om.schur()
    assert np.abs(Sg - So).max() <= 1e-10 * np.abs(So).max()
    run.close()


def test_alg1_backward_euler_matches_oracle(torch_cuda):
    """Spheres pressed into a 16 x 15 x 8 slab over four time steps of 1/30,
    three outer iterations of two inner ones per step, the library advancing
    velocity and inertial target after each step."""
    sc = P.scene_small(16, 15, 8, h=1.0, region_top_layers=2, seed=5, n_spheres=3,
                       depth_frac=0.05)
    om = opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region, density=RHO, dt=DT)
    run = _runner(sc)
    x_or = sc.rest.copy()
    y_or = sc.rest.copy()
    worst, active = 0.0, 0
    for step in range(1, 5):
        cen, rad = sc.spheres.centers(step), sc.spheres.radii
        run.set_spheres(cen, rad)
        det = opd.sphere_detector(om, sc.proxy_local(), cen, rad, sc.k_pen)
        x0 = x_or.copy()
        for _ in range(3):
            run.outer_iteration(n_inner=2)
            x_or = opd.alg1_outer_iteration(om, x_or, det, n_inner=2, y=y_or)
            active = max(active, int((host(run.c) > 0).sum()))
            scale = np.abs(x_or - sc.rest).max()
            worst = max(worst, np.abs(run.positions() - x_or).max() / scale)
        run.advance_time_step()
        v_or, y_or = opd.backward_euler_advance(x_or, x0, DT)
        assert np.abs(host(run.v, (3, -1)) - v_or).max() <= 1e-7 * max(np.abs(v_or).max(), 1e-30)
        assert np.abs(host(run.y, (3, -1)) - y_or).max() <= 1e-9 * scale
    assert active > 0
    assert worst <= 1e-9
    run.close()


def _free_scene():
    sc = P.scene_small(6, 5, 4, h=1.0, region_top_layers=2, seed=7)
    sc.dirichlet = np.zeros(sc.n_nodes, dtype=bool)
    return sc


def test_rigid_translation_and_momentum(torch_cuda):
    """No supports, no contact: a translated body moving uniformly lands on
    x_n + dt u after one iteration; a deformed body with random velocities
    keeps sum m x = sum m y after every iteration (masses from the oracle)."""
    sc = _free_scene()
    sc.proxies = np.zeros(0, np.int64)
    om = opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region, density=RHO, dt=DT)
    run = _runner(sc)
    run.set_spheres(np.zeros((3, 0)), np.zeros(0))
    c = np.array([[0.3], [-0.2], [0.1]])
    u = np.array([[1.5], [0.5], [-2.0]])
    run.set_state(sc.rest + c, np.broadcast_to(u, sc.rest.shape))
    run.outer_iteration(n_inner=2)
    assert np.abs(run.positions() - (sc.rest + c + DT * u)).max() <= 1e-12
    rng = np.random.default_rng(2)
    Z = sc.rest[2] / sc.rest[2].max()
    xn = sc.rest + 0.2 * np.vstack([np.sin(2 * Z), np.cos(3 * Z) - 1, Z ** 2])
    v = rng.normal(size=sc.rest.shape)
    run.set_state(xn, v)
    y = xn + DT * v
    mass = om.D * DT * DT
    p_ref = (mass[None, :] * y).sum(axis=1)
    for _ in range(3):
        run.outer_iteration(n_inner=2)
        x = run.positions()
        p = (mass[None, :] * x).sum(axis=1)
        assert np.abs(p - p_ref).max() <= 1e-10 * np.abs(mass[None, :] * x).sum()
    assert np.abs(run.positions() - xn).max() > 1e-3
    run.close()


def test_call_order_and_arguments(torch_cuda):
    from gpu_util import SMALL_SCENES, gpu_context
    from paper_2008_01541_amd import PDContext, PDError
    sc = SMALL_SCENES["g4x3x5"]()
    ctx = PDContext(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, density=RHO, dt=DT)
    x = dev(sc.rest)
    f = torch_cuda.empty_like(x)
    with pytest.raises(PDError):               # no inertial target yet
        ctx.local_step_full(x, f)
    y = x.clone()                              # kept alive: the context holds its pointer
    ctx.set_inertia_target(y)
    ctx.local_step_full(x, f)
    assert np.abs(host(f)).max() <= 1e-9       # rest state at rest: no force
    qs = gpu_context(sc)
    with pytest.raises(PDError):               # quasistatic: no target, no time step
        qs.set_inertia_target(x)
    with pytest.raises(PDError):
        qs.time_step_advance(x, x.clone(), x.clone(), x.clone())
    for bad in [dict(density=RHO, dt=-1.0), dict(density=0.0, dt=DT),
                dict(density=float("nan"), dt=DT)]:
        with pytest.raises(PDError):
            PDContext(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, **bad)
    ctx.close()
    qs.close()
