"""Checks at the full 56 x 56 x 32 (602,112-tet, 6,498-node region) size that
the oracle can afford: closed forms of S, Schur probes through one sparse
factorization, the E_alpha local step, both condensation sweeps, and the
refined low-precision solves on a random penalty set (residual recomputed by
the oracle through sparse solves, never from the GPU's S)."""
import numpy as np
import pytest

import pd_inputs as P
from gpu_util import dev, host, gpu_context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slab():
    import torch
    assert torch.cuda.is_available()
    sc = P.scene_slab56()
    ctx = gpu_context(sc)
    S = torch.empty(ctx.m * ctx.m, dtype=torch.float64, device="cuda")
    ctx.get_schur(S)
    return sc, ctx, S


@pytest.fixture(scope="module")
def oracle_slab(slab):
    from oracle import pd as opd
    sc = slab[0]
    return opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region, build_schur=False)


def test_slab_sizes(slab):
    sc, ctx, S = slab
    assert (ctx.m, ctx.n1, ctx.n_beta, ctx.n_levels) == (6498, 97470, 18816, 30)


def test_slab_closed_form_linear_field(slab):
    """v = z/L on the region: v^T S v = 2 mu A / L = 2 mu * 98; clamped to 1:
    2 mu * 3136 / 31 (linear fields are exact for linear tets)."""
    import torch
    sc, ctx, S = slab
    z = sc.rest[2, ctx.region_ids]
    mu = sc.mu
    for v, expect in [(z / 32.0, 2 * mu * 98.0), (np.ones_like(z), 2 * mu * 3136.0 / 31.0)]:
        vd = torch.tensor(v, device="cuda")
        Sm = S.reshape(ctx.m, ctx.m)
        val = float(vd @ (Sm @ vd))
        assert val == pytest.approx(expect, rel=1e-10)


def test_slab_schur_probes_match_oracle(slab, oracle_slab):
    """S v against K22 v - K21 K11^-1 K12 v for seeded random v."""
    import torch
    from oracle import schur as osch
    sc, ctx, S = slab
    om = oracle_slab
    rng = np.random.default_rng(12)
    Sm = S.reshape(ctx.m, ctx.m)
    for _ in range(4):
        v = rng.normal(size=ctx.m)
        ref = osch.schur_apply(om.lu11, om.A12, om.A21, om.A22, v)
        got = host(Sm @ torch.tensor(v, device="cuda"))
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


def test_slab_local_step_full_matches_oracle(slab, oracle_slab):
    import torch
    sc, ctx, S = slab
    om = oracle_slab
    rng = np.random.default_rng(3)
    x = sc.rest + 0.1 * rng.normal(size=sc.rest.shape)
    x[:, sc.dirichlet] = sc.rest[:, sc.dirichlet]
    f = torch.empty(3 * sc.n_nodes, dtype=torch.float64, device="cuda")
    ctx.local_step_full(dev(x), f)
    R = om.rotations(x, om.alpha)
    f_or = om.forces(x, R, om.alpha)
    got = host(f, (3, -1))
    assert np.abs(got - f_or).max() <= 1e-10 * np.abs(f_or).max()


def test_slab_condense_and_backsub_match_oracle(slab, oracle_slab):
    import torch
    from oracle import schur as osch
    sc, ctx, S = slab
    om = oracle_slab
    rng = np.random.default_rng(4)
    f = rng.normal(size=(3, sc.n_nodes))
    y2 = torch.empty(3 * ctx.m, dtype=torch.float64, device="cuda")
    ctx.condense_rhs(dev(f), y2)
    w1, y2_or = osch.forward_sub(om.lu11, om.A21, f[:, om.i1].T, f[:, om.i2].T)
    assert np.abs(host(y2, (3, -1)) - y2_or.T).max() <= 1e-10 * np.abs(y2_or).max()
    d2 = rng.normal(size=(3, ctx.m))
    x0 = np.zeros((3, sc.n_nodes))
    xd = dev(x0)
    ctx.backsub(dev(d2), xd)
    x1_or = osch.back_sub(om.lu11, om.A12, f[:, om.i1].T, d2.T).T
    got = host(xd, (3, -1))
    assert np.abs(got[:, om.i1] - x1_or).max() <= 1e-10 * np.abs(x1_or).max()
    assert np.array_equal(got[:, om.i2], d2)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_slab_refined_solves_random_penalties(slab, oracle_slab, prec):
    """Random penalty set of 1-5 % of the region (k = 1e6, targets below the
    proxies): the FP64, FP32-refined and BF16-refined solves all reach a
    residual <= 1e-8 of (S + P) u = g, with S applied by the oracle."""
    import torch
    from oracle import collision as ocol, schur as osch
    sc, ctx, S = slab
    om = oracle_slab
    m = ctx.m
    rng = np.random.default_rng(300 + prec)
    prox = sc.proxy_local()
    sel, depth = P.random_penalty_set(rng, prox.size, m)
    idx = np.full((sel.size, 8), -1, dtype=np.int32)
    idx[:, 0] = prox[sel]
    w = np.zeros((sel.size, 8)); w[:, 0] = 1.0
    c = np.full(sel.size, 1e6)
    x2 = sc.rest[:, om.i2]
    t = x2[:, prox[sel]].copy()
    t[2] -= depth
    fcol = torch.empty(3 * m, dtype=torch.float64, device="cuda")
    ctx.collision_update(dev(idx), dev(w), dev(c), dev(t), dev(x2), fcol)
    assert np.abs(host(fcol, (3, -1)) - ocol.penalty_force(m, idx, w, c, t, x2)).max() <= 1e-9
    g = rng.normal(size=(3, m))
    u = torch.empty(3 * m, dtype=torch.float64, device="cuda")
    info = ctx.global_solve(dev(g), u, prec=prec, want_info=True)
    assert info["status"] == 0, info
    ug = host(u, (3, -1))
    Pm_u = -ocol.penalty_force(m, idx, w, c, np.zeros_like(t), ug)
    Su = osch.schur_apply(om.lu11, om.A12, om.A21, om.A22, ug.T).T
    r = g - Su - Pm_u
    rel = max(np.linalg.norm(r[v]) / np.linalg.norm(g[v]) for v in range(3))
    assert rel <= (1e-10 if prec == 0 else 1e-8), rel


def _deformed_start(sc):
    """Seeded smooth deformation of the free nodes (zero on the pinned bottom),
    so that every tet has a non-trivial rotation."""
    rng = np.random.default_rng(21)
    X, Y, Z = sc.rest
    amp = rng.uniform(0.05, 0.15, 3)
    ph = rng.uniform(0.0, 2 * np.pi, 3)
    s = (Z / Z.max()) ** 2
    dx = np.vstack([amp[v] * s * np.sin(2 * np.pi * X / 56 + ph[v]) * np.cos(2 * np.pi * Y / 56)
                    for v in range(3)])
    x = sc.rest + dx
    x[:, sc.dirichlet] = sc.rest[:, sc.dirichlet]
    return x


@pytest.fixture(scope="module")
def slab_alg1_reference(oracle_slab):
    """The oracle's plain full-mesh PD iteration from the deformed start with the
    spheres of frame 40 (Alg. 1 with one inner iteration is this iterate)."""
    from oracle import pd as opd
    sc = P.scene_slab56()
    om = oracle_slab
    x0 = _deformed_start(sc)
    cen, rad = sc.spheres.centers(40), sc.spheres.radii
    det = opd.sphere_detector(om, sc.proxy_local(), cen, rad, sc.k_pen)
    n_active = int((det(x0[:, om.i2])[2] > 0).sum())
    return sc, x0, cen, rad, opd.plain_pd_iteration(om, x0, det), n_active


@pytest.mark.parametrize("pipelined", [False, True])
def test_slab_alg1_iteration_matches_oracle(slab, slab_alg1_reference, pipelined):
    """One Alg. 1 outer iteration (one inner) at full size, on one stream and on
    two streams (the benchmark's pipelined schedule, 384 factorization
    workgroups), element-wise against the oracle's full sparse solve."""
    import torch
    from paper_2008_01541_amd.driver import Alg1Runner
    sc, x0, cen, rad, x_or, n_active = slab_alg1_reference
    assert n_active >= 20
    run = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, sc.proxies, sc.k_pen)
    run.set_positions(x0)
    run.set_spheres(cen, rad)
    if pipelined:
        run.run_pipelined(1, n_workgroups=384, factor_stream=torch.cuda.Stream())
    else:
        run.outer_iteration(n_inner=1)
    torch.cuda.synchronize()
    assert int((run.c > 0).sum()) == n_active
    xg = run.positions()
    run.close()
    scale = np.abs(x_or - x0).max()
    assert scale > 0.05
    assert np.abs(xg - x_or).max() <= 1e-9 * scale


@pytest.fixture(scope="module")
def slab_nd():
    """The same slab with the nested-dissection interior factor."""
    import torch
    assert torch.cuda.is_available()
    sc = P.scene_slab56()
    ctx = gpu_context(sc, interior="nd")
    S = torch.empty(ctx.m * ctx.m, dtype=torch.float64, device="cuda")
    ctx.get_schur(S)
    return sc, ctx, S


def test_slab_nd_schur_probes_and_closed_form(slab_nd, oracle_slab):
    import torch
    from oracle import schur as osch
    sc, ctx, S = slab_nd
    assert (ctx.m, ctx.n1) == (6498, 97470) and 1 < ctx.n_levels <= 16
    om = oracle_slab
    Sm = S.reshape(ctx.m, ctx.m)
    rng = np.random.default_rng(12)
    for _ in range(3):
        v = rng.normal(size=ctx.m)
        ref = osch.schur_apply(om.lu11, om.A12, om.A21, om.A22, v)
        got = host(Sm @ torch.tensor(v, device="cuda"))
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
    z = sc.rest[2, ctx.region_ids]
    vd = torch.tensor(z / 32.0, device="cuda")
    assert float(vd @ (Sm @ vd)) == pytest.approx(2 * sc.mu * 98.0, rel=1e-10)


def test_slab_nd_condense_and_backsub_match_oracle(slab_nd, oracle_slab):
    import torch
    from oracle import schur as osch
    sc, ctx, S = slab_nd
    om = oracle_slab
    rng = np.random.default_rng(4)
    f = rng.normal(size=(3, sc.n_nodes))
    y2 = torch.empty(3 * ctx.m, dtype=torch.float64, device="cuda")
    ctx.condense_rhs(dev(f), y2)
    w1, y2_or = osch.forward_sub(om.lu11, om.A21, f[:, om.i1].T, f[:, om.i2].T)
    assert np.abs(host(y2, (3, -1)) - y2_or.T).max() <= 1e-10 * np.abs(y2_or).max()
    d2 = rng.normal(size=(3, ctx.m))
    xd = dev(np.zeros((3, sc.n_nodes)))
    ctx.backsub(dev(d2), xd)
    x1_or = osch.back_sub(om.lu11, om.A12, f[:, om.i1].T, d2.T).T
    got = host(xd, (3, -1))
    assert np.abs(got[:, om.i1] - x1_or).max() <= 1e-10 * np.abs(x1_or).max()
    assert np.array_equal(got[:, om.i2], d2)


def test_slab_nd_alg1_iteration_matches_oracle(slab_alg1_reference):
    """One Alg. 1 outer iteration at full size with the nested-dissection
    interior factor, element-wise against the oracle's full sparse solve."""
    import torch
    from paper_2008_01541_amd.driver import Alg1Runner
    sc, x0, cen, rad, x_or, n_active = slab_alg1_reference
    run = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, sc.proxies, sc.k_pen,
                     interior="nd")
    run.set_positions(x0)
    run.set_spheres(cen, rad)
    run.outer_iteration(n_inner=1)
    torch.cuda.synchronize()
    assert int((run.c > 0).sum()) == n_active
    xg = run.positions()
    run.close()
    scale = np.abs(x_or - x0).max()
    assert np.abs(xg - x_or).max() <= 1e-9 * scale
