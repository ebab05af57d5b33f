"""The nested-dissection interior factor (interior_order = 1) on the GPU
against the CPU FP64 oracle (sparse LU of A11), element by element: the
Schur complement with and without inertia, both condensation sweeps, the
warm-start response, and Alg. 1 iterations, on grid slabs and on jittered
meshes with a cap-shaped region (uneven breadth-first levels), with leaf
sizes that give single-tile, multi-tile and ragged fronts."""
import numpy as np
import pytest

import pd_inputs as P
from gpu_util import SMALL_SCENES, dev, gpu_context, host, oracle_model, rel
from oracle import pd as opd, schur as osch

pytestmark = pytest.mark.gpu
TOL = 1e-10

SCENES = dict(SMALL_SCENES)
SCENES["irregular"] = lambda: P.scene_irregular()
SCENES["irregular_large"] = lambda: P.scene_irregular(20, 18, 12, seed=3)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.mark.parametrize("name,leaf", [("cube8", 0), ("cube8", 16), ("g4x3x5", 4),
                                       ("g9x7x6", 0), ("g16x15x8", 0), ("g16x15x8", 70),
                                       ("g3x3x3_allregion", 0), ("irregular", 0),
                                       ("irregular", 9), ("irregular_large", 0),
                                       ("irregular_large", 100)])
def test_nd_schur_matches_oracle(torch_cuda, name, leaf):
    sc = SCENES[name]()
    om = oracle_model(sc)
    ctx = gpu_context(sc, interior="nd", nd_leaf=leaf)
    assert ctx.m == om.m and ctx.n1 == om.i1.size
    assert np.array_equal(ctx.region_ids, om.i2)
    S = torch_cuda.empty(ctx.m * ctx.m, dtype=torch_cuda.float64, device="cuda")
    ctx.get_schur(S)
    Sg = host(S, (ctx.m, ctx.m)).T
    So = om.schur()
    assert rel(Sg, So) <= TOL
    assert np.abs(Sg - Sg.T).max() <= 1e-12 * np.abs(So).max()


@pytest.mark.parametrize("name,leaf", [("cube8", 0), ("g4x3x5", 4), ("g16x15x8", 0),
                                       ("g16x15x8", 70), ("irregular", 9),
                                       ("irregular_large", 0)])
def test_nd_condense_and_backsub_match_oracle(torch_cuda, name, leaf):
    sc = SCENES[name]()
    om = oracle_model(sc, build_schur=False)
    ctx = gpu_context(sc, interior="nd", nd_leaf=leaf)
    rng = np.random.default_rng(5)
    f = rng.normal(size=(3, sc.n_nodes))
    y2 = torch_cuda.empty(3 * ctx.m, dtype=torch_cuda.float64, device="cuda")
    ctx.condense_rhs(dev(f), y2)
    w1, y2_or = osch.forward_sub(om.lu11, om.A21, f[:, om.i1].T, f[:, om.i2].T)
    assert rel(host(y2, (3, -1)), y2_or.T) <= TOL
    d2 = rng.normal(size=(3, ctx.m))
    x0 = rng.normal(size=(3, sc.n_nodes))
    xd = dev(x0)
    ctx.backsub(dev(d2), xd)
    x_or = x0.copy()
    x_or[:, om.i1] += osch.back_sub(om.lu11, om.A12, f[:, om.i1].T, d2.T).T
    x_or[:, om.i2] += d2
    got = host(xd, (3, -1))
    assert rel(got, x_or) <= TOL
    assert np.array_equal(got[:, sc.dirichlet], x0[:, sc.dirichlet])
    # the sweeps run in a fixed order: a repeat is bit for bit the same
    y2b = torch_cuda.empty_like(y2)
    ctx.condense_rhs(dev(f), y2b)
    assert torch_cuda.equal(y2, y2b)


@pytest.mark.parametrize("name", ["g16x15x8", "irregular"])
def test_nd_warmstart_apply_matches_oracle(torch_cuda, name):
    sc = SCENES[name]()
    om = oracle_model(sc, build_schur=False)
    ctx = gpu_context(sc, interior="nd")
    rng = np.random.default_rng(8)
    # a condensation first, so the right-hand sides the sweeps keep are not zero
    ctx.condense_rhs(dev(rng.normal(size=(3, sc.n_nodes))),
                     torch_cuda.empty(3 * ctx.m, dtype=torch_cuda.float64, device="cuda"))
    d32 = rng.normal(size=(3, ctx.m)).astype(np.float32)
    scale = 0.37
    x0 = sc.rest + 0.01 * rng.normal(size=sc.rest.shape)
    xd = dev(x0)
    ctx.warmstart_apply(dev(d32), scale, xd)
    d = scale * d32.astype(np.float64)
    x1 = osch.back_sub(om.lu11, om.A12, np.zeros((om.i1.size, 3)), d.T).T
    got = host(xd, (3, -1))
    assert np.abs(got[:, om.i2] - (x0[:, om.i2] + d)).max() <= 1e-14
    assert np.abs(got[:, om.i1] - (x0[:, om.i1] + x1)).max() <= 1e-10 * np.abs(x1).max()


@pytest.mark.parametrize("name", ["g9x7x6", "irregular"])
def test_nd_schur_with_inertia_matches_oracle(torch_cuda, name):
    from paper_2008_01541_amd import PDContext
    sc = SCENES[name]()
    rho, dt = 1000.0, 1.0 / 30.0
    om = opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region, density=rho, dt=dt)
    ctx = PDContext(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, density=rho, dt=dt,
                    interior="nd")
    S = torch_cuda.empty(ctx.m * ctx.m, dtype=torch_cuda.float64, device="cuda")
    ctx.get_schur(S)
    So = om.schur()
    assert rel(host(S, (ctx.m, ctx.m)).T, So) <= TOL


@pytest.mark.parametrize("name,inner", [("g16x15x8", 2), ("irregular", 1)])
def test_nd_alg1_iterations_match_oracle(torch_cuda, name, inner):
    from paper_2008_01541_amd.driver import Alg1Runner
    sc = SCENES[name]()
    om = oracle_model(sc)
    run = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, sc.proxies, sc.k_pen,
                     interior="nd")
    x_or = sc.rest.copy()
    worst = 0.0
    for s in range(1, 3):
        cen, rad = sc.spheres.centers(s), sc.spheres.radii
        run.set_spheres(cen, rad)
        det = opd.sphere_detector(om, sc.proxy_local(), cen, rad, sc.k_pen)
        for it in range(3):
            run.outer_iteration(n_inner=inner)
            x_or = opd.alg1_outer_iteration(om, x_or, det, n_inner=inner)
            disp = np.abs(x_or - sc.rest).max()
            worst = max(worst, np.abs(run.positions() - x_or).max() / max(disp, 1e-300))
    run.close()
    assert np.abs(x_or - sc.rest).max() > 1e-6 * sc.h
    assert worst <= 1e-9


def test_nd_rejects_bad_options(torch_cuda):
    from paper_2008_01541_amd import PDContext, PDError
    sc = SCENES["cube8"]()
    with pytest.raises(ValueError):
        PDContext(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, interior="amd")
    with pytest.raises(PDError):
        PDContext(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, interior="nd", nd_leaf=-1)
    with pytest.raises(PDError):
        PDContext(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, interior="nd",
                  nd_leaf=10000)


def test_nd_slit_alg1_matches_oracle(torch_cuda):
    """Self-contact of a slit (region in the middle of the mesh, interior on
    both sides, both faces prescribed) with the nested-dissection factor:
    Alg. 1 step by step against the oracle, on one stream and pipelined."""
    from paper_2008_01541_amd.driver import Alg1Runner
    from oracle import collision as ocol
    torch = torch_cuda
    sc = P.scene_slit(10, 10, 8, 4, 6, seed=5, steps=6)
    om = opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region)
    pl = sc.pairs_local()
    det = lambda x2: ocol.detect_pairs(x2, pl, sc.k_pen)
    run = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, np.zeros(0, np.int64),
                     sc.k_pen, interior="nd", nd_leaf=20)
    run.use_pairs(sc.pairs)
    x_or = sc.rest.copy()
    worst, active = 0.0, 0
    for step in range(1, 5):
        x_or = sc.prescribed(x_or, step)
        run.set_positions(sc.prescribed(run.positions(), step))
        for _ in range(2):
            run.outer_iteration(n_inner=2)
            x_or = opd.alg1_outer_iteration(om, x_or, det, n_inner=2)
            active = max(active, int((host(run.c) > 0).sum()))
            worst = max(worst, np.abs(run.positions() - x_or).max() /
                        np.abs(x_or - sc.rest).max())
    run.close()
    assert active > 0 and worst <= 1e-9
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        run = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, np.zeros(0, np.int64),
                         sc.k_pen, interior="nd")
        run.use_pairs(sc.pairs)
        steps = [1 + k // 2 for k in range(8)]
        bottom = torch.tensor(sc.bottom, device="cuda").long()
        poses = [torch.tensor(sc.prescribed(sc.rest, st)[:, sc.bottom], device="cuda")
                 for st in steps]

        def before_local(k):
            run.x.view(3, -1)[:, bottom] = poses[k]

        run.run_pipelined(8, n_workgroups=8, factor_stream=torch.cuda.Stream(),
                          before_local=before_local)
    torch.cuda.synchronize()
    x_or = sc.rest.copy()
    for st in steps:
        x_or = sc.prescribed(x_or, st)
        x_or = opd.alg1_outer_iteration(om, x_or, det, n_inner=1)
    assert np.abs(run.positions() - x_or).max() / np.abs(x_or - sc.rest).max() <= 1e-9
    run.close()


def test_nd_build_and_sweeps_bitwise_reproducible(torch_cuda):
    """Two builds of one mesh give the same S bit for bit, and their sweeps the
    same y2 and x (fixed summation orders throughout)."""
    sc = SCENES["irregular_large"]()
    rng = np.random.default_rng(17)
    f = dev(rng.normal(size=(3, sc.n_nodes)))
    d2 = None
    outs = []
    for _ in range(2):
        ctx = gpu_context(sc, interior="nd", nd_leaf=64)
        S = torch_cuda.empty(ctx.m * ctx.m, dtype=torch_cuda.float64, device="cuda")
        ctx.get_schur(S)
        y2 = torch_cuda.empty(3 * ctx.m, dtype=torch_cuda.float64, device="cuda")
        ctx.condense_rhs(f, y2)
        if d2 is None:
            d2 = dev(rng.normal(size=(3, ctx.m)))
        x = torch_cuda.zeros(3 * sc.n_nodes, dtype=torch_cuda.float64, device="cuda")
        ctx.backsub(d2, x)
        torch_cuda.cuda.synchronize()
        outs.append((S.clone(), y2.clone(), x.clone()))
        ctx.close()
    for a, b in zip(*outs):
        assert torch_cuda.equal(a, b)


def test_two_bodies_one_without_region(torch_cuda):
    """Two disjoint grids, each pinned at its bottom, the region on the top of
    the first only: the second body's interior never couples to the region
    (breadth-first levels: the unreachable level; nested dissection: roots
    whose boundary is empty).  S and both sweeps against the oracle, for both
    interior factors."""
    from gpu_util import rel as _rel
    from pd_inputs import kuhn_grid, layer_mask, lame_mu
    nx, ny, nz = 6, 5, 4
    r1, t1 = kuhn_grid(nx, ny, nz, 1.0)
    r2, t2 = kuhn_grid(nx, ny, nz, 1.0)
    n1 = r1.shape[1]
    r2 = r2 + np.array([[nx + 3.0], [0.0], [0.0]])
    rest = np.concatenate([r1, r2], axis=1)
    tets = np.concatenate([t1, t2 + n1], axis=1).astype(np.int32)
    bottom = layer_mask(nx, ny, nz, [0])
    dirichlet = np.concatenate([bottom, bottom])
    region = np.concatenate([layer_mask(nx, ny, nz, [nz - 1, nz]), np.zeros(n1, bool)])
    mu = lame_mu()
    om = opd.PDModel(rest, tets, mu, dirichlet, region)
    rng = np.random.default_rng(3)
    f = rng.normal(size=(3, rest.shape[1]))
    d2 = rng.normal(size=(3, om.m))
    w1, y2_or = osch.forward_sub(om.lu11, om.A21, f[:, om.i1].T, f[:, om.i2].T)
    x1_or = osch.back_sub(om.lu11, om.A12, f[:, om.i1].T, d2.T).T
    from paper_2008_01541_amd import PDContext
    for interior, leaf in [("levels", 0), ("nd", 0), ("nd", 8)]:
        ctx = PDContext(rest, tets, region, dirichlet, mu, interior=interior, nd_leaf=leaf)
        S = torch_cuda.empty(ctx.m * ctx.m, dtype=torch_cuda.float64, device="cuda")
        ctx.get_schur(S)
        assert _rel(host(S, (ctx.m, ctx.m)).T, om.schur()) <= TOL, interior
        y2 = torch_cuda.empty(3 * ctx.m, dtype=torch_cuda.float64, device="cuda")
        ctx.condense_rhs(dev(f), y2)
        assert _rel(host(y2, (3, -1)), y2_or.T) <= TOL, interior
        xd = dev(np.zeros_like(f))
        ctx.backsub(dev(d2), xd)
        got = host(xd, (3, -1))
        assert _rel(got[:, om.i1], x1_or) <= TOL, interior
        ctx.close()
