"""The self-contact slit at full size (64 x 64 x 40 cells, 983,040 tets, a
12,155-node region on both lips): the region system S + W^T C W with a seeded
set of active lip springs (0.5-3 % of the region, k = 5e5) solved in FP64 and
by the refined FP32 and BF16-operand factors, each residual recomputed by the
oracle through sparse solves with the interior factor (S is never read back
from the GPU)."""
import numpy as np
import pytest

import pd_inputs as P
from gpu_util import dev, host, gpu_context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slit():
    import torch
    assert torch.cuda.is_available()
    from oracle import pd as opd
    sc = P.scene_slit()
    ctx = gpu_context(sc)
    om = opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region, build_schur=False)
    yield sc, ctx, om
    ctx.close()


def _lip_springs(sc, om, seed):
    """Seeded active subset of the lip pairs: W rows [1, -1], target 0, c = k."""
    from oracle import collision as ocol
    rng = np.random.default_rng(seed)
    pl = sc.pairs_local()
    idx, w, _, t = ocol.detect_pairs(sc.rest[:, om.i2], pl, sc.k_pen)
    npair = pl.shape[1]
    frac = rng.uniform(0.005, 0.03)
    on = rng.choice(npair, size=int(frac * om.m), replace=False)
    c = np.zeros(npair)
    c[on] = sc.k_pen
    return idx, w, c, t


def test_slit_sizes(slit):
    sc, ctx, om = slit
    assert ctx.m == om.m == 12155
    assert ctx.n1 == om.i1.size


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_slit_refined_solves(slit, prec):
    """FP64: relative residual <= 1e-10; FP32-IR and BF16-IR (conjugate
    gradients preconditioned by the low-precision factor, FP64 residual):
    <= 1e-8 without falling back to FP64."""
    import torch
    from oracle import collision as ocol, schur as osch
    sc, ctx, om = slit
    m = ctx.m
    idx, w, c, t = _lip_springs(sc, om, 500 + prec)
    x2 = sc.rest[:, om.i2]
    fcol = torch.empty(3 * m, dtype=torch.float64, device="cuda")
    ctx.collision_update(dev(idx), dev(w), dev(c), dev(t), dev(x2), fcol)
    rng = np.random.default_rng(600 + prec)
    g = rng.normal(size=(3, m))
    u = torch.empty(3 * m, dtype=torch.float64, device="cuda")
    info = ctx.global_solve(dev(g), u, prec=prec, want_info=True)
    assert info["status"] == 0 and info["fell_back"] == 0, info
    ug = host(u, (3, -1))
    Pu = -ocol.penalty_force(m, idx, w, c, np.zeros_like(t), ug)
    Su = osch.schur_apply(om.lu11, om.A12, om.A21, om.A22, ug.T).T
    r = g - Su - Pu
    rel = max(np.linalg.norm(r[v]) / np.linalg.norm(g[v]) for v in range(3))
    assert rel <= (1e-10 if prec == 0 else 1e-8), rel
    assert info["rel_residual"] == pytest.approx(rel, rel=0.05, abs=1e-13)


def test_slit_nd_schur_probes_and_sweeps(slit):
    """The nested-dissection interior factor on the full slit (interior on
    both sides of the region): S v against the oracle's K22 v - K21 K11^-1 K12 v
    for seeded v, and both condensation sweeps against its sparse solves."""
    import torch
    from oracle import schur as osch
    sc, _, om = slit
    ctx = gpu_context(sc, interior="nd")
    try:
        assert ctx.m == om.m and ctx.n1 == om.i1.size
        S = torch.empty(ctx.m * ctx.m, dtype=torch.float64, device="cuda")
        ctx.get_schur(S)
        Sm = S.reshape(ctx.m, ctx.m)
        rng = np.random.default_rng(31)
        for _ in range(2):
            v = rng.normal(size=ctx.m)
            ref = osch.schur_apply(om.lu11, om.A12, om.A21, om.A22, v)
            got = host(Sm @ torch.tensor(v, device="cuda"))
            assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
        del S, Sm
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
    finally:
        ctx.close()
