"""Checks at the full 56 x 56 x 32 (602,112-tet, 6,498-node region) size that
the oracle can afford: closed forms of S, sampled Schur probes through one
sparse factorization, and a sampled solve."""
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


def test_slab_schur_probes_match_oracle(slab):
    """S v against K22 v - K21 K11^-1 K12 v for seeded random v (one sparse
    factorization of K11 by the oracle)."""
    import torch
    from oracle import pd as opd, schur as osch
    sc, ctx, S = slab
    om = opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region, build_schur=False)
    rng = np.random.default_rng(12)
    Sm = S.reshape(ctx.m, ctx.m)
    for _ in range(4):
        v = rng.normal(size=ctx.m)
        ref = osch.schur_apply(om.lu11, om.A12, om.A21, om.A22, v)
        got = host(Sm @ torch.tensor(v, device="cuda"))
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
