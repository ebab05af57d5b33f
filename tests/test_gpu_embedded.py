"""Embedded collision proxies and rest-pose level-set self-collision on the
GPU (Sec. 3.3 eq. p_j_v; Sec. 5.1) against the oracle: the embedding (tet
index exactly, barycentric weights), sphere detection through four-weight W
rows, the level-set springs (activity and W rows), and Alg. 1 iterations
driven by each detector.  The GPU embeds with its own kernel; the oracle
with its own routine; nothing crosses from one side to the other."""
import numpy as np
import pytest

import pd_inputs as P
from gpu_util import dev, host
from oracle import collision as ocol, pd as opd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _local(sc, ids):
    rid = sc.region_ids()
    pos = np.full(sc.n_nodes, -1, dtype=np.int64)
    pos[rid] = np.arange(rid.size)
    out = pos[ids]
    assert (out >= 0).all()
    return out.astype(np.int32)


def _slab_points(sc, n_face, seed):
    """Embedded proxies on the top face plus points inside the top cell layer."""
    pts = P.top_face_proxy_points(sc, n_face, seed=seed)
    rng = np.random.default_rng(seed + 1)
    k = n_face // 4
    inner = np.vstack([rng.uniform(0, sc.nx * sc.h, k), rng.uniform(0, sc.ny * sc.h, k),
                       rng.uniform((sc.nz - 0.95) * sc.h, (sc.nz - 0.05) * sc.h, k)])
    return np.concatenate([pts, inner], axis=1)


def test_embed_points_matches_oracle(torch_cuda):
    from paper_2008_01541_amd.driver import Alg1Runner
    sc = P.scene_small(16, 15, 8, h=1.0, region_top_layers=2, seed=5)
    run = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, sc.proxies, sc.k_pen)
    T = _local(sc, sc.tets[:, P.region_tets(sc.rest, sc.tets, sc.region, sc.dirichlet)])
    pts = _slab_points(sc, 300, seed=3)
    # plus region nodes themselves (on shared faces, edges and corners)
    rest2 = sc.rest[:, sc.region_ids()]
    pts = np.concatenate([pts, rest2[:, ::7]], axis=1)
    tet, eidx, ew = run.embed(pts, T)
    o_tet, o_idx, o_w = ocol.embed_points(pts, T, rest2)
    assert (o_tet >= 0).all()
    assert np.array_equal(host(tet), o_tet)
    assert np.array_equal(host(eidx, (-1, 4)), o_idx)
    assert np.abs(host(ew, (-1, 4)) - o_w).max() <= 1e-13
    # a point outside every candidate
    out = np.array([[-5.0], [-5.0], [100.0]])
    tet1, eidx1, ew1 = run.embed(out, T)
    assert host(tet1)[0] == -1 and (host(eidx1) == -1).all() and (host(ew1) == 0).all()
    run.close()


def test_detect_embedded_spheres_matches_oracle(torch_cuda):
    from paper_2008_01541_amd.driver import Alg1Runner
    sc = P.scene_small(16, 15, 8, h=1.0, region_top_layers=2, seed=5, n_spheres=3)
    run = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, sc.proxies, sc.k_pen)
    T = _local(sc, sc.tets[:, P.region_tets(sc.rest, sc.tets, sc.region, sc.dirichlet)])
    rest2 = sc.rest[:, sc.region_ids()]
    pts = _slab_points(sc, 400, seed=8)
    _, o_idx, o_w = ocol.embed_points(pts, T, rest2)
    rng = np.random.default_rng(9)
    x2 = rest2 + 0.05 * rng.normal(size=rest2.shape)
    cen, rad = sc.spheres.centers(6), sc.spheres.radii * 2.0
    oi, ow, oc, ot = ocol.embedded_sphere_penalties(x2, o_idx, o_w, cen, rad, sc.k_pen)
    assert (oc > 0).sum() >= 10
    _, eidx, ew = run.embed(pts, T)
    run.use_embedded(eidx, ew)
    run.set_spheres(cen, rad)
    run.x2.copy_(dev(x2))
    run.detect()
    assert np.array_equal(host(run.c), oc)
    assert np.array_equal(host(run.idx, (-1, 8)), oi)
    assert np.abs(host(run.w, (-1, 8)) - ow).max() <= 1e-13
    assert np.abs(host(run.t, (3, -1)) - ot).max() <= 1e-12
    run.close()


def test_alg1_with_embedded_proxies_matches_oracle(torch_cuda):
    """Spheres pressed into the top face of a 16 x 15 x 8 slab, detection
    through 1,200 embedded proxies; Alg. 1 (2 inner iterations) step by step."""
    from paper_2008_01541_amd.driver import Alg1Runner
    sc = P.scene_small(16, 15, 8, h=1.0, region_top_layers=2, seed=5, n_spheres=3,
                       depth_frac=0.05)
    om = opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region)
    run = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, sc.proxies, sc.k_pen)
    T = _local(sc, sc.tets[:, P.region_tets(sc.rest, sc.tets, sc.region, sc.dirichlet)])
    pts = P.top_face_proxy_points(sc, 1200, seed=21)
    _, o_idx, o_w = ocol.embed_points(pts, T, sc.rest[:, om.i2])
    _, eidx, ew = run.embed(pts, T)
    run.use_embedded(eidx, ew)
    x_or = sc.rest.copy()
    worst, active = 0.0, 0
    for step in range(1, 4):
        cen, rad = sc.spheres.centers(step), sc.spheres.radii
        run.set_spheres(cen, rad)
        det = lambda x2: ocol.embedded_sphere_penalties(x2, o_idx, o_w, cen, rad, sc.k_pen)
        for _ in range(2):
            run.outer_iteration(n_inner=2)
            x_or = opd.alg1_outer_iteration(om, x_or, det, n_inner=2)
            active = max(active, int((host(run.c) > 0).sum()))
            scale = np.abs(x_or - sc.rest).max()
            worst = max(worst, np.abs(run.positions() - x_or).max() / scale)
    assert active >= 8
    assert worst <= 1e-9
    run.close()


def _slit_setup(sc, run=None):
    """Lip bodies of the slit, the oracle's embedding per body, and (with a
    runner) the GPU's own embedding per body."""
    bd = P.slit_levelset_bodies(sc, per_cell=1.0, seed=15)
    rid = sc.region_ids()
    rest2 = sc.rest[:, rid]
    cand = _local(sc, bd.body_tets)
    o_idx = np.zeros((bd.proxy_body.size, 4), np.int32)
    o_w = np.zeros((bd.proxy_body.size, 4))
    g_idx = np.zeros_like(o_idx)
    g_w = np.zeros_like(o_w)
    for body in (0, 1):
        sel = np.nonzero(bd.proxy_body == body)[0]
        Tb = cand[:, bd.body_id == body]
        tet, ei, wi = ocol.embed_points(bd.proxy_points[:, sel], Tb, rest2)
        assert (tet >= 0).all()
        o_idx[sel], o_w[sel] = ei, wi
        if run is not None:
            gt, ge, gw = run.embed(bd.proxy_points[:, sel], Tb)
            assert np.array_equal(host(gt), tet)
            g_idx[sel], g_w[sel] = host(ge, (-1, 4)), host(gw, (-1, 4))
    return bd, rest2, cand, o_idx, o_w, g_idx, g_w


def test_detect_levelset_matches_oracle(torch_cuda):
    """A lifted lower lip (every proxy in contact) and a jaw pose with lateral
    noise: activity, W rows and targets against the oracle."""
    from paper_2008_01541_amd.driver import Alg1Runner
    sc = P.scene_slit(10, 10, 8, 4, 6, seed=5, steps=6)
    run = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, np.zeros(0, np.int64),
                     sc.k_pen)
    bd, rest2, cand, o_idx, o_w, g_idx, g_w = _slit_setup(sc, run)
    assert np.array_equal(g_idx, o_idx) and np.abs(g_w - o_w).max() <= 1e-13
    run.use_levelset(dev(g_idx), dev(g_w), bd.proxy_body, cand, bd.body_phi, bd.body_id)
    lower = np.unique(cand[:, bd.body_id == 0])
    upper = np.unique(cand[:, bd.body_id == 1])
    move = np.setdiff1d(lower, upper)
    rng = np.random.default_rng(31)
    states = []
    x2 = rest2.copy()
    x2[2, move] += 0.3 * sc.h
    states.append(x2)
    x2 = rest2.copy()
    x2[2, move] += 0.45 * sc.h
    x2[:2] += 0.05 * rng.normal(size=(2, rest2.shape[1]))
    states.append(x2)
    for x2 in states:
        oi, ow, oc, ot = ocol.levelset_penalties(x2, rest2, o_idx, o_w, bd.proxy_body, cand,
                                                 bd.body_phi, bd.body_id, sc.k_pen)
        assert (oc > 0).sum() >= 20
        run.x2.copy_(dev(x2))
        run.detect()
        assert np.array_equal(host(run.c), oc)
        assert np.array_equal(host(run.idx, (-1, 8)), oi)
        assert np.abs(host(run.w, (-1, 8)) - ow).max() <= 1e-12
        assert (host(run.t) == 0).all()
    run.close()


def test_alg1_with_levelset_self_collision_matches_oracle(torch_cuda):
    """The slit closed by the prescribed jaw rotation, self-contact found by
    the rest-pose level sets of the two lips; Alg. 1 step by step."""
    from paper_2008_01541_amd.driver import Alg1Runner
    sc = P.scene_slit(10, 10, 8, 4, 6, seed=5, steps=6)
    om = opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region)
    run = Alg1Runner(sc.rest, sc.tets, sc.region, sc.dirichlet, sc.mu, np.zeros(0, np.int64),
                     sc.k_pen)
    bd, rest2, cand, o_idx, o_w, g_idx, g_w = _slit_setup(sc, run)
    run.use_levelset(dev(g_idx), dev(g_w), bd.proxy_body, cand, bd.body_phi, bd.body_id)
    det = lambda x2: ocol.levelset_penalties(x2, rest2, o_idx, o_w, bd.proxy_body, cand,
                                             bd.body_phi, bd.body_id, sc.k_pen)
    x_or = sc.rest.copy()
    worst, active = 0.0, 0
    for step in range(2, 7):
        x_or = sc.prescribed(x_or, step)
        run.set_positions(sc.prescribed(run.positions(), step))
        run.outer_iteration(n_inner=2)
        x_or = opd.alg1_outer_iteration(om, x_or, det, n_inner=2)
        active = max(active, int((host(run.c) > 0).sum()))
        scale = np.abs(x_or - sc.rest).max()
        worst = max(worst, np.abs(run.positions() - x_or).max() / scale)
    assert active > 0
    assert worst <= 1e-9
    run.close()
