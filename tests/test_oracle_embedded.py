"""Pins of the embedded-proxy and rest-pose level-set oracle (Sec. 3.3 eq.
p_j_v, Sec. 5.1): barycentric embedding by definition, reduction to conforming
proxies, the Schur route with embedded penalty rows against the full solve,
and the level-set spring of a rigidly pushed lip in closed form."""
import numpy as np
import scipy.sparse.linalg as spla

import pd_inputs as P
from oracle import collision as ocol, pd as opd


def _model(sc):
    return opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region)


def _local(sc, ids):
    rid = sc.region_ids()
    pos = np.full(sc.n_nodes, -1, dtype=np.int64)
    pos[rid] = np.arange(rid.size)
    out = pos[ids]
    assert (out >= 0).all()
    return out.astype(np.int32)


def test_embedding_is_the_barycentric_definition():
    sc = P.scene_small(5, 4, 3, region_top_layers=2, seed=3)
    sel = P.region_tets(sc.rest, sc.tets, sc.region, sc.dirichlet)
    T = _local(sc, sc.tets[:, sel])
    rest2 = sc.rest[:, sc.region_ids()]
    pts = P.top_face_proxy_points(sc, 40, seed=1)
    # plus interior points of the top cell layer
    rng = np.random.default_rng(2)
    inner = np.vstack([rng.uniform(0, 5, 20), rng.uniform(0, 4, 20), rng.uniform(2.05, 2.95, 20)])
    pts = np.concatenate([pts, inner], axis=1)
    tet, idx, w = ocol.embed_points(pts, T, rest2)
    assert (tet >= 0).all()
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-14)
    assert (w >= -1e-12).all()
    rec = np.einsum("vjk,jk->vj", rest2[:, idx], w)
    assert np.abs(rec - pts).max() <= 1e-13
    for j in range(pts.shape[1]):      # no tet of lower index contains the point
        for e in range(tet[j]):
            b = ocol.barycentric(pts[:, j], rest2[:, T[:, e]])
            assert b.min() < -1e-12


def test_embedded_proxies_at_nodes_reduce_to_conforming():
    sc = P.scene_small(4, 4, 3, region_top_layers=2, seed=5, n_spheres=2, depth_frac=0.05)
    m = _model(sc)
    sel = P.region_tets(sc.rest, sc.tets, sc.region, sc.dirichlet)
    T = _local(sc, sc.tets[:, sel])
    rest2 = sc.rest[:, m.i2]
    pl = sc.proxy_local()
    tet, eidx, ew = ocol.embed_points(rest2[:, pl], T, rest2)
    # a node is embedded with weight 1 on itself
    for j in range(pl.size):
        k = np.argmax(ew[j])
        assert eidx[j, k] == pl[j] and abs(ew[j, k] - 1.0) <= 1e-14
    rng = np.random.default_rng(7)
    x2 = rest2 + 0.05 * rng.normal(size=rest2.shape)
    cen, rad = sc.spheres.centers(3), sc.spheres.radii
    pe = ocol.embedded_sphere_penalties(x2, eidx, ew, cen, rad, sc.k_pen)
    c, t = ocol.detect_spheres(x2[:, pl], cen, rad, sc.k_pen)
    pc = ocol.conforming_penalties(pl, c, t)
    assert (pe[2] > 0).sum() > 0
    assert np.allclose(ocol.penalty_matrix(m.m, *pe[:3]), ocol.penalty_matrix(m.m, *pc[:3]),
                       rtol=0, atol=1e-8)
    assert np.allclose(ocol.penalty_force(m.m, *pe, x2), ocol.penalty_force(m.m, *pc, x2),
                       rtol=0, atol=1e-6)


def test_schur_route_with_embedded_proxies_equals_full_solve():
    """P1 with general four-weight W rows: the Schur route reproduces the
    direct solve of (K + W^T C W) u = b over all free nodes."""
    sc = P.scene_small(4, 4, 3, region_top_layers=2, seed=11, n_spheres=2, depth_frac=0.05)
    m = _model(sc)
    sel = P.region_tets(sc.rest, sc.tets, sc.region, sc.dirichlet)
    T = _local(sc, sc.tets[:, sel])
    rest2 = sc.rest[:, m.i2]
    pts = P.top_face_proxy_points(sc, 60, seed=4)
    _, eidx, ew = ocol.embed_points(pts, T, rest2)
    cen = sc.spheres.centers(4)
    pen = ocol.embedded_sphere_penalties(rest2, eidx, ew, cen, sc.spheres.radii * 1.5, 1e6)
    assert (pen[2] > 0).sum() >= 3
    A, pos = opd.full_matrix_with_penalty(m, pen)
    b = np.random.default_rng(1).normal(size=(3, m.free.size))
    u_full = spla.spsolve(A, b.T).T
    u_schur = opd.three_step_solve(m, b, pen)
    assert np.linalg.norm(u_schur - u_full) <= 1e-12 * np.linalg.norm(u_full)


def _slit_bodies(nx=10, ny=10, nz=8, zs=4, ys=6):
    sc = P.scene_slit(nx, ny, nz, zs, ys, seed=5, steps=6)
    m = _model(sc)
    bd = P.slit_levelset_bodies(sc, per_cell=1.0, seed=15)
    rest2 = sc.rest[:, m.i2]
    cand = _local(sc, bd.body_tets)
    eidx = np.zeros((bd.proxy_body.size, 4), np.int32)
    ew = np.zeros((bd.proxy_body.size, 4))
    for body in (0, 1):
        sel = np.nonzero(bd.proxy_body == body)[0]
        Tb = cand[:, bd.body_id == body]
        tet, ei, wi = ocol.embed_points(bd.proxy_points[:, sel], Tb, rest2)
        assert (tet >= 0).all()
        eidx[sel], ew[sel] = ei, wi
    return sc, m, bd, rest2, cand, eidx, ew


def test_levelset_at_rest_has_no_contact():
    sc, m, bd, rest2, cand, eidx, ew = _slit_bodies()
    pen = ocol.levelset_penalties(rest2, rest2, eidx, ew, bd.proxy_body, cand, bd.body_phi,
                                  bd.body_id, sc.k_pen)
    assert (pen[2] == 0).all()


def test_levelset_spring_of_a_pushed_lip_in_closed_form():
    """Lower lip lifted rigidly by d (< one cell) into the fixed upper lip: each
    lower proxy away from the slit front is found inside the upper body at rest
    depth d, its target is the upper lip surface point straight above its rest
    position, so W x - t = (0, 0, d); each upper proxy is inside the lifted lower
    body and its target is the lifted lower surface: W x - t = (0, 0, -d)."""
    sc, m, bd, rest2, cand, eidx, ew = _slit_bodies()
    d = 0.3 * sc.h
    lower_nodes = np.unique(cand[:, bd.body_id == 0])
    upper_nodes = np.unique(cand[:, bd.body_id == 1])
    move = np.setdiff1d(lower_nodes, upper_nodes)        # not the shared front line
    x2 = rest2.copy()
    x2[2, move] += d
    pen = ocol.levelset_penalties(x2, rest2, eidx, ew, bd.proxy_body, cand, bd.body_phi,
                                  bd.body_id, sc.k_pen)
    idx, w, c, t = pen
    y = bd.proxy_points[1]
    away = y < (sc.meta_ys_end - 1.5) * sc.h
    assert (c[away] == sc.k_pen).all()
    for j in np.nonzero(away)[0]:
        sl = idx[j] >= 0
        r = x2[:, idx[j][sl]] @ w[j][sl] - t[:, j]
        want = np.array([0.0, 0.0, d if bd.proxy_body[j] == 0 else -d])
        assert np.abs(r - want).max() <= 1e-12, (j, r)
        assert abs(w[j][sl].sum()) <= 1e-12              # proxy minus surface point
    # force and Hessian of the springs are those of eq. E_col_C with these rows
    A, pos = opd.full_matrix_with_penalty(m, pen)
    b = np.random.default_rng(3).normal(size=(3, m.free.size))
    u_full = spla.spsolve(A, b.T).T
    assert np.linalg.norm(opd.three_step_solve(m, b, pen) - u_full) <= 1e-12 * np.linalg.norm(u_full)
