"""Pins of the backward-Euler oracle (Sec. 3.2: PD also serves implicit
backward Euler; the step minimises 1/(2 dt^2) ||x - y||_M^2 + E(x) with
y = x_n + dt v_n): lumped masses of the Kuhn grid in closed form, a rigid
translation that one iteration reproduces exactly, linear momentum conserved
by every iteration without supports or contact, the quasistatic limit, the
Schur route against the full solve, Alg. 1 with one inner iteration against
plain PD, and the incremental potential non-increasing under the local and
global steps."""
import numpy as np
import scipy.sparse.linalg as spla

import pd_inputs as P
from oracle import collision as ocol, fem, pd as opd

RHO = 1000.0
DT = 1.0 / 30.0


def _free_scene(nx=5, ny=4, nz=3, seed=3):
    """A grid scene with no Dirichlet node (free flight)."""
    sc = P.scene_small(nx, ny, nz, h=1.0, region_top_layers=2, seed=seed)
    sc.dirichlet = np.zeros(sc.n_nodes, dtype=bool)
    return sc


def _no_contact(m):
    return lambda x2: (np.full((0, 8), -1, np.int32), np.zeros((0, 8)), np.zeros(0),
                       np.zeros((3, 0)))


def _model(sc, **kw):
    return opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region, **kw)


def test_lumped_mass_closed_form():
    """Kuhn grid: a node inside the grid touches 24 tets of volume h^3/6, so
    its lumped mass is rho h^3; all masses add up to rho times the volume."""
    sc = P.scene_small(5, 4, 3, h=0.5, region_top_layers=2, seed=1)
    B, vol = fem.shape_matrices(sc.rest, sc.tets)
    m = fem.lumped_mass(sc.n_nodes, sc.tets, vol, RHO)
    assert abs(m.sum() - RHO * 5 * 4 * 3 * 0.5 ** 3) <= 1e-10 * m.sum()
    X = sc.rest / 0.5
    inner = np.all((X > 0.5) & (X < np.array([[5], [4], [3]]) - 0.5), axis=0)
    assert inner.sum() == 4 * 3 * 2
    assert np.allclose(m[inner], RHO * 0.5 ** 3, rtol=1e-13, atol=0)


def test_rigid_translation_is_reproduced_exactly():
    """Without supports or contact, a body translated by c moving at a uniform
    velocity u lands on y = x_n + dt u after a single iteration (F = I, so the
    elastic force vanishes and K annihilates uniform fields)."""
    sc = _free_scene()
    om = _model(sc, density=RHO, dt=DT)
    c = np.array([[0.3], [-0.2], [0.1]])
    u = np.array([[1.5], [0.5], [-2.0]])
    xn = sc.rest + c
    y = xn + DT * u
    det = _no_contact(om.m)
    for x1 in [opd.plain_pd_iteration(om, xn, det, y=y),
               opd.alg1_outer_iteration(om, xn, det, n_inner=1, y=y),
               opd.alg1_outer_iteration(om, xn, det, n_inner=3, y=y)]:
        assert np.abs(x1 - y).max() <= 1e-12


def test_momentum_conserved_by_every_iteration():
    """Each global step minimises the quadratic model exactly, and elastic
    forces sum to zero per element, so sum_a m_a (x_a - y_a) = 0 after every
    plain or nested iteration (no supports, no contact), whatever the start."""
    sc = _free_scene(6, 5, 4, seed=7)
    om = _model(sc, density=RHO, dt=DT)
    rng = np.random.default_rng(2)
    Z = sc.rest[2] / sc.rest[2].max()
    xn = sc.rest + 0.2 * np.vstack([np.sin(2 * Z), np.cos(3 * Z) - 1, Z ** 2])
    v = rng.normal(size=sc.rest.shape)
    y = xn + DT * v
    mass = om.D * DT * DT
    p_ref = (mass[None, :] * y).sum(axis=1)
    det = _no_contact(om.m)
    for step in [lambda x: opd.plain_pd_iteration(om, x, det, y=y),
                 lambda x: opd.alg1_outer_iteration(om, x, det, n_inner=1, y=y),
                 lambda x: opd.alg1_outer_iteration(om, x, det, n_inner=3, y=y)]:
        x = xn.copy()
        for _ in range(3):
            x = step(x)
            p = (mass[None, :] * x).sum(axis=1)
            assert np.abs(p - p_ref).max() <= 1e-11 * np.abs(mass[None, :] * x).sum()
        assert np.abs(x - xn).max() > 1e-3           # the body did move


def test_large_time_step_reduces_to_quasistatic():
    sc = P.scene_small(5, 4, 4, h=1.0, region_top_layers=2, seed=5, n_spheres=2, depth_frac=0.08)
    qs = _model(sc)
    be = _model(sc, density=RHO, dt=1e7)
    det = opd.sphere_detector(qs, sc.proxy_local(), sc.spheres.centers(3), sc.spheres.radii,
                              sc.k_pen)
    xq = xb = sc.rest.copy()
    for _ in range(3):
        xq = opd.alg1_outer_iteration(qs, xq, det, n_inner=2)
        xb = opd.alg1_outer_iteration(be, xb, det, n_inner=2, y=sc.rest)
    scale = np.abs(xq - sc.rest).max()
    assert scale > 1e-3
    assert np.abs(xb - xq).max() <= 1e-9 * scale


def test_schur_route_with_inertia_equals_full_solve():
    """P1 with the inertia diagonal in the constant matrix."""
    sc = P.scene_small(4, 4, 3, h=1.0, region_top_layers=2, seed=11, n_spheres=2,
                       depth_frac=0.05)
    om = _model(sc, density=RHO, dt=DT)
    det = opd.sphere_detector(om, sc.proxy_local(), sc.spheres.centers(4), sc.spheres.radii * 1.5,
                              1e6)
    pen = det(sc.rest[:, om.i2])
    assert (pen[2] > 0).sum() >= 2
    A, pos = opd.full_matrix_with_penalty(om, pen)
    b = np.random.default_rng(1).normal(size=(3, om.free.size))
    u_full = spla.spsolve(A, b.T).T
    assert np.linalg.norm(opd.three_step_solve(om, b, pen) - u_full) <= 1e-12 * np.linalg.norm(u_full)


def test_alg1_single_inner_equals_plain_pd_with_inertia():
    """P2 under backward Euler: Alg. 1 with one inner iteration is plain PD,
    iterate by iterate, over several time steps."""
    sc = P.scene_small(6, 5, 4, h=1.0, region_top_layers=2, seed=5, n_spheres=2,
                       depth_frac=0.05)
    om = _model(sc, density=RHO, dt=DT)
    xa = xp = sc.rest.copy()
    va = np.zeros_like(xa)
    ya = yp = sc.rest.copy()
    for step in range(1, 4):
        det = opd.sphere_detector(om, sc.proxy_local(), sc.spheres.centers(step),
                                  sc.spheres.radii, sc.k_pen)
        xa0, xp0 = xa.copy(), xp.copy()
        for _ in range(3):
            xa = opd.alg1_outer_iteration(om, xa, det, n_inner=1, y=ya)
            xp = opd.plain_pd_iteration(om, xp, det, y=yp)
            assert np.abs(xa - xp).max() <= 1e-12 * max(1.0, np.abs(xp).max())
        va, ya = opd.backward_euler_advance(xa, xa0, DT)
        _, yp = opd.backward_euler_advance(xp, xp0, DT)
    assert np.abs(va).max() > 0


def test_incremental_potential_non_increasing():
    """With the active set frozen (no contact), the local step lowers the
    incremental potential at fixed x and the global step at fixed R."""
    sc = P.scene_small(6, 5, 4, h=1.0, region_top_layers=2, seed=9)
    om = _model(sc, density=RHO, dt=DT)
    rng = np.random.default_rng(4)
    x = sc.rest + 0.15 * rng.normal(size=sc.rest.shape)
    x[:, sc.dirichlet] = sc.rest[:, sc.dirichlet]
    y = sc.rest + 0.05 * rng.normal(size=sc.rest.shape)
    det = _no_contact(om.m)
    Ra = om.rotations(x, om.alpha)
    Rb = om.rotations(x, om.beta)
    R0a = np.broadcast_to(np.eye(3), Ra.shape).copy()
    R0b = np.broadcast_to(np.eye(3), Rb.shape).copy()
    e_prev = om.energy(x, R0a, R0b, None, y)
    for _ in range(4):
        Ra, Rb = om.rotations(x, om.alpha), om.rotations(x, om.beta)
        e_loc = om.energy(x, Ra, Rb, None, y)
        assert e_loc <= e_prev * (1 + 1e-13)
        x = opd.plain_pd_iteration(om, x, det, y=y)
        e_glob = om.energy(x, Ra, Rb, None, y)
        assert e_glob <= e_loc * (1 + 1e-13)
        e_prev = e_glob
