"""Pins of the biphasic strain-limiting material in the oracle (Sec. 5.3):
energy density mu' ||F - Q||^2 + mu ||F - R||^2 with Q the closest matrix
whose singular values lie in [sigma_min, sigma_max].  The projection against
its definition (membership, identity inside the band, diagonal closed form,
optimality against random members of the band), forces as minus the
gradient of the minimised energy (finite differences), mu' = 0 reducing to
the corotated model, the Schur route against the full solve, Alg. 1 with one
inner iteration against plain PD, and the local/global steps lowering the
energy."""
import numpy as np
import scipy.sparse.linalg as spla

import pd_inputs as P
from oracle import collision as ocol, fem, pd as opd

SMIN, SMAX = 0.95, 1.05


def _rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.diag(r))


def test_projection_against_its_definition():
    rng = np.random.default_rng(1)
    F = rng.normal(size=(200, 3, 3)) * 0.4 + np.eye(3)
    Q = fem.clamped_projection(F, SMIN, SMAX)
    s = np.linalg.svd(Q, compute_uv=False)
    assert s.min() >= SMIN - 1e-12 and s.max() <= SMAX + 1e-12
    # optimality: no member of the band is closer (random members U diag(s) V^T)
    for k in range(50):
        A = np.stack([_rot(rng) @ np.diag(rng.uniform(SMIN, SMAX, 3)) @ _rot(rng)
                      for _ in range(200)])
        assert np.all(np.linalg.norm(F - Q, axis=(1, 2)) <= np.linalg.norm(F - A, axis=(1, 2)) + 1e-12)
    # inside the band Q = F
    G = np.stack([_rot(rng) @ np.diag(rng.uniform(SMIN + 0.01, SMAX - 0.01, 3)) @ _rot(rng)
                  for _ in range(20)])
    assert np.abs(fem.clamped_projection(G, SMIN, SMAX) - G).max() <= 1e-13
    # diagonal closed form, including a reflection
    D = np.diag([1.3, 0.5, -1.0])[None]
    assert np.allclose(fem.clamped_projection(D, SMIN, SMAX), np.diag([SMAX, SMIN, -1.0]), atol=1e-14)


def _one_tet():
    rest = np.array([[0.0, 1.0, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0], [0.0, 0.0, 0.0, 1.0]])
    return rest, np.array([[0], [1], [2], [3]])


def test_forces_are_minus_gradient_of_biphasic_energy():
    rng = np.random.default_rng(3)
    mu, mu_p = 2.0, 15.0
    for rest, tets in [_one_tet(), P.kuhn_grid(2, 2, 2, 1.0)]:
        B, vol = fem.shape_matrices(rest, tets)
        x = rest + 0.25 * rng.normal(size=rest.shape)

        def energy(xx):
            F = fem.deformation_gradients(xx, tets, B)
            return fem.pd_energy(xx, tets, B, vol, mu, fem.polar_rotation(F), None,
                                 fem.clamped_projection(F, SMIN, SMAX), mu_p)

        F = fem.deformation_gradients(x, tets, B)
        f = fem.nodal_forces(x, tets, B, vol, mu, fem.polar_rotation(F), None,
                             fem.clamped_projection(F, SMIN, SMAX), mu_p)
        h = 1e-6
        g = np.zeros_like(x)
        for i in range(3):
            for a in range(x.shape[1]):
                xp, xm = x.copy(), x.copy()
                xp[i, a] += h
                xm[i, a] -= h
                g[i, a] = (energy(xp) - energy(xm)) / (2 * h)
        assert np.abs(f + g).max() <= 1e-6 * np.abs(g).max()
        # the biphasic term is active somewhere
        sv = np.linalg.svd(F, compute_uv=False)
        assert ((sv < SMIN) | (sv > SMAX)).any()


def _scene():
    return P.scene_small(6, 5, 4, h=1.0, region_top_layers=2, seed=5, n_spheres=2,
                         depth_frac=0.12)


def _model(sc, **kw):
    return opd.PDModel(sc.rest, sc.tets, sc.mu, sc.dirichlet, sc.region, **kw)


def test_zero_mu_prime_is_corotated():
    sc = _scene()
    a = _model(sc)
    b = _model(sc, mu_prime=0.0, sigma_min=SMIN, sigma_max=SMAX)
    det = opd.sphere_detector(a, sc.proxy_local(), sc.spheres.centers(3), sc.spheres.radii,
                              sc.k_pen)
    xa = xb = sc.rest.copy()
    for _ in range(2):
        xa = opd.alg1_outer_iteration(a, xa, det, n_inner=2)
        xb = opd.alg1_outer_iteration(b, xb, det, n_inner=2)
    assert np.array_equal(xa, xb)


def test_schur_route_equals_full_solve_biphasic():
    sc = P.scene_small(4, 4, 3, h=1.0, region_top_layers=2, seed=11, n_spheres=2,
                       depth_frac=0.05)
    om = _model(sc, mu_prime=10 * sc.mu, sigma_min=SMIN, sigma_max=SMAX)
    det = opd.sphere_detector(om, sc.proxy_local(), sc.spheres.centers(4), sc.spheres.radii * 1.5,
                              1e6)
    pen = det(sc.rest[:, om.i2])
    assert (pen[2] > 0).sum() >= 2
    A, pos = opd.full_matrix_with_penalty(om, pen)
    b = np.random.default_rng(1).normal(size=(3, om.free.size))
    u_full = spla.spsolve(A, b.T).T
    assert np.linalg.norm(opd.three_step_solve(om, b, pen) - u_full) <= 1e-12 * np.linalg.norm(u_full)


def test_alg1_single_inner_equals_plain_pd_biphasic():
    sc = _scene()
    om = _model(sc, mu_prime=10 * sc.mu, sigma_min=SMIN, sigma_max=SMAX)
    xa = xp = sc.rest.copy()
    clamped = 0
    for step in range(1, 4):
        det = opd.sphere_detector(om, sc.proxy_local(), sc.spheres.centers(step),
                                  sc.spheres.radii, sc.k_pen)
        for _ in range(3):
            xa = opd.alg1_outer_iteration(om, xa, det, n_inner=1)
            xp = opd.plain_pd_iteration(om, xp, det)
            assert np.abs(xa - xp).max() <= 1e-12 * max(1.0, np.abs(xp).max())
        F = fem.deformation_gradients(xa, sc.tets, om.B)
        sv = np.linalg.svd(F, compute_uv=False)
        clamped = max(clamped, int(((sv < SMIN) | (sv > SMAX)).any(axis=1).sum()))
    assert clamped > 10                  # the strain limit is engaged


def test_local_and_global_steps_lower_the_energy():
    sc = P.scene_small(6, 5, 4, h=1.0, region_top_layers=2, seed=9)
    om = _model(sc, mu_prime=10 * sc.mu, sigma_min=SMIN, sigma_max=SMAX)
    rng = np.random.default_rng(4)
    x = sc.rest + 0.15 * rng.normal(size=sc.rest.shape)
    x[:, sc.dirichlet] = sc.rest[:, sc.dirichlet]
    no_contact = lambda x2: (np.full((0, 8), -1, np.int32), np.zeros((0, 8)), np.zeros(0),
                             np.zeros((3, 0)))
    e_prev = None
    for _ in range(4):
        Ra, Rb = om.rotations(x, om.alpha), om.rotations(x, om.beta)
        Qa, Qb = om.projections(x, om.alpha), om.projections(x, om.beta)
        if e_prev is not None:
            # local step at fixed x: from the previous (R, Q) to the new ones
            e_old = om.energy(x, *state, Q_alpha=state_q[0], Q_beta=state_q[1])
            assert om.energy(x, Ra, Rb, Q_alpha=Qa, Q_beta=Qb) <= e_old * (1 + 1e-13)
        e_loc = om.energy(x, Ra, Rb, Q_alpha=Qa, Q_beta=Qb)
        x = opd.plain_pd_iteration(om, x, no_contact)
        e_glob = om.energy(x, Ra, Rb, Q_alpha=Qa, Q_beta=Qb)
        assert e_glob <= e_loc * (1 + 1e-13)
        state, state_q, e_prev = (Ra, Rb), (Qa, Qb), e_glob
