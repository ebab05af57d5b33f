"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(closed forms, special cases, invariants, brute force on tiny meshes)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from hypothesis import given, settings, strategies as st

import pd_inputs as P
from oracle import fem, collision, schur, pd

MU = P.lame_mu()


def _model(scene, **kw):
    return pd.PDModel(scene.rest, scene.tets, scene.mu, scene.dirichlet, scene.region, **kw)


def test_mu_from_young_poisson():
    # lambda is dropped; only mu = E / (2 (1 + nu)) enters
    assert MU == pytest.approx(34482.758620689656, rel=1e-15)


def test_grid_counts():
    s = P.scene_cube8()
    assert (s.n_nodes, s.n_tets) == (729, 3072)
    m = _model(s, build_schur=False)
    assert m.m == 81 and m.beta.sum() == 0 and m.i1.size == 729 - 81 - 81
    assert np.allclose(m.vol, (1 / 8) ** 3 / 6)


def test_rest_state_identity():
    """Rest state: F = I, R = I, zero forces (P6)."""
    s = P.scene_small(3, 3, 3)
    m = _model(s, build_schur=False)
    F = fem.deformation_gradients(s.rest, s.tets, m.B)
    assert np.abs(F - np.eye(3)).max() < 1e-14
    R = fem.polar_rotation(F)
    assert np.abs(R - np.eye(3)).max() < 1e-14
    f = fem.nodal_forces(s.rest, s.tets, m.B, m.vol, MU, R)
    assert np.abs(f).max() < 1e-9


def _rand_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a*a+b*b-c*c-d*d, 2*(b*c-a*d), 2*(b*d+a*c)],
                     [2*(b*c+a*d), a*a-b*b+c*c-d*d, 2*(c*d-a*b)],
                     [2*(b*d-a*c), 2*(c*d+a*b), a*a-b*b-c*c+d*d]])


def test_rigid_invariance():
    """x = Q X + b: every rotation equals Q and all forces vanish (P7)."""
    rng = np.random.default_rng(3)
    s = P.scene_small(3, 2, 2)
    m = _model(s, build_schur=False)
    Q = _rand_rotation(rng)
    x = Q @ s.rest + rng.normal(size=(3, 1))
    F = fem.deformation_gradients(x, s.tets, m.B)
    R = fem.polar_rotation(F)
    assert np.abs(R - Q).max() < 1e-12
    f = fem.nodal_forces(x, s.tets, m.B, m.vol, MU, R)
    assert np.abs(f).max() < 1e-8


@settings(max_examples=60, deadline=None)
@given(st.integers(0, 10_000))
def test_polar_invariants(seed):
    """R^T R = I, det R = +1, R^T F symmetric positive semidefinite (P8), and
    R minimises ||F - R|| against random rotations."""
    rng = np.random.default_rng(seed)
    F = rng.normal(size=(1, 3, 3))
    R = fem.polar_rotation(F)[0]
    assert np.abs(R.T @ R - np.eye(3)).max() < 1e-12
    assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-12)
    Sm = R.T @ F[0]
    if np.linalg.det(F[0]) > 0:
        assert np.abs(Sm - Sm.T).max() < 1e-12
        assert np.linalg.eigvalsh(0.5 * (Sm + Sm.T)).min() > -1e-12
    best = np.linalg.norm(F[0] - R)
    for _ in range(20):
        Q = _rand_rotation(rng)
        assert best <= np.linalg.norm(F[0] - Q) + 1e-12


def test_forces_are_minus_energy_gradient():
    """f = -dE_hat/dx with R frozen, by central differences (P9)."""
    rng = np.random.default_rng(5)
    s = P.scene_small(2, 2, 1)
    m = _model(s, build_schur=False)
    x = s.rest + 0.1 * rng.normal(size=s.rest.shape)
    R = fem.polar_rotation(fem.deformation_gradients(x, s.tets, m.B))
    f = fem.nodal_forces(x, s.tets, m.B, m.vol, MU, R)
    eps = 1e-6
    for node in [0, 4, 7, 11]:
        for i in range(3):
            xp = x.copy(); xp[i, node] += eps
            xm = x.copy(); xm[i, node] -= eps
            g = (fem.pd_energy(xp, s.tets, m.B, m.vol, MU, R)
                 - fem.pd_energy(xm, s.tets, m.B, m.vol, MU, R)) / (2 * eps)
            assert -g == pytest.approx(f[i, node], rel=1e-6, abs=1e-3)


def test_stiffness_is_energy_hessian():
    """K (scalar block) is the Hessian of E_hat in each coordinate: E_hat is
    quadratic in x with R frozen, so E(x + d e_v) - E(x) - grad.d = 1/2 d^T K d."""
    rng = np.random.default_rng(6)
    s = P.scene_small(2, 2, 2)
    m = _model(s, build_schur=False)
    x = s.rest + 0.05 * rng.normal(size=s.rest.shape)
    R = fem.polar_rotation(fem.deformation_gradients(x, s.tets, m.B))
    f = fem.nodal_forces(x, s.tets, m.B, m.vol, MU, R)
    E0 = fem.pd_energy(x, s.tets, m.B, m.vol, MU, R)
    for v in range(3):
        d = rng.normal(size=s.n_nodes)
        xd = x.copy(); xd[v] += d
        E1 = fem.pd_energy(xd, s.tets, m.B, m.vol, MU, R)
        quad = E1 - E0 + f[v] @ d
        assert quad == pytest.approx(0.5 * d @ (m.K @ d), rel=1e-9)


def test_momentum_conservation():
    """Per tet the four forces sum to zero and exert no torque when
    R = polar(F) (P10)."""
    rng = np.random.default_rng(9)
    s = P.scene_small(2, 2, 2)
    m = _model(s, build_schur=False)
    x = s.rest + 0.2 * rng.normal(size=s.rest.shape)
    F = fem.deformation_gradients(x, s.tets, m.B)
    R = fem.polar_rotation(F)
    fe = fem.element_forces(F, R, m.B, m.vol, MU)
    assert np.abs(fe.sum(axis=1)).max() < 1e-9
    xe = np.moveaxis(x[:, s.tets], 0, -1)     # (4, T, 3)
    torque = np.cross(np.moveaxis(xe, 0, 1), fe).sum(axis=1)
    assert np.abs(torque).max() < 1e-8 * np.abs(fe).max()


def _linear_field_energy(m, scene, values_by_layer):
    """v^T S v for a region vector given per lattice layer."""
    nz = scene.nz
    kz = np.rint(scene.rest[2] / scene.h).astype(int)
    v = np.array([values_by_layer[k] for k in kz[m.i2]])
    return v @ m.schur() @ v


def test_schur_closed_form_cube8():
    """Linear fields are reproduced exactly by linear tets, so with the bottom
    pinned and the top layer as the region, 1^T S 1 = 2 mu A / L = 2 mu on the
    unit cube (P4)."""
    s = P.scene_cube8()
    m = _model(s)
    one = np.ones(m.m)
    assert one @ m.schur() @ one == pytest.approx(2 * MU, rel=1e-12)
    assert 2 * MU == pytest.approx(68965.51724137931, rel=1e-15)


@pytest.mark.parametrize("dims,h", [((4, 3, 5), 1.0), ((3, 4, 4), 0.5)])
def test_schur_closed_form_two_layer_region(dims, h):
    """Two-layer region: v = z/L on the region gives v^T S v = 2 mu A / L, and
    v clamped to 1 on both layers gives 2 mu A / (L - h) (P4)."""
    nx, ny, nz = dims
    s = P.scene_small(nx, ny, nz, h=h, region_top_layers=2)
    m = _model(s)
    A = nx * ny * h * h
    L = nz * h
    e1 = _linear_field_energy(m, s, {nz - 1: (nz - 1) / nz, nz: 1.0})
    assert e1 == pytest.approx(2 * MU * A / L, rel=1e-11)
    e2 = _linear_field_energy(m, s, {nz - 1: 1.0, nz: 1.0})
    assert e2 == pytest.approx(2 * MU * A / (L - h), rel=1e-11)


def test_schur_spd_symmetric():
    """S symmetric positive definite (P3)."""
    s = P.scene_small(4, 3, 4, region_top_layers=2)
    m = _model(s)
    S = m.schur()
    assert np.abs(S - S.T).max() <= 1e-13 * np.abs(S).max()
    assert np.linalg.eigvalsh(S).min() > 0


def test_schur_special_cases():
    """Region = all free nodes gives S = K_ff; a single interior node gives
    S = K22 - k21 k12 / k11 (P5)."""
    s = P.scene_small(2, 2, 2, region_top_layers=3)       # every free node is region
    m = _model(s)
    Kff = sp.csr_matrix(m.K)[m.free][:, m.free].toarray()
    assert m.i1.size == 0
    assert np.abs(m.schur() - Kff).max() < 1e-9
    # one interior node: nz = 2, region = top layer -> interior = layer 1 minus ...
    s = P.scene_small(1, 1, 2, region_top_layers=1)
    reg = s.region.copy()
    lay1 = np.nonzero(P.layer_mask(1, 1, 2, [1]))[0]
    reg[lay1[1:]] = True            # keep a single interior node
    m = pd.PDModel(s.rest, s.tets, s.mu, s.dirichlet, reg)
    assert m.i1.size == 1
    K11 = m.A11.toarray()[0, 0]
    k12 = m.A12.toarray()[0]
    k21 = m.A21.toarray()[:, 0]
    assert np.abs(m.schur() - (m.A22.toarray() - np.outer(k21, k12) / K11)).max() < 1e-9


def test_schur_probe_matches_dense():
    """Sigma v through one sparse solve equals the dense Sigma times v (P12)."""
    s = P.scene_small(5, 4, 4, region_top_layers=2)
    m = _model(s)
    rng = np.random.default_rng(0)
    for _ in range(4):
        v = rng.normal(size=m.m)
        a = schur.schur_apply(m.lu11, m.A12, m.A21, m.A22, v)
        assert np.linalg.norm(a - m.schur() @ v) <= 1e-12 * np.linalg.norm(a)


def _pushed_scene_state(nx=4, ny=4, nz=3, steps=2, seed=11):
    s = P.scene_small(nx, ny, nz, region_top_layers=2, seed=seed, n_spheres=2,
                      depth_frac=0.05)
    m = _model(s)
    det = pd.sphere_detector(m, s.proxy_local(), s.spheres.centers(steps),
                             s.spheres.radii, s.k_pen)
    return s, m, det


def test_three_step_solve_equals_full_solve():
    """Schur route (Steps 1-3 of Sec. 4.4 with eq. k22) reproduces the direct
    solve of (K + W^T C W) u = b over all free nodes (P1)."""
    s, m, det = _pushed_scene_state()
    pen = det(s.rest[:, m.i2])
    assert (pen[2] > 0).sum() > 0
    A, pos = pd.full_matrix_with_penalty(m, pen)
    rng = np.random.default_rng(1)
    b = rng.normal(size=(3, m.free.size))
    u_full = spla.spsolve(A, b.T).T
    u_schur = pd.three_step_solve(m, b, pen)
    assert np.linalg.norm(u_schur - u_full) <= 1e-12 * np.linalg.norm(u_full)


def test_alg1_single_inner_equals_plain_pd():
    """Alg. 1 with one inner iteration is plain full-mesh PD iterate by
    iterate (P2)."""
    s, m, det = _pushed_scene_state()
    x_a = s.rest.copy()
    x_b = s.rest.copy()
    for it in range(4):
        x_a = pd.alg1_outer_iteration(m, x_a, det, n_inner=1)
        x_b = pd.plain_pd_iteration(m, x_b, det)
        disp = np.linalg.norm(x_b - s.rest)
        assert disp > 0
        assert np.linalg.norm(x_a - x_b) <= 1e-11 * disp


def test_rest_state_no_contact_no_motion():
    """Rest state without contact: zero correction (P6)."""
    s = P.scene_small(3, 3, 3, region_top_layers=2)
    m = _model(s)
    det = pd.sphere_detector(m, s.proxy_local(), np.array([[100.], [100.], [100.]]),
                             np.array([1.0]), s.k_pen)
    x = pd.alg1_outer_iteration(m, s.rest, det, n_inner=2)
    assert np.abs(x - s.rest).max() <= 1e-12 * s.h


def test_energy_monotone_local_and_global():
    """Each local step and each global step (R, C, t frozen) does not increase
    E_hat (Sec. 3.2 alternating minimisation; P11)."""
    s, m, det = _pushed_scene_state()
    x = s.rest.copy()
    allt = np.ones(s.n_tets, dtype=bool)
    for it in range(4):
        R_old = m.rotations(x, allt) if it else np.broadcast_to(np.eye(3), (s.n_tets, 3, 3))
        pen = det(x[:, m.i2])
        e0 = fem.pd_energy(x, s.tets, m.B, m.vol, MU, R_old)
        R = m.rotations(x, allt)
        e1 = fem.pd_energy(x, s.tets, m.B, m.vol, MU, R)
        assert e1 <= e0 + 1e-9 * max(1.0, abs(e0))
        # global step with (R, C, t) frozen
        idx, w, c, t = pen
        E_before = e1 + collision.penalty_energy(idx, w, c, t, x[:, m.i2])
        A, pos = pd.full_matrix_with_penalty(m, pen)
        f = m.forces(x, R, allt)[:, m.free]
        f[:, pos[m.i2]] += collision.penalty_force(m.m, idx, w, c, t, x[:, m.i2])
        dx = spla.spsolve(A, f.T).T
        xn = x.copy()
        xn[:, m.free] += dx
        E_after = (fem.pd_energy(xn, s.tets, m.B, m.vol, MU, R)
                   + collision.penalty_energy(idx, w, c, t, xn[:, m.i2]))
        assert E_after <= E_before + 1e-9 * max(1.0, abs(E_before))
        x = xn


def test_alg1_inner_loop_monotone_with_frozen_contacts():
    """Inside the inner loop with the penalty set frozen, every E_beta local
    step + global solve pair does not raise E_hat (P11, frozen-set case)."""
    s, m, det = _pushed_scene_state(nx=4, ny=3, nz=3)
    pen0 = det(s.rest[:, m.i2])
    frozen = lambda x2: pen0
    log = pd.IterLog([], [])
    pd.alg1_outer_iteration(m, s.rest, frozen, n_inner=4, log=log, check_energy=True)
    e = np.array(log.energies)
    assert np.all(np.diff(e) <= 1e-9 * np.abs(e).max())


def test_penalty_separable_by_coordinate():
    """Only the x column of g nonzero -> u_y = u_z = 0 exactly (P13)."""
    s, m, det = _pushed_scene_state()
    pen = det(s.rest[:, m.i2])
    b = np.zeros((3, m.free.size))
    b[0] = np.random.default_rng(2).normal(size=m.free.size)
    u = pd.three_step_solve(m, b, pen)
    assert np.all(u[1:] == 0.0)


def test_penalty_matrix_and_force_by_definition():
    """W^T C W and -W^T C (W x - t) on a general (non-conforming) penalty:
    the force is minus the gradient of E_col, the matrix its Hessian."""
    rng = np.random.default_rng(4)
    mloc = 9
    idx = np.full((3, 8), -1, dtype=np.int32)
    idx[0, :4] = [0, 3, 5, 8]
    idx[1, :4] = [3, 4, 5, 6]
    idx[2, :1] = [2]
    w = np.zeros((3, 8))
    w[0, :4] = [1.0, -0.2, -0.3, -0.5]
    w[1, :4] = [0.25, 0.25, 0.25, 0.25]
    w[2, 0] = 1.0
    c = np.array([5.0, 3.0, 0.0])
    t = rng.normal(size=(3, 3))
    x2 = rng.normal(size=(3, mloc))
    f = collision.penalty_force(mloc, idx, w, c, t, x2)
    Pm = collision.penalty_matrix(mloc, idx, w, c)
    eps = 1e-6
    for a in range(mloc):
        for v in range(3):
            xp = x2.copy(); xp[v, a] += eps
            xm = x2.copy(); xm[v, a] -= eps
            g = (collision.penalty_energy(idx, w, c, t, xp)
                 - collision.penalty_energy(idx, w, c, t, xm)) / (2 * eps)
            assert -g == pytest.approx(f[v, a], abs=1e-6)
    d = rng.normal(size=mloc)
    xd = x2.copy(); xd[1] += d
    quad = (collision.penalty_energy(idx, w, c, t, xd) - collision.penalty_energy(idx, w, c, t, x2)
            + f[1] @ d)
    assert quad == pytest.approx(0.5 * d @ Pm @ d, rel=1e-9)
    assert np.abs(Pm - Pm.T).max() <= 1e-15 * np.abs(Pm).max()


def test_penalty_gap_shrinks_like_one_over_k():
    """A single free node tied to the ground by a spring of stiffness s and
    pulled to t by a penalty k settles at k t / (s + k); the gap to t is
    O(1/k) (P16)."""
    s_stiff, t = 2.0, 1.0
    gaps = []
    for k in [1e3, 1e4, 1e5, 1e6]:
        idx = np.full((1, 8), -1, dtype=np.int32); idx[0, 0] = 0
        w = np.zeros((1, 8)); w[0, 0] = 1.0
        H = s_stiff + collision.penalty_matrix(1, idx, w, np.array([k]))[0, 0]
        g = collision.penalty_force(1, idx, w, np.array([k]), np.full((3, 1), t),
                                    np.zeros((3, 1)))[0, 0]
        u = g / H
        assert u == pytest.approx(k * t / (s_stiff + k), rel=1e-14)
        gaps.append(t - u)
    r = np.array(gaps[:-1]) / np.array(gaps[1:])
    assert np.all(np.abs(r - 10) < 0.02)


def test_sphere_detection_rules():
    c_ = np.array([[0.0], [0.0], [0.0]])
    r = np.array([1.0])
    p = np.array([[0.5, 2.0, 1.0, 0.0], [0.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.0]])
    c, t = collision.detect_spheres(p, c_, r, 7.0)
    assert list(c) == [7.0, 0.0, 0.0, 7.0]           # strict inside test
    assert np.allclose(t[:, 0], [1, 0, 0])
    assert np.allclose(t[:, 3], [0, 0, 1])           # centre -> +z
    # two spheres: deepest wins, ties -> lowest index
    cs = np.array([[0.0, 0.3], [0.0, 0.0], [0.0, 0.0]])
    c, t = collision.detect_spheres(np.array([[0.25], [0.0], [0.0]]), cs, np.array([1.0, 1.0]), 1.0)
    assert np.allclose(t[:, 0], [-0.7, 0, 0])      # sphere 1 is deeper (0.95 > 0.75)
    cs = np.array([[-0.5, 0.5], [0.0, 0.0], [0.0, 0.0]])
    c, t = collision.detect_spheres(np.array([[0.0], [0.0], [0.0]]), cs, np.array([1.0, 1.0]), 1.0)
    assert np.allclose(t[:, 0], [0.5, 0, 0])


def test_cholesky_definition():
    """The dense factor used for H = S + P is the unique lower factor with a
    positive diagonal: L L^T = H to rounding (P14)."""
    import scipy.linalg as sla
    s, m, det = _pushed_scene_state()
    pen = det(s.rest[:, m.i2])
    H = m.schur() + collision.penalty_matrix(m.m, *pen[:3])
    L = np.tril(sla.cho_factor(H, lower=True)[0])
    assert np.all(np.diag(L) > 0)
    assert np.linalg.norm(L @ L.T - H) <= 10 * H.shape[0] * np.finfo(float).eps * np.linalg.norm(H)


def test_slit_mesh_and_pair_detection():
    """Slit grid: positive volumes, lips only shared at the front line; pair
    detection fires only for interpenetrating twins, and the pair spring is
    the gradient/Hessian of c/2 ||p_a - p_b||^2."""
    s = P.scene_slit(6, 6, 6, 3, 4)
    m = pd.PDModel(s.rest, s.tets, s.mu, s.dirichlet, s.region, build_schur=False)
    assert np.all(m.vol > 0)
    pl = s.pairs_local()
    x2 = s.rest[:, m.i2].copy()
    idx, w, c, t = collision.detect_pairs(x2, pl, 5e5)
    assert np.all(c == 0)                       # rest: lips touch, no penetration
    x2[2, pl[0, 0]] += 0.1                      # lower lip node pushed up through
    idx, w, c, t = collision.detect_pairs(x2, pl, 5e5)
    assert np.nonzero(c)[0].tolist() == [0]
    f = collision.penalty_force(m.m, idx, w, c, t, x2)
    a, b = pl[0, 0], pl[1, 0]
    assert f[2, a] == pytest.approx(-5e5 * 0.1) and f[2, b] == pytest.approx(5e5 * 0.1)
    Pm = collision.penalty_matrix(m.m, idx, w, c)
    assert Pm[a, a] == 5e5 and Pm[b, b] == 5e5 and Pm[a, b] == -5e5


def test_slit_schur_route_equals_full_solve():
    """The Schur route reproduces the full solve with two-node (off-diagonal)
    penalties (P1 for non-conforming W)."""
    s = P.scene_slit(6, 6, 6, 3, 4)
    m = pd.PDModel(s.rest, s.tets, s.mu, s.dirichlet, s.region)
    pl = s.pairs_local()
    x2 = s.rest[:, m.i2].copy()
    x2[2, pl[0, :5]] += 0.05
    pen = collision.detect_pairs(x2, pl, 5e5)
    A, pos = pd.full_matrix_with_penalty(m, pen)
    b = np.random.default_rng(3).normal(size=(3, m.free.size))
    u_full = spla.spsolve(A, b.T).T
    u_schur = pd.three_step_solve(m, b, pen)
    assert np.linalg.norm(u_schur - u_full) <= 1e-11 * np.linalg.norm(u_full)


def test_corotated_energy_closed_form():
    """E(x) = min_R E_hat(x, R) (Sec. 3.2): for F = Q1 diag(s) Q2 with proper
    rotations Q1, Q2 the minimum is mu Vol sum_i (s_i - 1)^2; for an inverted F
    (one negative factor, R restricted to SO(3)) the smallest singular value
    enters as (sigma_3 + 1)^2; and no random rotation does better."""
    rng = np.random.default_rng(41)
    rest = np.array([[0.0, 1.0, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0], [0.0, 0.0, 0.0, 1.0]]) * 0.7
    tets = np.array([[0], [1], [2], [3]])
    B, vol = fem.shape_matrices(rest, tets)
    for inverted in (False, True):
        for _ in range(5):
            s = np.sort(rng.uniform(0.3, 1.8, size=3))[::-1]
            Q1, Q2 = _rand_rotation(rng), _rand_rotation(rng)
            d = s.copy()
            if inverted:
                d[2] = -d[2]
            F = Q1 @ np.diag(d) @ Q2
            x = F @ rest + rng.normal(size=(3, 1))
            e = fem.corotated_energy(x, tets, B, vol, MU)
            if inverted:
                want = (s[0] - 1) ** 2 + (s[1] - 1) ** 2 + (s[2] + 1) ** 2
            else:
                want = np.sum((s - 1) ** 2)
            want *= MU * vol[0]
            assert e == pytest.approx(want, rel=1e-12)
            for _ in range(20):
                Rr = _rand_rotation(rng)[None]
                assert fem.pd_energy(x, tets, B, vol, MU, Rr) >= e * (1 - 1e-12)


def test_alg1_nested_iteration_reaches_plain_pd_fixed_point():
    """The inner loop only reorganises the minimisation (Sec. 4.5): Alg. 1 with
    three inner iterations, iterated to convergence, stops at the fixed point of
    plain full-mesh PD (f_tot = 0 with R = polar(F) and the penalty set
    consistent with the positions), not at a different state."""
    s, m, det = _pushed_scene_state(nx=4, ny=3, nz=3, steps=3)

    def converge(step, tol=1e-12, cap=3000):
        x = s.rest.copy()
        for it in range(cap):
            xn = step(x)
            if np.linalg.norm(xn - x) <= tol * np.linalg.norm(xn - s.rest):
                return xn, it + 1
            x = xn
        raise AssertionError("no convergence")

    x_plain, it_plain = converge(lambda x: pd.plain_pd_iteration(m, x, det))
    x_nest, it_nest = converge(lambda x: pd.alg1_outer_iteration(m, x, det, n_inner=3))
    disp = np.linalg.norm(x_plain - s.rest)
    assert disp > 0 and (det(x_plain[:, m.i2])[2] > 0).any()
    assert np.linalg.norm(x_nest - x_plain) <= 1e-9 * disp
    # the nested state is itself a fixed point of the plain iteration
    assert np.linalg.norm(pd.plain_pd_iteration(m, x_nest, det) - x_nest) <= 1e-10 * disp
    # and the inner loop needs no more outer iterations than plain PD
    assert it_nest <= it_plain
