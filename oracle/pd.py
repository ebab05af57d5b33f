"""Projective Dynamics with localized collisions: the reference iteration.

Follows Alg. 1 of the paper ("Optimized solve with collisions") together with
Sec. 4.4-4.5, and plain full-mesh PD (Sec. 3.2-3.3) as the fixed point it
must agree with.  Conventions:
  * positions x are (3, n) float64 in global node order; Dirichlet nodes are
    prescribed and not unknowns;
  * x2 = collision-prone free nodes in ascending global id ("region-local"
    order), x1 = the remaining free nodes;
  * E_beta = tets whose four vertices are all in x2, E_alpha = the rest
    (Sec. 4.5 and the caption of the partitioning figure);
  * A = K restricted to free nodes; A^(beta)_22 = the part of A22 coming from
    E_beta, Sigma_alpha = Sigma - A^(beta)_22 where Sigma is the Schur
    complement of the full K (A11, A12 and A21 only involve E_alpha tets).
Readings of the paper used here:
  * Step 4.7 subtracts Sigma_alpha u2 (not Sigma u2).
  * Step 5 is the full back substitution x1 += A11^-1 (f1 - A12 Delta2) with
    Delta2 the sum of the inner corrections (the three-step solve of Sec. 4.4,
    Step 3); the printed "L1^T u1 = y1" omits the coupling term.
  * The local step on E_beta runs inside the inner loop (Sec. 4.5), and
    detection and the E_beta local step both read the same x2, so their order
    does not matter.
"""
from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import fem, schur, collision


class PDModel:
    """Constant data of one mesh: shape operators, partition, K blocks,
    sparse factor of A11 and (lazily) the dense Schur complement.

    Backward-Euler dynamics (dt > 0): the step minimises the incremental
    potential 1/(2 dt^2) (x - y)^T M (x - y) + E(x) with y = x_n + dt v_n and
    lumped masses M, the quasistatic energy plus an inertia term that is
    quadratic in x and independent of the rotations.  Its Hessian D = M/dt^2
    (diagonal) joins the constant matrix (K + D), so the Schur complement is
    built once as before; its force -D (x - y) joins the outer-loop force of
    every free node, with the E_alpha terms (it does not depend on R, so the
    inner loop's update of f~2 by Sigma_alpha u2 keeps it exact)."""

    def __init__(self, rest, tets, mu, dirichlet, region, build_schur=True, density=0.0,
                 dt=0.0, mu_prime=0.0, sigma_min=0.0, sigma_max=np.inf):
        self.rest = np.asarray(rest, dtype=np.float64)
        self.tets = np.asarray(tets)
        self.mu = float(mu)
        n = self.rest.shape[1]
        self.n = n
        self.dirichlet = np.asarray(dirichlet, dtype=bool)
        self.region = np.asarray(region, dtype=bool)
        free = ~self.dirichlet
        self.i2 = np.nonzero(self.region & free)[0]
        self.i1 = np.nonzero(~self.region & free)[0]
        self.free = np.nonzero(free)[0]
        in2 = np.zeros(n, dtype=bool)
        in2[self.i2] = True
        self.beta = np.all(in2[self.tets], axis=0)
        self.alpha = ~self.beta
        self.B, self.vol = fem.shape_matrices(self.rest, self.tets)
        # biphasic material (Sec. 5.3): a second projective term mu' ||F - Q||^2
        # with Q the strain-limited projection of F; its constant Hessian adds
        # mu' to mu in K
        self.mu_p = float(mu_prime)
        self.sigma = (float(sigma_min), float(sigma_max))
        self.K = fem.scalar_stiffness(n, self.tets, self.B, self.vol, self.mu + self.mu_p)
        self.D = None
        if dt > 0.0:
            self.D = fem.lumped_mass(n, self.tets, self.vol, density) / (dt * dt)
            self.K = sp.csr_matrix(self.K + sp.diags(self.D))
        Kb = fem.scalar_stiffness(n, self.tets, self.B, self.vol, self.mu + self.mu_p,
                                  subset=self.beta)
        self.A11, self.A12, self.A21, self.A22 = schur.blocks(self.K, self.i1, self.i2)
        self.Abeta22 = sp.csr_matrix(Kb)[self.i2][:, self.i2]
        self.lu11 = schur.sparse_factor(self.A11) if self.i1.size else None
        self._S = None
        if build_schur:
            self.schur()

    @property
    def m(self):
        return self.i2.size

    def schur(self):
        """Sigma = A22 - A21 A11^-1 A12 (eq. par_chol / eq. k22, collision-free)."""
        if self._S is None:
            if self.i1.size == 0:
                self._S = self.A22.toarray()
            else:
                self._S = schur.schur_complement(self.A11, self.A12, self.A21, self.A22,
                                                 self.lu11)
        return self._S

    def sigma_alpha(self):
        return self.schur() - self.Abeta22.toarray()

    # --- local step and forces -------------------------------------------
    def rotations(self, x, subset):
        F = fem.deformation_gradients(x, self.tets[:, subset], self.B[subset])
        return fem.polar_rotation(F)

    def projections(self, x, subset):
        """Biphasic local step (Sec. 5.3): Q_e = clamped-SVD projection of F_e for
        the tets in `subset`; None for the plain corotated material."""
        if self.mu_p == 0.0:
            return None
        F = fem.deformation_gradients(x, self.tets[:, subset], self.B[subset])
        return fem.clamped_projection(F, *self.sigma)

    def forces(self, x, R, subset, Q=None):
        """Elastic forces (3, n) from the tets in `subset` with rotations R (and
        biphasic projections Q), one per tet of the subset."""
        return fem.nodal_forces(x, self.tets, self.B, self.vol, self.mu, R, subset, Q, self.mu_p)

    def inertia_force(self, x, y):
        """-D (x - y) (3, n), zero on Dirichlet nodes; zero without dynamics."""
        if self.D is None or y is None:
            return np.zeros_like(x)
        f = -self.D[None, :] * (x - y)
        f[:, self.dirichlet] = 0.0
        return f

    def energy(self, x, R_alpha, R_beta, pen=None, y=None, Q_alpha=None, Q_beta=None):
        """E_hat(x, R) + E_col (eq. energyHat + Sec. 3.3) with the given rotations
        and frozen penalty set, plus the inertia term 1/2 (x - y)^T D (x - y)
        over the free nodes under backward Euler."""
        e = fem.pd_energy(x, self.tets, self.B, self.vol, self.mu, R_alpha, self.alpha, Q_alpha,
                          self.mu_p)
        if self.D is not None and y is not None:
            d = (x - y)[:, self.free]
            e += 0.5 * float(np.sum(self.D[self.free][None, :] * d * d))
        if self.beta.any():
            e += fem.pd_energy(x, self.tets, self.B, self.vol, self.mu, R_beta, self.beta, Q_beta,
                               self.mu_p)
        if pen is not None:
            idx, w, c, t = pen
            e += collision.penalty_energy(idx, w, c, t, x[:, self.i2])
        return e


@dataclass
class IterLog:
    u2_norms: list
    energies: list


def _solve_cols(lu, b):
    """Apply A^-1 to each coordinate row of b (3, k)."""
    return lu.solve(np.ascontiguousarray(b.T)).T


def _x1_completed(model, x, f1, delta2, x2):
    """Positions with x2 given and x1 at the minimiser of E_hat_alpha over x1
    (the nested minimisation of Sec. 4.5 that defines E~_alpha(x2))."""
    xe = x.copy()
    if model.i1.size:
        xe[:, model.i1] += _solve_cols(model.lu11, f1 - (model.A12 @ delta2.T).T)
    xe[:, model.i2] = x2
    return xe


def alg1_outer_iteration(model, x, detect, n_inner=1, log=None, check_energy=False, y=None):
    """One outer iteration of Alg. 1.  `detect(x2) -> (idx, w, c, t)` returns the
    penalty set for the current region positions.  Under backward Euler, y is
    the inertial target x_n + dt v_n.  Returns the new x (3, n)."""
    x = x.copy()
    i1, i2 = model.i1, model.i2
    # 1. local step on E_alpha (rotations, and strain-limited projections for
    #    the biphasic material)
    R_a = model.rotations(x, model.alpha)
    Q_a = model.projections(x, model.alpha)
    # 2. forces from E_alpha only (plus inertia under backward Euler)
    f = model.forces(x, R_a, model.alpha, Q_a) + model.inertia_force(x, y)
    f1, f2 = f[:, i1], f[:, i2]
    # 3. forward substitution: w = A11^-1 f1, y2 = f2 - A21 w  (steps 3.1, 3.2)
    if i1.size:
        w = _solve_cols(model.lu11, f1)
        ft = f2 - (model.A21 @ w.T).T
    else:
        w = np.zeros_like(f1)
        ft = f2.copy()
    S = model.schur()
    Sa = model.sigma_alpha()
    x2 = x[:, i2].copy()
    delta2 = np.zeros_like(x2)
    m = model.m
    for _ in range(n_inner):
        # 4.1 detection and 4.2 local step on E_beta, both at the current x2
        pen = detect(x2)
        xfull = x.copy()
        xfull[:, i2] = x2
        R_b = model.rotations(xfull, model.beta) if model.beta.any() else np.zeros((0, 3, 3))
        Q_b = model.projections(xfull, model.beta) if model.beta.any() else None
        idx, wts, c, t = pen
        # 4.3 H = Sigma_alpha + A22^(beta) + C22 = Sigma + W^T C W
        H = S + collision.penalty_matrix(m, idx, wts, c)
        # 4.4 g = f~2 + f2^(beta) + f2^(col)
        fb = model.forces(xfull, R_b, model.beta, Q_b)[:, i2] if model.beta.any() else 0.0
        g = ft + fb + collision.penalty_force(m, idx, wts, c, t, x2)
        if check_energy and log is not None:
            log.energies.append(model.energy(_x1_completed(model, x, f1, delta2, x2),
                                             R_a, R_b, pen, y, Q_a, Q_b))
        # 4.5 dense Cholesky solve, three right-hand sides
        cf = sla.cho_factor(H, lower=True)
        u2 = sla.cho_solve(cf, g.T).T
        # 4.6, 4.7
        x2 += u2
        delta2 += u2
        ft -= (Sa @ u2.T).T
        if log is not None:
            log.u2_norms.append(float(np.linalg.norm(u2)))
            if check_energy:
                log.energies.append(model.energy(_x1_completed(model, x, f1, delta2, x2),
                                                 R_a, R_b, pen, y, Q_a, Q_b))
    # 5. back substitution x1 += A11^-1 (f1 - A12 Delta2)
    if i1.size:
        x[:, i1] += _solve_cols(model.lu11, f1 - (model.A12 @ delta2.T).T)
    x[:, i2] = x2
    return x


def full_matrix_with_penalty(model, pen):
    """Free-node global-step matrix K + W^T C W (Sec. 4.1) as CSC."""
    idx, w, c, t = pen
    Kf = sp.csr_matrix(model.K)[model.free][:, model.free]
    pos = np.full(model.n, -1)
    pos[model.free] = np.arange(model.free.size)
    m = model.m
    Pm = sp.coo_matrix(collision.penalty_matrix(m, idx, w, c))
    loc = pos[model.i2]
    Pf = sp.csr_matrix((Pm.data, (loc[Pm.row], loc[Pm.col])), shape=Kf.shape)
    return sp.csc_matrix(Kf + Pf), pos


def plain_pd_iteration(model, x, detect, y=None):
    """Plain full-mesh PD iteration (Sec. 3.2-3.3): local step on every tet,
    detection, then one solve of (K + W^T C W) dx = f_el + f_col over all free
    nodes (K including D and f_el the inertia force under backward Euler,
    inertial target y).  Returns the new x."""
    x = x.copy()
    every = np.ones(model.tets.shape[1], dtype=bool)
    R = model.rotations(x, every)
    Q = model.projections(x, every)
    f = model.forces(x, R, every, Q) + model.inertia_force(x, y)
    pen = detect(x[:, model.i2])
    idx, w, c, t = pen
    A, pos = full_matrix_with_penalty(model, pen)
    rhs = f[:, model.free].copy()
    fcol = collision.penalty_force(model.m, idx, w, c, t, x[:, model.i2])
    rhs[:, pos[model.i2]] += fcol
    dx = schur.sparse_factor(A).solve(np.ascontiguousarray(rhs.T))
    x[:, model.free] += dx.T
    return x


def three_step_solve(model, b_free, pen):
    """Solve (K + W^T C W) u = b over the free nodes through the Schur route
    (Sec. 4.4 Steps 1-3 with eq. k22).  b_free (3, n_free) in free order."""
    idx, w, c, t = pen
    pos = np.full(model.n, -1)
    pos[model.free] = np.arange(model.free.size)
    b1 = b_free[:, pos[model.i1]]
    b2 = b_free[:, pos[model.i2]]
    if model.i1.size:
        w1, y2 = schur.forward_sub(model.lu11, model.A21, b1.T, b2.T)
    else:
        w1, y2 = np.zeros((0, 3)), b2.T
    H = model.schur() + collision.penalty_matrix(model.m, idx, w, c)
    z2 = sla.cho_solve(sla.cho_factor(H, lower=True), y2)
    u = np.zeros_like(b_free)
    u[:, pos[model.i2]] = z2.T
    if model.i1.size:
        u[:, pos[model.i1]] = schur.back_sub(model.lu11, model.A12, b1.T, z2).T
    return u


def sphere_detector(model, proxy_local, centers, radii, k):
    """Detection closure for conforming proxies (region nodes) and spheres."""
    def detect(x2):
        c, t = collision.detect_spheres(x2[:, proxy_local], centers, radii, k)
        return collision.conforming_penalties(proxy_local, c, t)
    return detect


def backward_euler_advance(x_new, x_old, dt):
    """End of a backward-Euler step: v_{n+1} = (x_{n+1} - x_n) / dt and the
    next step's inertial target y = x_{n+1} + dt v_{n+1}.  Returns (v, y)."""
    v = (x_new - x_old) / dt
    return v, x_new + dt * v
