"""Linear-tetrahedron FEM quantities for the Projective Dynamics energy.

Paper Sec. 3.2: the deformation gradient F_e is constant per tet and linear
in the node positions; the PD energy density is mu*||F - R||_F^2 with R an
independent rotation (eq. psihat_f), integrated with the rest volume
(eq. energyHat); the local step sets R_e = U V^T from the SVD of F_e; the
first Piola stress is P = 2 mu (F - R) and the elemental force follows from
it; the Hessian K_el is block diagonal with three identical scalar blocks.
lambda is dropped (Sec. 3.2, after eq. psi_f).
"""
import numpy as np
import scipy.sparse as sp


def shape_matrices(rest, tets):
    """Rest shape matrix D_m = [X1-X0, X2-X0, X3-X0] per tet, Vol_e = det(D_m)/6,
    and the gradient operator B_e (4x3): rows 1..3 are the rows of D_m^-1,
    row 0 is minus their sum, so that F_e = sum_a x_a (B_e)_a^T = D_s D_m^-1.

    rest: (3, n), tets: (4, T) -> B (T, 4, 3), vol (T,)
    """
    X = rest[:, tets]                                   # (3, 4, T)
    Dm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=-1)
    Dm = np.moveaxis(Dm, 1, 0)                          # (T, 3, 3), columns are edges
    vol = np.linalg.det(Dm) / 6.0
    if np.any(vol <= 0):
        raise ValueError("inverted or degenerate rest tetrahedron")
    Dminv = np.linalg.inv(Dm)
    B = np.empty((tets.shape[1], 4, 3))
    B[:, 1:, :] = Dminv
    B[:, 0, :] = -Dminv.sum(axis=1)
    return B, vol


def deformation_gradients(x, tets, B):
    """F_e[i, j] = sum_a x_{a,i} B_e[a, j]  (Sec. 3.2, F linear in x).  -> (T, 3, 3)"""
    Xe = x[:, tets]                                     # (3, 4, T)
    return np.einsum("iat,taj->tij", Xe, B)


def polar_rotation(F):
    """Local step (Sec. 3.2): the rotation minimizing ||F - R||_F over SO(3),
    R = U diag(1, 1, det(U V^T)) V^T from the SVD F = U Sigma V^T.
    The sign fix keeps R a proper rotation when F is inverted."""
    U, s, Vt = np.linalg.svd(F)
    d = np.sign(np.linalg.det(U @ Vt))
    d[d == 0] = 1.0
    D = np.zeros_like(F)
    D[:, 0, 0] = 1.0
    D[:, 1, 1] = 1.0
    D[:, 2, 2] = d
    return U @ D @ Vt


def clamped_projection(F, sigma_min, sigma_max):
    """Biphasic strain limit (Sec. 5.3): the closest matrix to F whose singular
    values lie in [sigma_min, sigma_max], Q = U clamp(Sigma) V^T from the SVD
    F = U Sigma V^T (singular values >= 0, no sign fix: the set is not limited
    to rotations)."""
    U, s, Vt = np.linalg.svd(F)
    return U @ (np.clip(s, sigma_min, sigma_max)[..., :, None] * Vt)


def element_forces(F, R, B, vol, mu, Q=None, mu_p=0.0):
    """Per-vertex elemental forces f_{e,a} = -Vol_e P (B_e)_a with P = 2 mu (F - R)
    (Sec. 3.2: first Piola stress of the PD energy, R held fixed), plus
    2 mu' (F - Q) for the biphasic material of Sec. 5.3 (Q held fixed).
    -> (T, 4, 3)"""
    P = 2.0 * mu * (F - R)
    if Q is not None and mu_p != 0.0:
        P = P + 2.0 * mu_p * (F - Q)
    return -vol[:, None, None] * np.einsum("tij,taj->tai", P, B)


def nodal_forces(x, tets, B, vol, mu, R, subset=None, Q=None, mu_p=0.0):
    """Sum elemental forces onto nodes.  subset: boolean tet mask or None (all);
    R (and Q for the biphasic term) hold one matrix per tet of the subset.
    Returns f (3, n)."""
    if subset is not None:
        tets, B, vol = tets[:, subset], B[subset], vol[subset]
    F = deformation_gradients(x, tets, B)
    fe = element_forces(F, R, B, vol, mu, Q, mu_p)      # (T, 4, 3)
    f = np.zeros_like(x)
    for a in range(4):
        for i in range(3):
            np.add.at(f[i], tets[a], fe[:, a, i])
    return f


def pd_energy(x, tets, B, vol, mu, R, subset=None, Q=None, mu_p=0.0):
    """E_hat(x, R) = sum_e Vol_e mu ||F_e(x) - R_e||_F^2  (eq. energyHat), plus
    Vol_e mu' ||F_e - Q_e||^2 for the biphasic material (Sec. 5.3).
    R (and Q) hold one matrix per tet of the subset."""
    if subset is not None:
        tets, B, vol = tets[:, subset], B[subset], vol[subset]
    F = deformation_gradients(x, tets, B)
    e = np.sum(vol * mu * np.sum((F - R) ** 2, axis=(1, 2)))
    if Q is not None and mu_p != 0.0:
        e += np.sum(vol * mu_p * np.sum((F - Q) ** 2, axis=(1, 2)))
    return float(e)


def corotated_energy(x, tets, B, vol, mu):
    """E(x) = min_R E_hat(x, R) (Sec. 3.2, lambda = 0)."""
    F = deformation_gradients(x, tets, B)
    return pd_energy(x, tets, B, vol, mu, polar_rotation(F))


def scalar_stiffness(n, tets, B, vol, mu, subset=None):
    """One of the three identical coordinate blocks of K_el (Sec. 3.2):
    K = sum_e 2 mu Vol_e B_e B_e^T scattered to the tet's four nodes.  (n x n CSR)"""
    if subset is not None:
        tets, B, vol = tets[:, subset], B[subset], vol[subset]
    Ke = 2.0 * mu * vol[:, None, None] * np.einsum("tai,tbi->tab", B, B)   # (T,4,4)
    rows = np.repeat(tets.T, 4, axis=1).ravel()       # tets.T[t, a] repeated over b
    cols = np.tile(tets.T, (1, 4)).ravel()
    return sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(n, n))


def lumped_mass(n, tets, vol, density):
    """Lumped nodal masses for backward-Euler dynamics (Sec. 3.2 notes that PD
    applies to implicit backward Euler as well): each tet gives a quarter of
    density * Vol_e to each of its four nodes.  -> (n,)"""
    m = np.zeros(n)
    for a in range(4):
        np.add.at(m, tets[a], 0.25 * density * vol)
    return m
