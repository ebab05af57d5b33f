"""Partitioned global step and its Schur complement (paper Sec. 4.2-4.4).

Free nodes are split into collision-safe x1 and collision-prone x2
(Sec. 4.2, eq. block1).  The partial Cholesky factorization (eq. par_chol)
leaves the Schur complement Sigma = A22 - A21 A11^-1 A12; since collisions
only add C22 to the x2-x2 block, Sigma_col = Sigma_no-col + C22 (eq. k22).
The three-step solve (eq. par_chol2, Steps 1-3) is the forward substitution
y2 = b2 - A21 A11^-1 b1, the dense solve Sigma z2 = y2 and the back
substitution x1 = A11^-1 (b1 - A12 z2).

Here A11^-1 is applied through a sparse LU (SuperLU, symmetric ordering) of
A11 and nothing else: no level structure, no explicit inverses.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def sparse_factor(A):
    """Factor a sparse SPD matrix once; returns an object with .solve(b)."""
    A = sp.csc_matrix(A)
    return spla.splu(A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                     options=dict(SymmetricMode=True))


def blocks(K, i1, i2):
    """Split a (free-node) matrix into A11, A12, A21, A22 for index sets i1, i2."""
    K = sp.csr_matrix(K)
    K1 = K[i1]
    K2 = K[i2]
    return K1[:, i1], K1[:, i2], K2[:, i1], K2[:, i2]


def schur_complement(A11, A12, A21, A22, lu11=None):
    """Dense Sigma = A22 - A21 A11^-1 A12 (eq. par_chol).  Only the columns of
    A12 that have a nonzero are solved for."""
    if lu11 is None:
        lu11 = sparse_factor(A11)
    A12 = sp.csc_matrix(A12)
    S = A22.toarray().astype(np.float64)
    if A12.shape[0] == 0:
        return S
    cols = np.nonzero(np.diff(A12.indptr))[0]
    if cols.size:
        X = lu11.solve(A12[:, cols].toarray())         # A11^-1 A12[:, cols]
        S[:, cols] -= sp.csr_matrix(A21) @ X
    return S


def schur_apply(A11_lu, A12, A21, A22, v):
    """Sigma v = A22 v - A21 (A11^-1 (A12 v)) without forming Sigma (one sparse solve)."""
    v = np.asarray(v, dtype=np.float64)
    w = A12 @ v
    return A22 @ v - A21 @ A11_lu.solve(w)


def forward_sub(A11_lu, A21, b1, b2):
    """Step 1 of the three-step solve, in the form of Alg. 1 step 3.1:
    returns (A11^-1 b1, y2 = b2 - A21 A11^-1 b1)."""
    w = A11_lu.solve(b1)
    return w, b2 - A21 @ w


def back_sub(A11_lu, A12, b1, z2):
    """Step 3: x1 = A11^-1 (b1 - A12 z2)."""
    return A11_lu.solve(b1 - A12 @ z2)
