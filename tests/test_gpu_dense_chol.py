"""Standalone dense FP64 Cholesky (pd_chol_*) against numpy.linalg.cholesky:
orders around the 64-wide tile edges, padded leading dimensions whose
padding rows hold NaN (never read, never written), the transposed copy in the
upper triangle, the first non-positive pivot, and argument checks."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    m = rng.normal(size=(n, n))
    return m @ m.T / n + np.eye(n)


def _to_device(torch, a, lda):
    n = a.shape[0]
    buf = np.full((n, lda), np.nan)          # row c = column c of the column-major matrix
    buf[:, :n] = a.T
    return torch.tensor(buf.reshape(-1), device="cuda")


@pytest.mark.parametrize("n,pad", [(1, 15), (63, 1), (64, 0), (65, 15), (130, 14), (700, 4)])
def test_dense_cholesky_matches_numpy(torch_cuda, n, pad):
    from paper_2008_01541_amd import DenseCholesky
    lda = (n + pad + 15) // 16 * 16
    a = _spd(n, n)
    dA = _to_device(torch_cuda, a, lda)
    chol = DenseCholesky(1000)
    assert chol.factor(dA, n, lda) == 0
    out = dA.cpu().numpy().reshape(n, lda)
    lo = np.tril(out[:, :n].T)                 # lower triangle, column-major view
    up = np.triu(out[:, :n].T, 1)
    ref = np.linalg.cholesky(a)
    assert np.abs(lo - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(up, np.triu(lo.T, 1))
    assert np.isnan(out[:, n:]).all()          # padding rows untouched
    chol.close()


def test_dense_cholesky_reports_first_bad_pivot(torch_cuda):
    from paper_2008_01541_amd import DenseCholesky
    n, lda = 150, 160
    a = np.eye(n) * 4.0
    a[70, 70] = -1.0
    a[120, 120] = 0.0
    dA = _to_device(torch_cuda, a, lda)
    chol = DenseCholesky(n)
    assert chol.factor(dA, n, lda) == 71
    chol.close()


def test_dense_cholesky_rejects_bad_arguments(torch_cuda):
    from paper_2008_01541_amd import DenseCholesky, PDError
    chol = DenseCholesky(100)
    dA = torch_cuda.zeros(128 * 128, dtype=torch_cuda.float64, device="cuda")
    with pytest.raises(PDError):
        chol.factor(dA[: 100 * 100], 100, 100)      # lda not a multiple of 16
    with pytest.raises(PDError):
        chol.factor(dA, 128, 128)                   # n above n_max
    with pytest.raises(PDError):
        chol.factor(dA[1: 1 + 100 * 112], 100, 112)  # view not aligned to 128 bytes
    with pytest.raises(PDError):
        chol.factor(dA[8: 8 + 100 * 112], 100, 112)  # 64 bytes: still not a line
    chol.close()


@pytest.mark.parametrize("n_wg", [1, 3])
def test_dense_cholesky_few_workgroups(torch_cuda, n_wg):
    """Every task waits only on tasks with smaller tickets, so the persistent
    schedule completes with any number of workgroups, one included."""
    from paper_2008_01541_amd import DenseCholesky
    n, lda = 300, 304
    a = _spd(n, 11)
    dA = _to_device(torch_cuda, a, lda)
    chol = DenseCholesky(n)
    assert chol.factor(dA, n, lda, n_workgroups=n_wg) == 0
    lo = np.tril(dA.cpu().numpy().reshape(n, lda)[:, :n].T)
    ref = np.linalg.cholesky(a)
    assert np.abs(lo - ref).max() <= 1e-12 * np.abs(ref).max()
    chol.close()


def test_dense_cholesky_order_12155_matches_numpy(torch_cuda):
    """The order of the self-contact slit's region system (n = 12,155, 190
    tiles, ragged last tile) on a seeded SPD matrix of the benchmark's class
    (symmetric U[-0.5, 0.5] entries plus n/2 on the diagonal): the factor
    element-wise against numpy.linalg.cholesky and the residual
    ||L L^T v - A v|| / ||A v|| recomputed on the host."""
    from paper_2008_01541_amd import DenseCholesky
    n, lda = 12155, 12160
    rng = np.random.default_rng(12155)
    a = rng.uniform(-0.5, 0.5, size=(n, n))
    a += a.T
    a *= 0.5
    a[np.diag_indices(n)] += 0.5 * n
    buf = np.zeros((n, lda))
    buf[:, :n] = a                              # symmetric: row c = column c
    dA = torch_cuda.tensor(buf.reshape(-1), device="cuda")
    del buf
    chol = DenseCholesky(n)
    assert chol.factor(dA, n, lda) == 0
    chol.close()
    lo = np.tril(dA.cpu().numpy().reshape(n, lda)[:, :n].T)
    del dA
    ref = np.linalg.cholesky(a)
    assert np.abs(lo - ref).max() <= 1e-12 * np.abs(ref).max()
    v = rng.normal(size=(n, 3))
    av = a @ v
    assert np.linalg.norm(lo @ (lo.T @ v) - av) <= 1e-14 * np.linalg.norm(av)
