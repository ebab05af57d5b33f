"""pd_chol_factor_noalloc (static workspace, no allocation) against
pd_chol_factor (handle workspace) and numpy: two calls in a row, the second
with a smaller matrix, bit for bit equal to the handle's factorization (the
same kernel and task order); the size limit is rejected before anything is
enqueued."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    m = rng.normal(size=(n, n))
    return m @ m.T / n + np.eye(n)


def _to_device(torch, a, lda):
    n = a.shape[0]
    buf = np.full((n, lda), np.nan)          # row c = column c of the column-major matrix
    buf[:, :n] = a.T
    return torch.tensor(buf.reshape(-1), device="cuda")


def test_noalloc_factor_matches_handle_factor():
    import torch
    from paper_2008_01541_amd import DenseCholesky, chol_factor_noalloc
    assert torch.cuda.is_available()
    stream = torch.cuda.current_stream()
    chol = DenseCholesky(1500)
    for n, pad in [(1300, 12), (257, 3)]:          # the second call is smaller
        lda = (n + pad + 15) // 16 * 16
        a = _spd(n, n)
        d_ref = _to_device(torch, a, lda)
        d_na = d_ref.clone()
        assert chol.factor(d_ref, n, lda) == 0
        assert chol_factor_noalloc(d_na, n, lda, stream=stream) == 0
        torch.cuda.synchronize()
        assert torch.equal(torch.nan_to_num(d_na, nan=7.0), torch.nan_to_num(d_ref, nan=7.0))
        out = d_na.cpu().numpy().reshape(n, lda)
        lo = np.tril(out[:, :n].T)
        ref = np.linalg.cholesky(a)
        assert np.abs(lo - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.isnan(out[:, n:]).all()          # padding rows untouched
    chol.close()


def test_noalloc_factor_reports_bad_pivot_and_limits():
    import ctypes
    import torch
    from paper_2008_01541_amd import PD_CHOL_NOALLOC_MAX_N, chol_factor_noalloc, load_library
    n, lda = 200, 208
    a = _spd(n, 3)
    a[150, 150] = -1.0
    dA = _to_device(torch, a, lda)
    assert chol_factor_noalloc(dA, n, lda) == 151     # 1-based first non-positive pivot
    lib = load_library()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    big = PD_CHOL_NOALLOC_MAX_N + 1
    info = ctypes.c_int32(-7)
    # size beyond the static workspace, bad lda, offset view: rejected, nothing enqueued
    assert lib.pd_chol_factor_noalloc(ctypes.c_void_p(dA.data_ptr()), big + 15, big, 0, st,
                                      ctypes.byref(info)) == -1
    assert lib.pd_chol_factor_noalloc(ctypes.c_void_p(dA.data_ptr()), 201, n, 0, st,
                                      ctypes.byref(info)) == -1
    assert lib.pd_chol_factor_noalloc(ctypes.c_void_p(dA.data_ptr() + 8), lda, n, 0, st,
                                      ctypes.byref(info)) == -1
    assert info.value == -7
    # the workspace still serves a good call afterwards
    b = _spd(n, 4)
    dB = _to_device(torch, b, lda)
    assert chol_factor_noalloc(dB, n, lda) == 0
    lo = np.tril(dB.cpu().numpy().reshape(n, lda)[:, :n].T)
    assert np.abs(lo - np.linalg.cholesky(b)).max() <= 1e-12 * np.abs(lo).max()
