"""Host-side model of the index ranges the dataflow factorization kernel
touches (task mapping, ragged edge tiles, the fused right-hand-side row):
every load and store must stay inside the buffers the library allocates."""
import numpy as np
import pytest

NB = 64


def dataflow_tasks(nt, rhs):
    out = []
    for j in range(nt):
        for i in range(j, nt + (1 if rhs else 0)):
            out.append((i, j))
    return out


def task_of_ticket(q, nt, rhs):
    j, start = 0, 0
    while start + (nt - j + rhs) <= q:
        start += nt - j + rhs
        j += 1
    return j + (q - start), j


@pytest.mark.parametrize("n", [17, 64, 65, 81, 127, 128, 200, 6498, 3249])
@pytest.mark.parametrize("rhs", [0, 1])
def test_dataflow_indices_in_bounds(n, rhs):
    nt = (n + NB - 1) // NB
    lda = (n + 15) // 16 * 16
    ntask = nt * (nt + 1) // 2 + rhs * nt
    assert [task_of_ticket(q, nt, rhs) for q in range(ntask)] == dataflow_tasks(nt, rhs)
    a_size = lda * n
    yt_size = NB * n
    flags_size = (nt + 1) * nt
    r = np.arange(NB)[:, None]
    c = np.arange(NB)[None, :]
    for (i, j) in dataflow_tasks(nt, rhs):
        rrow = i == nt
        r0 = 0 if rrow else i * NB
        mr = 3 if rrow else min(NB, n - r0)
        c0 = j * NB
        mc = min(NB, n - c0)
        ldai = NB if rrow else lda
        size_i = yt_size if rrow else a_size
        assert i * nt + j < flags_size
        # C build / result store of the tile (bounded by mr, mc)
        sel = (r < mr) & (c < mc)
        idx = (r0 + r) + (c0 + c) * ldai
        assert idx[sel].max() < size_i
        if not rrow and i != j:
            # transposed copy into the upper triangle
            idxu = (c0 + c.T) + (r0 + r.T) * lda      # U(c0 + r', r0 + c')
            selu = (r.T < mr) & (c.T < mc)
            assert idxu[selu].max() < a_size
        # operand loads of the accumulation: rows < mr of Ai, rows < mc of A, k < j*NB
        if j > 0:
            kmax = j * NB - 1
            assert (r0 + mr - 1) + kmax * ldai < size_i
            assert (c0 + mc - 1) + kmax * lda < a_size
