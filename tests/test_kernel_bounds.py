"""Host-side model of the index ranges the dataflow factorization kernel
touches (task mapping, ragged edge tiles, the fused right-hand-side row, the
sub-diagonal tiles finished by the diagonal tasks and their partial sums):
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
    flags_size = (nt + 2) * nt
    sbuf_size = nt * NB * NB
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
        sub = (not rrow) and i == j + 1
        if sub:
            # partial sum of the sub-diagonal tile: sbuf slot i, flag after the tile flags
            assert (nt + 1) * nt + i < flags_size
            assert i * NB * NB + (NB - 1) + (NB - 1) * NB < sbuf_size
        if i == j and j > 0:
            # the diagonal task finishes tile (j, j - 1): rows < mr, all 64 columns,
            # reads sbuf slot j, Linv of tile j - 1, and writes the transposed copy
            cs = (j - 1) * NB
            assert n - cs >= NB                       # column block j - 1 is never ragged
            idx = (r0 + r) + (cs + c) * lda
            assert idx[np.broadcast_to(r < mr, idx.shape)].max() < a_size
            idxu = (cs + r) + (r0 + c) * lda          # U(cs + r', r0 + c'), c' < mr
            assert idxu[np.broadcast_to(c < mr, idxu.shape)].max() < a_size
            assert (nt + 1) * nt + j < flags_size
            assert j * NB * NB + NB * NB - 1 < sbuf_size
            assert (j - 1) * nt + (j - 1) < flags_size
        # C build / result store of the tile (bounded by mr, mc)
        sel = (r < mr) & (c < mc)
        idx = (r0 + r) + (c0 + c) * ldai
        assert idx[sel].max() < size_i
        if not rrow and i != j:
            # transposed copy into the upper triangle
            idxu = (c0 + c.T) + (r0 + r.T) * lda      # U(c0 + r', r0 + c')
            selu = (r.T < mr) & (c.T < mc)
            assert idxu[selu].max() < a_size
        # operand loads of the accumulation: rows < mr of Ai, rows < mc of A,
        # k < kend*NB (the diagonal task stops one step early)
        kend = max(j - 1, 0) if i == j else j
        if kend > 0:
            kmax = kend * NB - 1
            assert (r0 + mr - 1) + kmax * ldai < size_i
            assert (c0 + mc - 1) + kmax * lda < a_size


def task_of_ticket_supplied_rhs(q, nt):
    """Ticket order when the right-hand side arrives during the factorization:
    all tiles column by column, then the right-hand-side row."""
    ntile = nt * (nt + 1) // 2
    if q < ntile:
        j, start = 0, 0
        while start + (nt - j) <= q:
            start += nt - j
            j += 1
        return j + (q - start), j
    return nt, q - ntile


@pytest.mark.parametrize("nt", [1, 2, 3, 7, 51, 102])
def test_supplied_rhs_ticket_order(nt):
    tasks = [task_of_ticket_supplied_rhs(q, nt) for q in range(nt * (nt + 1) // 2 + nt)]
    assert sorted(tasks) == sorted(dataflow_tasks(nt, 1))
    # every dependency of a task has a smaller ticket: tiles (i, k), (j, k) for
    # k < j, Linv_j, the first sub-diagonal partial sum, and Y_k (k < j) for the RHS row
    pos = {t: q for q, t in enumerate(tasks)}
    for (i, j), q in pos.items():
        deps = [(j, j)] if i != j else []
        deps += [(i, k) for k in range(j)] + [(j, k) for k in range(j)]
        if i == j and j > 0:
            deps.append((j, j - 1))
        for d in deps:
            if d in pos and d != (i, j):
                assert pos[d] < q, ((i, j), d)
