"""Index ranges the dataflow factorization kernel touches, checked on the
host against the buffers the library allocates (task mapping, ragged edge
tiles, the fused right-hand-side row, the sub-diagonal tiles finished by the
diagonal tasks and their partial sums).  The ticket -> task mapping and the
accumulation depth come from the library itself (pd_dataflow_task, the code
the kernels decode their tickets with), so drift in the kernel's schedule
shows up here; no GPU work is done."""
import ctypes as C

import numpy as np
import pytest

NB = 64


def _lib():
    from paper_2008_01541_amd import load_library
    return load_library()


def schedule(n, rhs):
    """[(i, j, kend)] of every ticket, from the library."""
    lib = _lib()
    i, j, kend, ntask = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
    assert lib.pd_dataflow_task(n, rhs, -1, None, None, None, C.byref(ntask)) == 0
    out = []
    for q in range(ntask.value):
        st = lib.pd_dataflow_task(n, rhs, q, C.byref(i), C.byref(j), C.byref(kend),
                                  C.byref(ntask))
        assert st == 0
        out.append((i.value, j.value, kend.value))
    return out


def test_schedule_rejects_bad_arguments():
    lib = _lib()
    i, j, kend, ntask = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
    args = (C.byref(i), C.byref(j), C.byref(kend), C.byref(ntask))
    assert lib.pd_dataflow_task(0, 0, 0, *args) == -1
    assert lib.pd_dataflow_task(100, 2, 0, *args) == -1
    assert lib.pd_dataflow_task(100, 0, 3, *args) == -1          # 2 tiles -> 3 tasks: q = 3 out
    assert lib.pd_dataflow_task(100, 0, 2, *args) == 0
    assert (i.value, j.value, kend.value, ntask.value) == (1, 1, 0, 3)


@pytest.mark.parametrize("n", [17, 64, 65, 81, 127, 128, 200, 6498, 3249])
@pytest.mark.parametrize("rhs", [0, 1])
def test_dataflow_indices_in_bounds(n, rhs):
    nt = (n + NB - 1) // NB
    lda = (n + 15) // 16 * 16
    sched = schedule(n, rhs)
    tiles = [(i, j) for (i, j, _) in sched]
    # every tile of the lower triangle (and the right-hand-side row) exactly once
    expect = [(i, j) for j in range(nt) for i in range(j, nt)] + ([(nt, j) for j in range(nt)]
                                                                  if rhs else [])
    assert sorted(tiles) == sorted(expect)
    a_size = lda * n
    yt_size = NB * n
    flags_size = (nt + 2) * nt
    sbuf_size = nt * NB * NB
    r = np.arange(NB)[:, None]
    c = np.arange(NB)[None, :]
    for (i, j, kend) in sched:
        rrow = i == nt
        r0 = 0 if rrow else i * NB
        mr = 3 if rrow else min(NB, n - r0)
        c0 = j * NB
        mc = min(NB, n - c0)
        ldai = NB if rrow else lda
        size_i = yt_size if rrow else a_size
        assert i * nt + j < flags_size
        assert kend == (max(j - 1, 0) if i == j else j)
        sub = (not rrow) and i == j + 1
        if sub:
            # partial sum of the sub-diagonal tile: sbuf slot i, flag after the tile flags
            assert (nt + 1) * nt + i < flags_size
            assert i * NB * NB + (NB - 1) + (NB - 1) * NB < sbuf_size
        if i == j and j > 0:
            # the diagonal task finishes tile (j, j - 1): rows < mr, all 64 columns
            # (loads from rows clamped to mr - 1), reads sbuf slot j, Linv of
            # tile j - 1, and writes the transposed copy
            cs = (j - 1) * NB
            assert n - cs >= NB                       # column block j - 1 is never ragged
            idx = (r0 + np.minimum(r, mr - 1)) + (cs + c) * lda
            assert idx.max() < a_size
            idxu = (cs + r) + (r0 + c) * lda          # U(cs + r', r0 + c'), c' < mr
            assert idxu[np.broadcast_to(c < mr, idxu.shape)].max() < a_size
            assert (nt + 1) * nt + j < flags_size
            assert j * NB * NB + NB * NB - 1 < sbuf_size
            assert (j - 1) * nt + (j - 1) < flags_size
        # C build (loads from clamped rows and columns) / result store of the tile
        idx = (r0 + np.minimum(r, mr - 1)) + (c0 + np.minimum(c, mc - 1)) * ldai
        assert idx.max() < size_i
        sel = (r < mr) & (c < mc)
        idx = (r0 + r) + (c0 + c) * ldai
        assert idx[sel].max() < size_i
        if not rrow and i != j:
            # transposed copy into the upper triangle
            idxu = (c0 + c.T) + (r0 + r.T) * lda      # U(c0 + r', r0 + c')
            selu = (r.T < mr) & (c.T < mc)
            assert idxu[selu].max() < a_size
        # operand loads of the accumulation: rows < mr of Ai, rows < mc of A,
        # k < kend * NB
        if kend > 0:
            kmax = kend * NB - 1
            assert (r0 + mr - 1) + kmax * ldai < size_i
            assert (c0 + mc - 1) + kmax * lda < a_size


@pytest.mark.parametrize("n", [1, 64, 130, 200, 3249, 6498])
@pytest.mark.parametrize("rhs", [0, 1])
def test_ticket_order_respects_dependencies(n, rhs):
    """A task only waits on tasks with smaller tickets (so a persistent launch
    cannot deadlock): tiles (i, k), (j, k) for k < kend, Linv_j, the partial
    sum and tile (j, j - 1) of a diagonal task, and the right-hand-side row's
    earlier steps."""
    sched = schedule(n, rhs)
    pos = {(i, j): q for q, (i, j, _) in enumerate(sched)}
    for q, (i, j, kend) in enumerate(sched):
        deps = [(j, j)] if i != j else []
        deps += [(i, k) for k in range(kend)] + [(j, k) for k in range(kend)]
        if i == j and j > 0:
            deps += [(j, j - 1), (j - 1, j - 1)]
        for d in deps:
            if d != (i, j):
                assert d in pos and pos[d] < q, ((i, j), d)
