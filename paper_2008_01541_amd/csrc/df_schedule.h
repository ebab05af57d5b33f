// Task schedule of the single-launch dataflow Cholesky (FP64 and low
// precision): the ticket -> tile mapping and the accumulation depth of a
// task.  Host and device: the kernels decode their tickets with it, and the
// library exports it (pd_dataflow_task) so that the host can check the index
// ranges of every task against the buffers.
#pragma once
#include <hip/hip_runtime.h>

namespace pdk {

// Ticket q -> tile (i, j), 0 <= j <= i < nt, i == nt for the right-hand-side
// row.  Tickets go column by column; in column j the diagonal tile first,
// then the tiles below it in order, then (rhs = 1) the right-hand-side row.
__host__ __device__ inline void df_task_of_ticket(int q, int nt, int rhs, int& i, int& j) {
  int jj = 0, start = 0;
  while (start + (nt - jj + rhs) <= q) start += nt - jj++ + rhs;
  j = jj;
  i = jj + (q - start);
}

// Number of tasks: nt (nt + 1) / 2 tiles, plus nt with a right-hand side.
__host__ __device__ inline int df_task_count(int nt, int rhs) { return nt * (nt + 1) / 2 + rhs * nt; }

// 64-column steps accumulated by task (i, j): k < j, and k < j - 1 for the
// diagonal task (it finishes the sub-diagonal tile's last step itself).
__host__ __device__ inline int df_task_kend(int i, int j) {
  return i == j ? (j > 0 ? j - 1 : 0) : j;
}

}  // namespace pdk
