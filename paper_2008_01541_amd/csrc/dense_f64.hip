// Dense FP64 kernels for gfx950: tiled Cholesky of the Schur system and of the
// interior level blocks, triangular inverse, symmetric inverse assembly,
// three-right-hand-side triangular solves and the symmetric matrix-vector
// product.  Tiles are NB x NB (NB = 64), column-major.  Products run on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64) with operands staged through LDS.
#include <algorithm>
#include <climits>
#include "common.h"
#include "tile_factor_f64.h"
#include "publish.h"
#include "df_schedule.h"

namespace pdk {

constexpr int KC = 16;           // K-chunk staged through LDS per step

struct Acc {                     // one wave's 32 x 32 share of a 64 x 64 tile
  double4_t c[2][2];
};

__device__ inline void acc_zero(Acc& a) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) a.c[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
}

// Tile-local coordinates of accumulator element (mb, nb, q) of this lane.
// The product is issued with the column operand in the MFMA "A" slot, so the
// 16x16 result block D[i][j] (lane l, register q: i = l/16 + 4q, j = l%16)
// holds C(row = j, col = i): consecutive lanes walk down a column of C, which
// makes loads and stores of C coalesced.
__device__ inline int acc_row(int mb) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  return (w >> 1) * 32 + mb * 16 + (lane & 15);
}
__device__ inline int acc_col(int nb, int q) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  return (w & 1) * 32 + nb * 16 + (lane >> 4) + 4 * q;
}

// Ls[k][r] = op(G)(r0 + r, k0 + k) for r < NB, k < KC; zero outside (mr, kr).
// TRANS = false: element (r, k) at G[r + k*ld]; TRANS = true: at G[k + r*ld].
template <bool TRANS>
__device__ inline void load_chunk(double (*Ls)[LDS_LD], const double* __restrict__ G, long ld,
                                  int r0, int k0, int mr, int kr) {
  const int t = threadIdx.x;
  if (!TRANS) {
    const int r = t & 63;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = (t >> 6) + 4 * q;
      double v = 0.0;
      if (r < mr && k < kr) v = G[(long)(r0 + r) + (long)(k0 + k) * ld];
      Ls[k][r] = v;
    }
  } else {
    const int k = t & 15;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = (t >> 4) + 16 * q;
      double v = 0.0;
      if (r < mr && k < kr) v = G[(long)(k0 + k) + (long)(r0 + r) * ld];
      Ls[k][r] = v;
    }
  }
}

// acc(r, c) += sum_{kk < K} Ahat(r, kk) * Bhat(c, kk) where
// Ahat(r, kk) = opA(A)(ar0 + r, ak0 + kk) and Bhat(c, kk) = opB(B)(br0 + c, bk0 + kk);
// rows r >= amr and cols c >= bmr read as zero.
template <bool TA, bool TB>
__device__ void gemm_acc(Acc& acc, double (*As)[LDS_LD], double (*Bs)[LDS_LD],
                         const double* __restrict__ A, long lda, int ar0, int amr, int ak0,
                         const double* __restrict__ B, long ldb, int br0, int bmr, int bk0,
                         int K) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
  for (int kk = 0; kk < K; kk += KC) {
    __syncthreads();
    load_chunk<TA>(As, A, lda, ar0, ak0 + kk, amr, K - kk);
    load_chunk<TB>(Bs, B, ldb, br0, bk0 + kk, bmr, K - kk);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int k = ks * 4 + (lane >> 4);
      const double a0 = As[k][wr * 32 + (lane & 15)];
      const double a1 = As[k][wr * 32 + 16 + (lane & 15)];
      const double b0 = Bs[k][wc * 32 + (lane & 15)];
      const double b1 = Bs[k][wc * 32 + 16 + (lane & 15)];
      acc.c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a0, acc.c[0][0], 0, 0, 0);
      acc.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, acc.c[0][1], 0, 0, 0);
      acc.c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a1, acc.c[1][0], 0, 0, 0);
      acc.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, acc.c[1][1], 0, 0, 0);
    }
  }
}

__device__ inline void tri_index(int b, int& i, int& j) {
  // b -> (i, j) with 0 <= j <= i, b = i (i + 1) / 2 + j
  int ii = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= b) ++ii;
  while (ii * (ii + 1) / 2 > b) --ii;
  i = ii;
  j = b - ii * (ii + 1) / 2;
}

// An empty asm that takes all sixteen values: every load feeding them is
// issued before it and they are waited for once, instead of the compiler
// turning each select of a loaded value into a branch with its own wait.
__device__ inline void regs_ready(double (&v)[16]) {
  asm volatile(""
               : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]),
                 "+v"(v[6]), "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11]),
                 "+v"(v[12]), "+v"(v[13]), "+v"(v[14]), "+v"(v[15]));
}

// ---------------------------------------------------------------------------
// Single-launch tiled Cholesky.  Persistent workgroups claim lower tiles in
// column-major order from a ticket counter; the workgroup that owns tile
// (i, j) accumulates sum_{k<j} L_ik L_jk^T on the matrix cores as soon as each
// pair of operand tiles is published (operands double-buffered through LDS
// with the next chunk's loads in flight during the current products), then
// either factors the diagonal tile (blocked, in LDS) and publishes L_jj and its
// inverse, or waits for Linv_jj and forms L_ij = (A_ij - acc) Linv_jj^T.  Each
// factor tile is also written transposed into the upper triangle, so the
// backward substitution reads L^T with unit stride.  A task only waits on
// tasks with a smaller ticket, all of which belong to running workgroups, so
// the schedule cannot deadlock; waits are bounded and raise *err instead.
// Resets the task ticket and advances the launch epoch kept in ctr[1]; the
// factorization kernel reads the epoch from memory, so a captured graph that
// replays the pair still gets a fresh epoch every time.
__global__ void k_reset_counter(unsigned* ctr) {
  ctr[0] = 0u;
  ctr[1] = ctr[1] + 1u;
}

// acc += sum_{k<kend} L_ik L_jk^T, one 64-deep k-step at a time.  The two
// operand tiles of step k+1 are loaded into registers while the products of
// step k run from LDS, and the ready flags of step k+2 are read while step
// k+1 is loaded, so neither the flag round trip nor the operand latency sits
// on the path when the producers are ahead.
__device__ bool df_accumulate(Acc& acc, double (*As)[LDS_LD], double (*Bs)[LDS_LD],
                              const double* __restrict__ Ar, int ldar, int r0, int mr,
                              const double* __restrict__ A, int lda, int c0,
                              int mc, int i, int j, int kend, int nt, const int* flags, int epoch,
                              int* err, int* s_ok, const int* mark) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int r = t & 63;
  const int kq = __builtin_amdgcn_readfirstlane(t >> 6);   // the wave index, uniform: addresses stay scalar
  if (kend == 0) return true;
  double ra[16], rb[16];
  auto load_tile = [&](int k) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const long kc = (long)(k * NB + kq + 4 * q);
      ra[q] = (r < mr) ? Ar[(long)(r0 + r) + kc * ldar] : 0.0;
      rb[q] = (r < mc) ? A[(long)(c0 + r) + kc * lda] : 0.0;
    }
  };
  int fi = 0, fj = 0;          // thread 0: flags of the next step, read ahead
  int fm = 0;                  // thread 0: this unit's courtesy mark (mark != NULL)
  if (t == 0) {
    if (!df_wait(&flags[i * nt], epoch, err) || !df_wait(&flags[j * nt], epoch, err)) *s_ok = 0;
  }
  __syncthreads();
  if (!*s_ok) return false;
  load_tile(0);
  if (t == 0 && kend > 1) {
    fi = __hip_atomic_load(&flags[i * nt + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    fj = __hip_atomic_load(&flags[j * nt + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  for (int k = 0; k < kend; ++k) {
    __syncthreads();                         // previous step's products are done with LDS
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      As[kq + 4 * q][r] = ra[q];
      Bs[kq + 4 * q][r] = rb[q];
    }
    const bool nxt = k + 1 < kend;
    if (t == 0 && fm == epoch) cu_pause(mark, epoch);
    if (t == 0 && nxt && (fi != epoch || fj != epoch)) {
      if (!df_wait(&flags[i * nt + k + 1], epoch, err) ||
          !df_wait(&flags[j * nt + k + 1], epoch, err))
        *s_ok = 0;
    }
    __syncthreads();
    if (!*s_ok) return false;
    if (nxt) {
      load_tile(k + 1);
      if (t == 0 && k + 2 < kend) {
        fi = __hip_atomic_load(&flags[i * nt + k + 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        fj = __hip_atomic_load(&flags[j * nt + k + 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (t == 0 && mark) fm = __hip_atomic_load(mark, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int ks = 0; ks < NB / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      const double a0 = As[kk][wr * 32 + (lane & 15)];
      const double a1 = As[kk][wr * 32 + 16 + (lane & 15)];
      const double b0 = Bs[kk][wc * 32 + (lane & 15)];
      const double b1 = Bs[kk][wc * 32 + 16 + (lane & 15)];
      acc.c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a0, acc.c[0][0], 0, 0, 0);
      acc.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, acc.c[0][1], 0, 0, 0);
      acc.c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a1, acc.c[1][0], 0, 0, 0);
      acc.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, acc.c[1][1], 0, 0, 0);
    }
  }
  return true;
}

// acc(r, c) += sum_kk As[kk][r] Bs[kk][c] over one 64-deep block in LDS (this
// wave's 32 x 32 share, the layout of Acc).
__device__ inline void lds_product(Acc& acc, double (*As)[LDS_LD], double (*Bs)[LDS_LD]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
#pragma unroll 4
  for (int ks = 0; ks < NB / 4; ++ks) {
    const int k = ks * 4 + (lane >> 4);
    const double a0 = As[k][wr * 32 + (lane & 15)];
    const double a1 = As[k][wr * 32 + 16 + (lane & 15)];
    const double b0 = Bs[k][wc * 32 + (lane & 15)];
    const double b1 = Bs[k][wc * 32 + 16 + (lane & 15)];
    acc.c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a0, acc.c[0][0], 0, 0, 0);
    acc.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, acc.c[0][1], 0, 0, 0);
    acc.c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a1, acc.c[1][0], 0, 0, 0);
    acc.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, acc.c[1][1], 0, 0, 0);
  }
}

// Triangular right factor: acc(r, c) = sum_k As[k][r] Bs[k][c] where
// Bs[k][c] = 0 for k > c (Bs holds the transpose of a lower-triangular
// tile), so column block cb only takes the k-blocks 0..cb.  The waves of
// column half 0 own column blocks 0 and 3 and those of half 1 blocks 1 and 2
// (40 products per wave instead of 64); accumulator block nb of this wave is
// column block tri_cb(nb).  Only exact zeros are skipped, so the result is
// the full product's.
__device__ inline int tri_cb(int nb) {
  const int wc = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) & 1;
  return wc ? 1 + nb : 3 * nb;
}
__device__ inline int tri_col(int nb, int q) {
  return 16 * tri_cb(nb) + (int)((threadIdx.x & 63) >> 4) + 4 * q;
}
__device__ inline void lds_product_tri(Acc& acc, double (*As)[LDS_LD], double (*Bs)[LDS_LD]) {
  const int lane = threadIdx.x & 63;
  const int wr = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) >> 1;
  const int cb0 = tri_cb(0), cb1 = tri_cb(1);
  const int kA = 4 * (cb0 + 1), kB = 4 * (cb1 + 1);     // 4-deep steps per block, kA < kB
#pragma unroll 4
  for (int ks = 0; ks < kA; ++ks) {
    const int k = ks * 4 + (lane >> 4);
    const double a0 = As[k][wr * 32 + (lane & 15)];
    const double a1 = As[k][wr * 32 + 16 + (lane & 15)];
    const double b0 = Bs[k][16 * cb0 + (lane & 15)];
    const double b1 = Bs[k][16 * cb1 + (lane & 15)];
    acc.c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a0, acc.c[0][0], 0, 0, 0);
    acc.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, acc.c[0][1], 0, 0, 0);
    acc.c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a1, acc.c[1][0], 0, 0, 0);
    acc.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, acc.c[1][1], 0, 0, 0);
  }
#pragma unroll 4
  for (int ks = kA; ks < kB; ++ks) {
    const int k = ks * 4 + (lane >> 4);
    const double a0 = As[k][wr * 32 + (lane & 15)];
    const double a1 = As[k][wr * 32 + 16 + (lane & 15)];
    const double b1 = Bs[k][16 * cb1 + (lane & 15)];
    acc.c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, acc.c[0][1], 0, 0, 0);
    acc.c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, acc.c[1][1], 0, 0, 0);
  }
}

// T[c][r] = sign * acc(r, c)
__device__ inline void acc_to_lds(const Acc& acc, double (*T)[LDS_LD], double sign) {
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) T[acc_col(nb, qq)][acc_row(mb)] = sign * acc.c[mb][nb][qq];
}

// T[e >> 6][e & 63] = src[e] for the 4096 elements of a 64 x 64 tile, with
// all sixteen loads of a thread in flight before the LDS writes.
__device__ inline void stage_tile(double (*T)[LDS_LD], const double* __restrict__ src) {
  const int t = threadIdx.x;
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = src[t + 256 * q];
#pragma unroll
  for (int q = 0; q < 16; ++q) T[(t >> 6) + 4 * q][t & 63] = v[q];
}

// Task kinds in column j (tickets in this order):
//  * diagonal (j, j): accumulates k < j - 1, then finishes the sub-diagonal
//    tile itself, L_{j,j-1} = (A_{j,j-1} - S_j) Linv_{j-1}^T with the partial
//    sum S_j of the task below, adds its last product and factors the tile.
//    The first sub-diagonal tile thus never takes a hand-off of its own on the
//    chain diag(j-1) -> diag(j), the critical path of the factorization.
//  * sub-diagonal (j + 1, j): S_{j+1} = sum_{k<j} L_{j+1,k} L_{j,k}^T into
//    the workspace sbuf (published with its own flag, no Linv wait).
//  * (i, j), i >= j + 2: accumulates k < j, waits for Linv_jj, forms
//    L_ij = (A_ij - acc) Linv_jj^T.
//  * with Yt != NULL the three right-hand sides ride along as an extra tile
//    row (Yt: 64 x n, column-major, rows 0..2 = g^T on entry): its tasks
//    compute Y_j = (G_j - sum_{k<j} Y_k L_jk^T) Linv_jj^T, i.e. the forward
//    substitution y = L^-1 g, on the same schedule.
// Flags: nt x nt for the tiles, nt more for the right-hand-side row, nt more
// for the partial sums.
__global__ __launch_bounds__(256, 2) void k_potrf_dataflow(double* A, int lda, int n, int nt,
                                                           double* linv_ws, double* sbuf,
                                                           int* flags, unsigned* ticket, int* info,
                                                           int* err, double* Yt, int* cu_marks) {
  const int epoch = (int)ticket[1];
  const int rhs = Yt != nullptr ? 1 : 0;
  int* const mark = cu_marks ? cu_marks + cu_slot() : nullptr;
  int* sflags = flags + (nt + 1) * nt;
  // two 64 x 68 double tiles (69,632 bytes): operands of the accumulation,
  // then the tile and its inverse / Linv during the finishing step
  __shared__ double buf0[NB][LDS_LD];
  __shared__ double buf1[NB][LDS_LD];
  __shared__ int s_task, s_ok;
  const int t = threadIdx.x;
  const int ntask = df_task_count(nt, rhs);
  for (;;) {
    __syncthreads();
    if (t == 0) {
      s_task = (int)atomicAdd(ticket, 1u);
      s_ok = 1;
    }
    __syncthreads();
    const int q = s_task;
    if (q >= ntask) return;
    int i, j;
    df_task_of_ticket(q, nt, rhs, i, j);
    const bool rrow = (i == nt);
    const bool diag = (i == j), sub = !rrow && i == j + 1;
    double* Ai = rrow ? Yt : A;
    const int ldai = rrow ? NB : lda;
    const int r0 = rrow ? 0 : i * NB, c0 = j * NB;
    const int mr = rrow ? 3 : min(NB, n - r0), mc = min(NB, n - c0);
    // the diagonal chain issues first
    const bool critical = diag || sub;
    if (critical) __builtin_amdgcn_s_setprio(2);
    // acc <- -A_ij (read now so that the load is off the path after the last
    // product; padding: identity on the diagonal tile, zero elsewhere), or 0
    Acc acc;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int r = acc_row(mb), c = acc_col(nb, qq);
          acc.c[mb][nb][qq] = sub ? 0.0
                            : (r < mr && c < mc)
                                ? -coherent_load(&Ai[(long)(r0 + r) + (long)(c0 + c) * ldai])
                                : ((diag && r == c) ? -1.0 : 0.0);
        }
    const int kend = df_task_kend(i, j);
    if (!df_accumulate(acc, buf0, buf1, Ai, ldai, r0, mr, A, lda, c0, mc, i, j, kend, nt, flags,
                       epoch, err, &s_ok, critical ? nullptr : mark))
      return;
    // the diagonal task's local phase: no waits from here to the inverse's flag
    const auto mark_unit = [&]() {
      if (t == 0 && mark) __hip_atomic_store(mark, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    if (sub) {
      double* Sb = sbuf + (long)i * NB * NB;
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq)
            coherent_store(&Sb[acc_row(mb) + NB * acc_col(nb, qq)], acc.c[mb][nb][qq]);
      publish_flag(&sflags[i], epoch);
      __builtin_amdgcn_s_setprio(0);
      continue;
    }
    if (diag && j > 0) {
      // tile (j, j - 1): rows of block j (mr of them), 64 columns
      const int cs = (j - 1) * NB;
      __syncthreads();                             // last products done with buf0
      {
        const int r = t & 63;
        double v[16];
#pragma unroll
        for (int qq = 0; qq < 16; ++qq)
          v[qq] = coherent_load(&A[(long)(r0 + min(r, mr - 1)) + (long)(cs + (t >> 6) + 4 * qq) * lda]);
        regs_ready(v);
#pragma unroll
        for (int qq = 0; qq < 16; ++qq) buf0[(t >> 6) + 4 * qq][r] = (r < mr) ? v[qq] : 0.0;
      }
      // the partial sum is usually published well before Linv_{j-1}: take it
      // (each thread the elements it loaded above) while Linv is awaited
      if (t == 0 && !df_wait(&sflags[j], epoch, err)) s_ok = 0;
      __syncthreads();
      if (!s_ok) return;
      {
        const double* Sb = sbuf + (long)j * NB * NB;
        double v[16];
#pragma unroll
        for (int qq = 0; qq < 16; ++qq) v[qq] = Sb[t + 256 * qq];
#pragma unroll
        for (int qq = 0; qq < 16; ++qq) buf0[(t >> 6) + 4 * qq][t & 63] -= v[qq];   // S(r, c)
      }
      if (t == 0 && !df_wait(&flags[(j - 1) * nt + (j - 1)], epoch, err)) s_ok = 0;
      __syncthreads();
      if (!s_ok) return;
      mark_unit();
      stage_tile(buf1, linv_ws + (long)(j - 1) * NB * NB);   // buf1[kk][c] = Linv(c, kk)
      __syncthreads();
      Acc l;                                       // columns tri_col(nb, q)
      acc_zero(l);
      lds_product_tri(l, buf0, buf1);              // L = S Linv^T
      __syncthreads();
      // L into buf1 (the tile factor's inverse slot, which takes the last
      // rank-64 update C -= L L^T block by block while its first diagonal
      // block is factored), C without that term into buf0
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) buf1[tri_col(nb, qq)][acc_row(mb)] = l.c[mb][nb][qq];
      acc_to_lds(acc, buf0, -1.0);
      // the tile goes to memory straight from the registers (each lane's
      // sixteen rows of 16-lane runs); the tile factor publishes its flag
      // once the stores have drained
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int r = acc_row(mb), c = tri_col(nb, qq);
            if (r < mr) coherent_store(&A[(long)(r0 + r) + (long)(cs + c) * lda], l.c[mb][nb][qq]);
          }
      // (its transposed copy is written after the tile, off the critical path)
    } else {
      __syncthreads();
      acc_to_lds(acc, buf0, -1.0);                 // C = A_ij - sum_k L_ik L_jk^T
    }
    __syncthreads();
    if (diag) {
      if (j == 0) mark_unit();
      factor_tile_blocked(buf0, buf1, mr, r0, info, j > 0 ? &flags[j * nt + (j - 1)] : nullptr,
                          epoch);
      // only the inverse is read inside this launch: publish it first, then
      // write L (lower) and its transposed copy (strictly upper) for the solves
      double* Li = linv_ws + (long)j * NB * NB;
      for (int e = t; e < NB * NB; e += 256) coherent_store(&Li[e], buf1[e >> 6][e & 63]);
      // the mark is cleared before the flag is stored (publish_flag waits for
      // both), so the next diagonal task, which may run on this unit, sets its
      // own mark after this clear
      if (t == 0 && mark) __hip_atomic_store(mark, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      publish_flag(&flags[i * nt + j], epoch);
      for (int e = t; e < NB * NB; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (r < mr && c < mr)
          A[(long)(r0 + r) + (long)(r0 + c) * lda] = (r >= c) ? buf0[c][r] : buf0[r][c];
      }
      if (j > 0) {
        // transposed copy of the sub-diagonal tile finished above, read back
        // (coalesced, coherent) and turned through LDS:
        // U(cs + r', r0 + c') = L(r0 + c', cs + r')
        const int cs = (j - 1) * NB;
        {
          const int r = t & 63;
          double v[16];
#pragma unroll
          for (int qq = 0; qq < 16; ++qq)
            v[qq] = coherent_load(&A[(long)(r0 + min(r, mr - 1)) + (long)(cs + (t >> 6) + 4 * qq) * lda]);
          regs_ready(v);
#pragma unroll
          for (int qq = 0; qq < 16; ++qq) buf1[(t >> 6) + 4 * qq][r] = (r < mr) ? v[qq] : 0.0;
        }
        __syncthreads();
        for (int e = t; e < NB * NB; e += 256) {
          const int r = e & 63, c = e >> 6;
          if (c < mr) A[(long)(cs + r) + (long)(r0 + c) * lda] = buf1[r][c];
        }
      }
    } else {
      if (t == 0 && !df_wait(&flags[j * nt + j], epoch, err)) s_ok = 0;
      __syncthreads();
      if (!s_ok) return;
      stage_tile(buf1, linv_ws + (long)j * NB * NB);   // buf1[kk][c] = Linv(c, kk)
      __syncthreads();
      acc_zero(acc);
      lds_product(acc, buf0, buf1);
      // stored straight from the registers (the right-hand-side row also runs
      // over the last, ragged, column block); the LDS copy is for the
      // transposed copy below
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int r = acc_row(mb), c = acc_col(nb, qq);
            if (r < mr && c < mc)
              coherent_store(&Ai[(long)(r0 + r) + (long)(c0 + c) * ldai], acc.c[mb][nb][qq]);
          }
      __syncthreads();
      acc_to_lds(acc, buf0, 1.0);
      publish_flag(&flags[i * nt + j], epoch);
      // transposed copy, read only by the backward solve after this launch:
      // U(c0 + r', r0 + c') = L(r0 + c', c0 + r') with r' = e & 63, c' = e >> 6
      if (!rrow) {
        for (int e = t; e < NB * NB; e += 256) {
          const int r = e & 63, c = e >> 6;
          if (c < mr && r < mc) A[(long)(c0 + r) + (long)(r0 + c) * lda] = buf0[r][c];
        }
      }
    }
    if (critical) __builtin_amdgcn_s_setprio(0);
  }
}

void potrf_dataflow(double* A, int lda, int n, double* linv_ws, double* sbuf, int* flags,
                    unsigned* ticket, int* info, int* err, int n_wg, double* Yt, hipStream_t st,
                    int* cu_marks, hipEvent_t after_reset) {
  const int nt = (n + NB - 1) / NB;
  const int ntask = df_task_count(nt, Yt ? 1 : 0);
  k_reset_counter<<<1, 1, 0, st>>>(ticket);
  if (after_reset) (void)hipEventRecord(after_reset, st);
  k_potrf_dataflow<<<std::min(ntask, n_wg), 256, 0, st>>>(A, lda, n, nt, linv_ws, sbuf, flags,
                                                          ticket, info, err, Yt, cu_marks);
}

int potrf_cu_slots() { return CU_SLOTS; }

// Yt[v + r * 64] = g[v * ldg + r] (v < 3) and back.
__global__ void k_rhs_pack(int n, const double* __restrict__ g, int ldg, double* __restrict__ Yt) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int v = 0; v < 3; ++v) Yt[v + (long)r * NB] = g[(long)v * ldg + r];
}
__global__ void k_rhs_unpack(int n, const double* __restrict__ Yt, double* __restrict__ y, int ldy) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int v = 0; v < 3; ++v) y[(long)v * ldy + r] = Yt[v + (long)r * NB];
}
void rhs_pack(int n, const double* g, int ldg, double* Yt, hipStream_t st) {
  k_rhs_pack<<<(n + 255) / 256, 256, 0, st>>>(n, g, ldg, Yt);
}
void rhs_unpack(int n, const double* Yt, double* y, int ldy, hipStream_t st) {
  k_rhs_unpack<<<(n + 255) / 256, 256, 0, st>>>(n, Yt, y, ldy);
}

__global__ void k_copy_f64(long n, const double* __restrict__ src, double* __restrict__ dst) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = src[e];
}
__global__ void k_copy_i32(long n, const int32_t* __restrict__ src, int32_t* __restrict__ dst) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = src[e];
}
void copy_f64(long n, const double* src, double* dst, hipStream_t st) {
  if (n > 0) k_copy_f64<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, src, dst);
}
void copy_i32(long n, const int32_t* src, int32_t* dst, hipStream_t st) {
  if (n > 0) k_copy_i32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, src, dst);
}

__global__ void k_zero_int(int* p) { *p = 0; }
void zero_int(int* p, hipStream_t st) { k_zero_int<<<1, 1, 0, st>>>(p); }

__global__ void k_zero_f64(long n, double* p) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = 0.0;
}
void zero_f64(long n, double* p, hipStream_t st) {
  if (n > 0) k_zero_f64<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, p);
}

// ---------------------------------------------------------------------------
// Triangular inverse X = L^-1 from the tiled factor:
//   M_ip = Linv_ii L_ip (p < i), X_ii = Linv_ii, X_ic = -sum_{p=c}^{i-1} M_ip X_pc.

__global__ __launch_bounds__(256) void k_scale_offdiag(const double* L, int ldl, int n,
                                                       const double* linv_ws, double* M,
                                                       int ldm) {
  __shared__ double As[KC][LDS_LD];
  __shared__ double Bs[KC][LDS_LD];
  int i, p;
  tri_index(blockIdx.x, i, p);
  i += 1;                                   // strictly lower tiles: p < i
  const int r0 = i * NB, mr = min(NB, n - r0);
  Acc acc;
  acc_zero(acc);
  // C(r, c) = sum_kk Linv_ii(r, kk) L_ip(kk, c): Ahat = Linv (normal), Bhat(c, kk) = L(i*NB+kk, p*NB+c)
  gemm_acc<false, true>(acc, As, Bs, linv_ws + (long)i * NB * NB, NB, 0, NB, 0, L, ldl,
                        p * NB, NB, i * NB, mr);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = acc_row(mb), c = acc_col(nb, q);
        if (r < mr) M[(long)(r0 + r) + (long)(p * NB + c) * ldm] = acc.c[mb][nb][q];
      }
}

// Block row i of X: workgroup c < i computes X_ic, workgroup c = i copies Linv_ii.
__global__ __launch_bounds__(256) void k_trtri_row(const double* M, int ldm, int n, int i,
                                                   const double* linv_ws, double* X, int ldx) {
  __shared__ double As[KC][LDS_LD];
  __shared__ double Bs[KC][LDS_LD];
  const int c = blockIdx.x;
  const int r0 = i * NB, mr = min(NB, n - r0);
  if (c == i) {
    const double* Li = linv_ws + (long)i * NB * NB;
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
      const int r = e & 63, cc = e >> 6;
      if (r < mr && cc < mr) X[(long)(r0 + r) + (long)(r0 + cc) * ldx] = Li[e];
    }
    return;
  }
  Acc acc;
  acc_zero(acc);
  // C(r, cc) = sum_kk M(r0 + r, c*NB + kk) X(c*NB + kk, c*NB + cc), kk < (i - c) * NB
  gemm_acc<false, true>(acc, As, Bs, M, ldm, r0, mr, c * NB, X, ldx, c * NB, NB, c * NB,
                        (i - c) * NB);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = acc_row(mb), cc = acc_col(nb, q);
        if (r < mr) X[(long)(r0 + r) + (long)(c * NB + cc) * ldx] = -acc.c[mb][nb][q];
      }
}

void trtri_from_factor(const double* L, int ldl, int n, const double* linv_ws, double* M,
                       double* X, int ldx, hipStream_t st) {
  // M (strictly lower tiles, leading dimension ldx) and X must not alias:
  // block row i of X reads every M_ip of its row while writing X_ic.
  const int nt = (n + NB - 1) / NB;
  if (nt > 1) {
    const int cnt = (nt - 1) * nt / 2;
    k_scale_offdiag<<<cnt, 256, 0, st>>>(L, ldl, n, linv_ws, M, ldx);
  }
  for (int i = 0; i < nt; ++i) k_trtri_row<<<i + 1, 256, 0, st>>>(M, ldx, n, i, linv_ws, X, ldx);
}

// Z = X^T X (X lower) written in full symmetric storage.
__global__ __launch_bounds__(256) void k_lauum_full(const double* X, int ldx, int n, double* Z,
                                                    int ldz) {
  __shared__ double As[KC][LDS_LD];
  __shared__ double Bs[KC][LDS_LD];
  int i, j;
  tri_index(blockIdx.x, i, j);
  const int r0 = i * NB, c0 = j * NB;
  const int mr = min(NB, n - r0), mc = min(NB, n - c0);
  Acc acc;
  acc_zero(acc);
  // Z(r0 + r, c0 + c) = sum_{p >= r0} X(p, r0 + r) X(p, c0 + c)
  gemm_acc<true, true>(acc, As, Bs, X, ldx, r0, mr, r0, X, ldx, c0, mc, r0, n - r0);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = acc_row(mb), c = acc_col(nb, q);
        if (r < mr && c < mc) {
          Z[(long)(r0 + r) + (long)(c0 + c) * ldz] = acc.c[mb][nb][q];
          Z[(long)(c0 + c) + (long)(r0 + r) * ldz] = acc.c[mb][nb][q];
        }
      }
}

void lauum_full(const double* X, int ldx, int n, double* Z, int ldz, hipStream_t st) {
  const int nt = (n + NB - 1) / NB;
  k_lauum_full<<<nt * (nt + 1) / 2, 256, 0, st>>>(X, ldx, n, Z, ldz);
}

// C = beta C + alpha A B^T, one 64 x 64 tile of C per workgroup (tiles on or
// below the diagonal only when lower; B lower triangular when blower, so the
// sum for a column tile j stops at the end of B's diagonal tile j).
__global__ __launch_bounds__(256) void k_gemm_nt(const double* A, long lda, const double* B,
                                                 long ldb, double* C, long ldc, int m, int nc,
                                                 int K, double alpha, double beta, int lower,
                                                 int blower) {
  __shared__ double As[KC][LDS_LD];
  __shared__ double Bs[KC][LDS_LD];
  int i, j;
  if (lower) {
    tri_index(blockIdx.x, i, j);
  } else {
    const int mt = (m + NB - 1) / NB;
    i = blockIdx.x % mt;
    j = blockIdx.x / mt;
  }
  const int r0 = i * NB, c0 = j * NB;
  const int mr = min(NB, m - r0), mc = min(NB, nc - c0);
  const int kend = blower ? min(K, c0 + NB) : K;
  Acc acc;
  acc_zero(acc);
  gemm_acc<false, false>(acc, As, Bs, A, lda, r0, mr, 0, B, ldb, c0, mc, 0, kend);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = acc_row(mb), c = acc_col(nb, q);
        if (r < mr && c < mc) {
          double* p = C + (long)(r0 + r) + (long)(c0 + c) * ldc;
          const double v = alpha * acc.c[mb][nb][q];
          *p = beta == 0.0 ? v : beta * *p + v;
        }
      }
}

void gemm_nt(const double* A, long lda, const double* B, long ldb, double* C, long ldc, int m,
             int nc, int K, double alpha, double beta, int lower, int blower, hipStream_t st) {
  if (m <= 0 || nc <= 0) return;
  const long mt = (m + NB - 1) / NB, ntc = (nc + NB - 1) / NB;
  const long cnt = lower ? mt * (mt + 1) / 2 : mt * ntc;
  k_gemm_nt<<<(unsigned)cnt, 256, 0, st>>>(A, lda, B, ldb, C, ldc, m, nc, K, alpha, beta, lower,
                                           blower);
}

__global__ __launch_bounds__(256) void k_copy_lower_tiles(const double* S, int lds, double* H,
                                                          int ldh, int n) {
  int i, j;
  tri_index(blockIdx.x, i, j);
  const int r0 = i * NB, c0 = j * NB;
  const int mr = min(NB, n - r0), mc = min(NB, n - c0);
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e & 63, c = e >> 6;
    if (r < mr && c < mc) H[(long)(r0 + r) + (long)(c0 + c) * ldh] = S[(long)(r0 + r) + (long)(c0 + c) * lds];
  }
}

void copy_lower_tiles(const double* S, int lds, double* H, int ldh, int n, hipStream_t st) {
  const int nt = (n + NB - 1) / NB;
  k_copy_lower_tiles<<<nt * (nt + 1) / 2, 256, 0, st>>>(S, lds, H, ldh, n);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// y = alpha * A v + beta * y, A symmetric in full storage: element i of the
// product is the dot of column i with v.  A workgroup owns 8 columns (two per
// wave); the three right-hand sides are staged through LDS in chunks of 512
// rows, so each matrix element costs one 16-byte-per-lane streaming load and
// the vector is read from L2 once per 8 columns.
constexpr int SV_CHUNK = 512;
__global__ __launch_bounds__(256) void k_symv3(const double* __restrict__ A, long lda, int n,
                                               const double* __restrict__ v, long ldv,
                                               double alpha, double beta, double* y, long ldy) {
  __shared__ double vs[3][SV_CHUNK];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int c0 = blockIdx.x * 8 + w * 2;
  const bool has0 = c0 < n, has1 = c0 + 1 < n;
  const double* a0 = A + (long)min(c0, n - 1) * lda;
  const double* a1 = A + (long)min(c0 + 1, n - 1) * lda;
  const bool vec = ((lda & 1) == 0) && ((((unsigned long)A) & 15) == 0);
  double s[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int j0 = 0; j0 < n; j0 += SV_CHUNK) {
    const int cnt = min(SV_CHUNK, n - j0);
    __syncthreads();
    for (int e = t; e < 3 * SV_CHUNK; e += 256) {
      const int vv = e / SV_CHUNK, jj = e % SV_CHUNK;
      vs[vv][jj] = (jj < cnt) ? v[(long)vv * ldv + j0 + jj] : 0.0;
    }
    __syncthreads();
    if (vec && cnt == SV_CHUNK) {
#pragma unroll
      for (int it = 0; it < SV_CHUNK / 128; ++it) {
        const int jj = it * 128 + 2 * lane;
        const double2 x0 = *(const double2*)(a0 + j0 + jj);
        const double2 x1 = *(const double2*)(a1 + j0 + jj);
#pragma unroll
        for (int vv = 0; vv < 3; ++vv) {
          const double p = vs[vv][jj], q = vs[vv][jj + 1];
          s[0][vv] += x0.x * p + x0.y * q;
          s[1][vv] += x1.x * p + x1.y * q;
        }
      }
    } else {
      for (int jj = lane; jj < cnt; jj += 64) {
        const double x0 = a0[j0 + jj], x1 = a1[j0 + jj];
#pragma unroll
        for (int vv = 0; vv < 3; ++vv) {
          s[0][vv] += x0 * vs[vv][jj];
          s[1][vv] += x1 * vs[vv][jj];
        }
      }
    }
  }
#pragma unroll
  for (int cc = 0; cc < 2; ++cc)
#pragma unroll
    for (int vv = 0; vv < 3; ++vv) s[cc][vv] = wave_sum(s[cc][vv]);
  if (lane == 0) {
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
      if (!(cc == 0 ? has0 : has1)) continue;
      const int col = c0 + cc;
#pragma unroll
      for (int vv = 0; vv < 3; ++vv) {
        double* yo = y + (long)vv * ldy + col;
        *yo = (beta == 0.0) ? alpha * s[cc][vv] : alpha * s[cc][vv] + beta * *yo;
      }
    }
  }
}

void symv3(const double* A, int lda, int n, const double* v, int ldv, double alpha, double beta,
           double* y, int ldy, hipStream_t st) {
  if (n > 0) k_symv3<<<(n + 7) / 8, 256, 0, st>>>(A, lda, n, v, ldv, alpha, beta, y, ldy);
}

}  // namespace pdk
