// Dense FP64 kernels for gfx950: tiled Cholesky of the Schur system and of the
// interior level blocks, triangular inverse, symmetric inverse assembly,
// three-right-hand-side triangular solves and the symmetric matrix-vector
// product.  Tiles are NB x NB (NB = 64), column-major.  Products run on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64) with operands staged through LDS.
#include <climits>
#include "common.h"

namespace pdk {

constexpr int KC = 16;           // K-chunk staged through LDS per step
constexpr int LDS_LD = NB + 4;   // padded LDS row (doubles)

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

// ---------------------------------------------------------------------------
// Cholesky building blocks

// Factor diagonal tile k in place (lower) and write its inverse (64x64, lower,
// identity-padded past the matrix edge) to linv_ws + k*NB*NB.  A non-positive
// pivot stores its 1-based global index in *info (first one wins) and is
// replaced by 1 so that the factorization stays finite.
__global__ __launch_bounds__(256) void k_potrf_diag(double* A, int lda, int n, int k,
                                                    double* linv_ws, int* info) {
  __shared__ double T[NB][NB + 1];   // T[c][r] = tile(r, c)
  __shared__ double X[NB][NB + 1];   // X[c][r] = inverse(r, c)
  __shared__ double inv_d[NB];
  const int t = threadIdx.x;
  const int r0 = k * NB;
  const int mr = min(NB, n - r0);
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e & 63, c = e >> 6;
    double v;
    if (r < mr && c < mr) v = (r >= c) ? A[(long)(r0 + r) + (long)(r0 + c) * lda] : 0.0;
    else v = (r == c) ? 1.0 : 0.0;
    T[c][r] = v;
  }
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    __syncthreads();                       // trailing update of step j-1 complete
    double d = T[j][j];
    if (!(d > 0.0)) {
      if (t == 0 && j < mr) atomicCAS(info, 0, r0 + j + 1);
      d = 1.0;
    }
    const double ljj = sqrt(d);
    const double il = 1.0 / ljj;
    __syncthreads();
    if (t == 0) { T[j][j] = ljj; inv_d[j] = il; }
    if (t > j && t < NB) T[j][t] *= il;
    __syncthreads();
    const int r = t & 63;
    for (int c = j + 1 + (t >> 6); c < NB; c += 4)
      if (r >= c) T[c][r] -= T[j][r] * T[j][c];
  }
  __syncthreads();
  // inverse of the lower factor, one column per lane of wave 0:
  // x_c = 1/L_cc, x_i = -(sum_{p=c}^{i-1} L_ip x_p) / L_ii
  if (t < NB) {
    const int c = t;
    for (int i = 0; i < c; ++i) X[c][i] = 0.0;
    X[c][c] = inv_d[c];
    for (int i = c + 1; i < NB; ++i) {
      double s0 = 0.0, s1 = 0.0;
      int p = c;
      for (; p + 1 < i; p += 2) {
        s0 += T[p][i] * X[c][p];
        s1 += T[p + 1][i] * X[c][p + 1];
      }
      if (p < i) s0 += T[p][i] * X[c][p];
      X[c][i] = -(s0 + s1) * inv_d[i];
    }
  }
  __syncthreads();
  double* Li = linv_ws + (long)k * NB * NB;
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e & 63, c = e >> 6;
    Li[e] = X[c][r];
    if (r < mr && c < mr && r >= c) A[(long)(r0 + r) + (long)(r0 + c) * lda] = T[c][r];
  }
}

// Panel: L_ik = A_ik * Linv_kk^T for tiles i > k (one workgroup per tile).
__global__ __launch_bounds__(256) void k_trsm_panel(double* A, int lda, int n, int k,
                                                    const double* linv_ws) {
  __shared__ double As[KC][LDS_LD];
  __shared__ double Bs[KC][LDS_LD];
  const int i = k + 1 + blockIdx.x;
  const int r0 = i * NB, mr = min(NB, n - r0);
  Acc acc;
  acc_zero(acc);
  gemm_acc<false, false>(acc, As, Bs, A, lda, r0, mr, k * NB,
                         linv_ws + (long)k * NB * NB, NB, 0, NB, 0, NB);
  __syncthreads();
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = acc_row(mb), c = acc_col(nb, q);
        if (r < mr) A[(long)(r0 + r) + (long)(k * NB + c) * lda] = acc.c[mb][nb][q];
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

// Trailing update of step k: A_ij -= L_ik L_jk^T for k < j <= i.
__global__ __launch_bounds__(256) void k_syrk_update(double* A, int lda, int n, int k) {
  __shared__ double As[KC][LDS_LD];
  __shared__ double Bs[KC][LDS_LD];
  int ii, jj;
  tri_index(blockIdx.x, ii, jj);
  const int i = k + 1 + ii, j = k + 1 + jj;
  const int r0 = i * NB, c0 = j * NB;
  const int mr = min(NB, n - r0), mc = min(NB, n - c0);
  Acc acc;
  acc_zero(acc);
  gemm_acc<false, false>(acc, As, Bs, A, lda, r0, mr, k * NB, A, lda, c0, mc, k * NB, NB);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = acc_row(mb), c = acc_col(nb, q);
        if (r < mr && c < mc) A[(long)(r0 + r) + (long)(c0 + c) * lda] -= acc.c[mb][nb][q];
      }
}

void potrf_tiled(double* A, int lda, int n, double* linv_ws, int* info, hipStream_t st) {
  const int nt = (n + NB - 1) / NB;
  for (int k = 0; k < nt; ++k) {
    k_potrf_diag<<<1, 256, 0, st>>>(A, lda, n, k, linv_ws, info);
    const int R = nt - k - 1;
    if (R > 0) {
      k_trsm_panel<<<R, 256, 0, st>>>(A, lda, n, k, linv_ws);
      k_syrk_update<<<R * (R + 1) / 2, 256, 0, st>>>(A, lda, n, k);
    }
  }
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

// ---------------------------------------------------------------------------
// Three-right-hand-side triangular solves with the tiled factor.  One
// workgroup per block row; rows are claimed in dependency order through a
// ticket counter, so every claimed row only waits on rows claimed earlier by
// running workgroups.  Row completion is published with a per-call epoch.

constexpr long SPIN_LIMIT = 1L << 24;

__device__ inline bool wait_flag(int* f, int epoch, int* err) {
  long spins = 0;
  while (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(1);
    if (++spins > SPIN_LIMIT) {
      atomicExch(err, 1);
      return false;
    }
  }
  return true;
}

__device__ inline double coherent_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void coherent_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// L y = g.
__global__ __launch_bounds__(256) void k_trsv3_fwd(const double* __restrict__ L, int ld, int n,
                                                   int nt, const double* __restrict__ linv,
                                                   const double* __restrict__ g, int ldg,
                                                   double* y, int ldy,
                                                   unsigned long long* ticket, int* flags,
                                                   int* err) {
  __shared__ int s_row, s_epoch, s_ok;
  __shared__ double ys[3][NB];
  __shared__ double part[4][3][NB];
  const int t = threadIdx.x;
  if (t == 0) {
    const unsigned long long tk = atomicAdd(ticket, 1ull);
    s_row = (int)(tk % (unsigned long long)nt);
    s_epoch = (int)(tk / (unsigned long long)nt) + 1;
    s_ok = 1;
  }
  __syncthreads();
  const int i = s_row, epoch = s_epoch;
  const int r0 = i * NB, mr = min(NB, n - r0);
  const int r = t & 63, cg = t >> 6;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int p = 0; p < i; ++p) {
    double lv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
      lv[q] = (r < mr) ? L[(long)(r0 + r) + (long)(p * NB + cg * 16 + q) * ld] : 0.0;
    if (t == 0 && !wait_flag(&flags[p], epoch, err)) s_ok = 0;
    __syncthreads();
    if (!s_ok) return;
    if (t < 3 * NB) ys[t >> 6][t & 63] = coherent_load(&y[(long)(t >> 6) * ldy + p * NB + (t & 63)]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = cg * 16 + q;
      a0 += lv[q] * ys[0][c];
      a1 += lv[q] * ys[1][c];
      a2 += lv[q] * ys[2][c];
    }
    __syncthreads();
  }
  part[cg][0][r] = a0;
  part[cg][1][r] = a1;
  part[cg][2][r] = a2;
  __syncthreads();
  if (t < 3 * NB) {
    const int v = t >> 6, rr = t & 63;
    const double b = (rr < mr) ? g[(long)v * ldg + r0 + rr] : 0.0;
    ys[v][rr] = b - (part[0][v][rr] + part[1][v][rr] + part[2][v][rr] + part[3][v][rr]);
  }
  __syncthreads();
  const double* Li = linv + (long)i * NB * NB;
  if (t < 3 * NB) {
    const int v = t >> 6, rr = t & 63;
    double s = 0.0;
    for (int c = 0; c <= rr; ++c) s += Li[rr + c * NB] * ys[v][c];
    if (rr < mr) coherent_store(&y[(long)v * ldy + r0 + rr], s);
  }
  __threadfence();
  __syncthreads();
  if (t == 0) __hip_atomic_store(&flags[i], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// L^T x = y.
__global__ __launch_bounds__(256) void k_trsv3_bwd(const double* __restrict__ L, int ld, int n,
                                                   int nt, const double* __restrict__ linv,
                                                   const double* __restrict__ y, int ldy,
                                                   double* x, int ldx,
                                                   unsigned long long* ticket, int* flags,
                                                   int* err) {
  __shared__ int s_row, s_epoch, s_ok;
  __shared__ double xs[3][NB];
  __shared__ double part[4][3][NB];
  const int t = threadIdx.x;
  if (t == 0) {
    const unsigned long long tk = atomicAdd(ticket, 1ull);
    s_row = nt - 1 - (int)(tk % (unsigned long long)nt);
    s_epoch = (int)(tk / (unsigned long long)nt) + 1;
    s_ok = 1;
  }
  __syncthreads();
  const int i = s_row, epoch = s_epoch;
  const int r0 = i * NB, mr = min(NB, n - r0);
  const int c = t & 63, rg = t >> 6;     // lane walks down a column of L
  double acc[16][3];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
  for (int p = nt - 1; p > i; --p) {
    const int pr0 = p * NB, pmr = min(NB, n - pr0);
    double lv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int rr = rg + 4 * q;
      lv[q] = (c < pmr && rr < mr) ? L[(long)(pr0 + c) + (long)(r0 + rr) * ld] : 0.0;
    }
    if (t == 0 && !wait_flag(&flags[p], epoch, err)) s_ok = 0;
    __syncthreads();
    if (!s_ok) return;
    if (t < 3 * NB) {
      const int v = t >> 6, cc = t & 63;
      xs[v][cc] = (cc < pmr) ? coherent_load(&x[(long)v * ldx + pr0 + cc]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      acc[q][0] += lv[q] * xs[0][c];
      acc[q][1] += lv[q] * xs[1][c];
      acc[q][2] += lv[q] * xs[2][c];
    }
    __syncthreads();
  }
  // reduce over the 64 lanes (c) of each wave
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const double s0 = wave_sum(acc[q][0]);
    const double s1 = wave_sum(acc[q][1]);
    const double s2 = wave_sum(acc[q][2]);
    if (c == 0) {
      part[0][0][rg + 4 * q] = s0;
      part[0][1][rg + 4 * q] = s1;
      part[0][2][rg + 4 * q] = s2;
    }
  }
  __syncthreads();
  if (t < 3 * NB) {
    const int v = t >> 6, rr = t & 63;
    const double b = (rr < mr) ? y[(long)v * ldy + r0 + rr] : 0.0;
    xs[v][rr] = b - part[0][v][rr];
  }
  __syncthreads();
  const double* Li = linv + (long)i * NB * NB;
  if (t < 3 * NB) {
    const int v = t >> 6, rr = t & 63;
    double s = 0.0;
    for (int cc = rr; cc < NB; ++cc) s += Li[cc + rr * NB] * xs[v][cc];
    if (rr < mr) coherent_store(&x[(long)v * ldx + r0 + rr], s);
  }
  __threadfence();
  __syncthreads();
  if (t == 0) __hip_atomic_store(&flags[i], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

void trsv3_forward(const double* L, int ld, int n, const double* linv_ws, const double* g,
                   int ldg, double* y, int ldy, unsigned long long* ticket, int* flags,
                   int* err, hipStream_t st) {
  const int nt = (n + NB - 1) / NB;
  k_trsv3_fwd<<<nt, 256, 0, st>>>(L, ld, n, nt, linv_ws, g, ldg, y, ldy, ticket, flags, err);
}

void trsv3_backward(const double* L, int ld, int n, const double* linv_ws, const double* y,
                    int ldy, double* x, int ldx, unsigned long long* ticket, int* flags,
                    int* err, hipStream_t st) {
  const int nt = (n + NB - 1) / NB;
  k_trsv3_bwd<<<nt, 256, 0, st>>>(L, ld, n, nt, linv_ws, y, ldy, x, ldx, ticket, flags, err);
}

// ---------------------------------------------------------------------------
// y = alpha * A v + beta * y, A symmetric in full storage: element i of the
// product is the dot of column i with v, one wave per column (contiguous reads).
__global__ __launch_bounds__(256) void k_symv3(const double* __restrict__ A, long lda, int n,
                                               const double* __restrict__ v, long ldv,
                                               double alpha, double beta, double* y, long ldy) {
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= n) return;
  const double* a = A + (long)col * lda;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  int j = lane;
  for (; j + 192 < n; j += 256) {
    const double x0 = a[j], x1 = a[j + 64], x2 = a[j + 128], x3 = a[j + 192];
    s0 += x0 * v[j] + x1 * v[j + 64] + x2 * v[j + 128] + x3 * v[j + 192];
    s1 += x0 * v[ldv + j] + x1 * v[ldv + j + 64] + x2 * v[ldv + j + 128] + x3 * v[ldv + j + 192];
    s2 += x0 * v[2 * ldv + j] + x1 * v[2 * ldv + j + 64] + x2 * v[2 * ldv + j + 128] +
          x3 * v[2 * ldv + j + 192];
  }
  for (; j < n; j += 64) {
    const double x0 = a[j];
    s0 += x0 * v[j];
    s1 += x0 * v[ldv + j];
    s2 += x0 * v[2 * ldv + j];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    if (beta == 0.0) {
      y[col] = alpha * s0;
      y[ldy + col] = alpha * s1;
      y[2 * ldy + col] = alpha * s2;
    } else {
      y[col] = alpha * s0 + beta * y[col];
      y[ldy + col] = alpha * s1 + beta * y[ldy + col];
      y[2 * ldy + col] = alpha * s2 + beta * y[2 * ldy + col];
    }
  }
}

void symv3(const double* A, int lda, int n, const double* v, int ldv, double alpha, double beta,
           double* y, int ldy, hipStream_t st) {
  k_symv3<<<(n + 3) / 4, 256, 0, st>>>(A, lda, n, v, ldv, alpha, beta, y, ldy);
}

}  // namespace pdk
