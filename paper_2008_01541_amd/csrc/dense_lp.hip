// Low-precision factorization of the Schur system for the refined solve:
// the equilibrated matrix D (S + P) D is factored in FP32, with the O(n^3)
// tile products on the FP32 matrix cores (v_mfma_f32_16x16x4f32) or with
// BF16 operands and FP32 accumulation (v_mfma_f32_16x16x32_bf16); diagonal
// tiles and panel solves stay in FP32.  Triangular solves run in FP32 on
// FP64 inputs/outputs; the refinement residual is computed in FP64 elsewhere.
#include <algorithm>
#include "common.h"

namespace pdk {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

constexpr int LP_LD = NB + 4;     // FP32 LDS row (floats)
constexpr int KC32 = 32;          // K chunk of the staged products
constexpr int BF_LD = KC32 + 8;   // BF16 LDS row (k contiguous, 16-byte aligned rows)

struct AccF {
  float4_t c[2][2];
};

__device__ inline void accf_zero(AccF& a) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) a.c[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
}
// FP32-accumulator MFMA result D[4(l/16)+q][l%16], issued with the column
// operand first, holds C(row = l%16, col = 4(l/16) + q).
__device__ inline int accf_row(int mb) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  return (w >> 1) * 32 + mb * 16 + (lane & 15);
}
__device__ inline int accf_col(int nb, int q) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  return (w & 1) * 32 + nb * 16 + 4 * (lane >> 4) + q;
}

// ---- FP32-operand product: acc += Ahat Bhat^T, Ahat/Bhat read as tiles of a
// column-major FP32 matrix (rows r0.., cols k0..), K = 64 (one tile).
__device__ void gemm_f32_tile(AccF& acc, float (*As)[LP_LD], float (*Bs)[LP_LD],
                              const float* __restrict__ A, long lda, int ar0, int amr,
                              const float* __restrict__ B, long ldb, int br0, int bmr, int k0) {
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  for (int kk = 0; kk < NB; kk += KC32) {
    __syncthreads();
    const int r = t & 63;
#pragma unroll
    for (int q = 0; q < KC32 / 4; ++q) {
      const int k = (t >> 6) + 4 * q;
      As[k][r] = (r < amr) ? A[(long)(ar0 + r) + (long)(k0 + kk + k) * lda] : 0.f;
      Bs[k][r] = (r < bmr) ? B[(long)(br0 + r) + (long)(k0 + kk + k) * ldb] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC32 / 4; ++ks) {
      const int k = ks * 4 + (lane >> 4);
      const float a0 = As[k][wr * 32 + (lane & 15)];
      const float a1 = As[k][wr * 32 + 16 + (lane & 15)];
      const float b0 = Bs[k][wc * 32 + (lane & 15)];
      const float b1 = Bs[k][wc * 32 + 16 + (lane & 15)];
      acc.c[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(b0, a0, acc.c[0][0], 0, 0, 0);
      acc.c[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(b1, a0, acc.c[0][1], 0, 0, 0);
      acc.c[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(b0, a1, acc.c[1][0], 0, 0, 0);
      acc.c[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(b1, a1, acc.c[1][1], 0, 0, 0);
    }
  }
}

// ---- BF16-operand product (FP32 accumulation), same contract.
__device__ void gemm_bf16_tile(AccF& acc, __bf16 (*As)[BF_LD], __bf16 (*Bs)[BF_LD],
                               const float* __restrict__ A, long lda, int ar0, int amr,
                               const float* __restrict__ B, long ldb, int br0, int bmr, int k0) {
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  for (int kk = 0; kk < NB; kk += KC32) {
    __syncthreads();
    const int r = t & 63;
#pragma unroll
    for (int q = 0; q < KC32 / 4; ++q) {
      const int k = (t >> 6) + 4 * q;
      As[r][k] = (__bf16)((r < amr) ? A[(long)(ar0 + r) + (long)(k0 + kk + k) * lda] : 0.f);
      Bs[r][k] = (__bf16)((r < bmr) ? B[(long)(br0 + r) + (long)(k0 + kk + k) * ldb] : 0.f);
    }
    __syncthreads();
    const int ko = 8 * (lane >> 4);
    const bf16x8_t a0 = *(const bf16x8_t*)&As[wr * 32 + (lane & 15)][ko];
    const bf16x8_t a1 = *(const bf16x8_t*)&As[wr * 32 + 16 + (lane & 15)][ko];
    const bf16x8_t b0 = *(const bf16x8_t*)&Bs[wc * 32 + (lane & 15)][ko];
    const bf16x8_t b1 = *(const bf16x8_t*)&Bs[wc * 32 + 16 + (lane & 15)][ko];
    acc.c[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b0, a0, acc.c[0][0], 0, 0, 0);
    acc.c[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b1, a0, acc.c[0][1], 0, 0, 0);
    acc.c[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b0, a1, acc.c[1][0], 0, 0, 0);
    acc.c[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b1, a1, acc.c[1][1], 0, 0, 0);
  }
}

// FP32 Cholesky + inverse of an LDS tile (T[c][r] = tile(r, c)); see the FP64 version.
__device__ void factor_tile_lds_f32(float (*T)[LP_LD], float (*X)[LP_LD], float* inv_d, int mr,
                                    int gbase, int* info) {
  const int t = threadIdx.x;
  for (int j = 0; j < NB; ++j) {
    __syncthreads();
    float d = T[j][j];
    if (!(d > 0.f)) {
      if (t == 0 && j < mr) atomicCAS(info, 0, gbase + j + 1);
      d = 1.f;
    }
    const float ljj = sqrtf(d);
    const float il = 1.f / ljj;
    __syncthreads();
    if (t == 0) { T[j][j] = ljj; inv_d[j] = il; }
    if (t > j && t < NB) T[j][t] *= il;
    __syncthreads();
    const int r = t & 63;
    for (int c = j + 1 + (t >> 6); c < NB; c += 4)
      if (r >= c) T[c][r] -= T[j][r] * T[j][c];
  }
  __syncthreads();
  if (t < NB) {
    const int c = t;
    for (int i = 0; i < c; ++i) X[c][i] = 0.f;
    X[c][c] = inv_d[c];
    for (int i = c + 1; i < NB; ++i) {
      float s0 = 0.f, s1 = 0.f;
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
}

constexpr long LP_SPIN_LIMIT = 1L << 24;
// Same publication protocol as the FP64 kernels: agent-coherent stores of
// published data, vmcnt(0) + barrier, then a coherent flag store; consumers
// poll with coherent loads and read immutable published data with plain loads.
__device__ inline bool lp_wait(const int* f, int epoch, int* err) {
  long spins = 0;
  while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(1);
    if (++spins > LP_SPIN_LIMIT) {
      atomicExch(err, 1);
      return false;
    }
  }
  return true;
}
__device__ inline void lp_publish(int* f, int epoch) {
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(f, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline float cload(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void cstore(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// acc += sum_{k<j} L_ik L_jk^T for an FP32 factor; operands of step k+1 are
// loaded into registers during step k, flags of step k+2 are read ahead.
// BF16: operands are rounded to BF16 when staged; FP32 accumulation.
constexpr int BFL = NB + 8;   // BF16 LDS row: 64 k values + pad (16-byte aligned)
template <bool BF16>
__device__ bool lp_accumulate(AccF& acc, float (*buf0)[LP_LD], float (*buf1)[LP_LD],
                              const float* __restrict__ A, int lda, int r0, int mr, int c0, int mc,
                              int i, int j, int nt, const int* flags, int epoch, int* err,
                              int* s_ok) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int r = t & 63, kq = t >> 6;
  if (j == 0) return true;
  float ra[16], rb[16];
  auto load_tile = [&](int k) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const long col = (long)(k * NB + kq + 4 * q) * lda;
      ra[q] = (r < mr) ? A[(long)(r0 + r) + col] : 0.f;
      rb[q] = (r < mc) ? A[(long)(c0 + r) + col] : 0.f;
    }
  };
  __bf16 (*Ab)[BFL] = (__bf16 (*)[BFL]) & buf0[0][0];
  __bf16 (*Bb)[BFL] = (__bf16 (*)[BFL]) & buf1[0][0];
  int fi = 0, fj = 0;
  if (t == 0) {
    if (!lp_wait(&flags[i * nt], epoch, err) || !lp_wait(&flags[j * nt], epoch, err)) *s_ok = 0;
  }
  __syncthreads();
  if (!*s_ok) return false;
  load_tile(0);
  if (t == 0 && j > 1) {
    fi = __hip_atomic_load(&flags[i * nt + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    fj = __hip_atomic_load(&flags[j * nt + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  for (int k = 0; k < j; ++k) {
    __syncthreads();
    if (BF16) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        Ab[r][kq + 4 * q] = (__bf16)ra[q];
        Bb[r][kq + 4 * q] = (__bf16)rb[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        buf0[kq + 4 * q][r] = ra[q];
        buf1[kq + 4 * q][r] = rb[q];
      }
    }
    const bool nxt = k + 1 < j;
    if (t == 0 && nxt && (fi != epoch || fj != epoch)) {
      if (!lp_wait(&flags[i * nt + k + 1], epoch, err) || !lp_wait(&flags[j * nt + k + 1], epoch, err))
        *s_ok = 0;
    }
    __syncthreads();
    if (!*s_ok) return false;
    if (nxt) {
      load_tile(k + 1);
      if (t == 0 && k + 2 < j) {
        fi = __hip_atomic_load(&flags[i * nt + k + 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        fj = __hip_atomic_load(&flags[j * nt + k + 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (BF16) {
#pragma unroll
      for (int ks = 0; ks < NB / 32; ++ks) {
        const int ko = ks * 32 + 8 * (lane >> 4);
        const bf16x8_t a0 = *(const bf16x8_t*)&Ab[wr * 32 + (lane & 15)][ko];
        const bf16x8_t a1 = *(const bf16x8_t*)&Ab[wr * 32 + 16 + (lane & 15)][ko];
        const bf16x8_t b0 = *(const bf16x8_t*)&Bb[wc * 32 + (lane & 15)][ko];
        const bf16x8_t b1 = *(const bf16x8_t*)&Bb[wc * 32 + 16 + (lane & 15)][ko];
        acc.c[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b0, a0, acc.c[0][0], 0, 0, 0);
        acc.c[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b1, a0, acc.c[0][1], 0, 0, 0);
        acc.c[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b0, a1, acc.c[1][0], 0, 0, 0);
        acc.c[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b1, a1, acc.c[1][1], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < NB / 4; ++ks) {
        const int kk = ks * 4 + (lane >> 4);
        const float a0 = buf0[kk][wr * 32 + (lane & 15)];
        const float a1 = buf0[kk][wr * 32 + 16 + (lane & 15)];
        const float b0 = buf1[kk][wc * 32 + (lane & 15)];
        const float b1 = buf1[kk][wc * 32 + 16 + (lane & 15)];
        acc.c[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(b0, a0, acc.c[0][0], 0, 0, 0);
        acc.c[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(b1, a0, acc.c[0][1], 0, 0, 0);
        acc.c[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(b0, a1, acc.c[1][0], 0, 0, 0);
        acc.c[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(b1, a1, acc.c[1][1], 0, 0, 0);
      }
    }
  }
  return true;
}

__global__ void k_reset_counter_lp(unsigned* ctr) {
  ctr[0] = 0u;
  ctr[1] = ctr[1] + 1u;
}

// Dataflow Cholesky of a float matrix (same schedule as the FP64 kernel).
template <bool BF16>
__global__ __launch_bounds__(256, 2) void k_potrf_dataflow_lp(float* A, int lda, int n, int nt,
                                                              float* linv_ws, int* flags,
                                                              unsigned* ticket, int* info,
                                                              int* err) {
  const int epoch = (int)ticket[1];
  __shared__ float buf0[NB][LP_LD];
  __shared__ float buf1[NB][LP_LD];
  __shared__ float inv_d[NB];
  __shared__ int s_task, s_ok;
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int ntask = nt * (nt + 1) / 2;
  for (;;) {
    __syncthreads();
    if (t == 0) {
      s_task = (int)atomicAdd(ticket, 1u);
      s_ok = 1;
    }
    __syncthreads();
    const int q = s_task;
    if (q >= ntask) return;
    int j = 0, start = 0;
    while (start + (nt - j) <= q) {
      start += nt - j;
      ++j;
    }
    const int i = j + (q - start);
    const int r0 = i * NB, c0 = j * NB;
    const int mr = min(NB, n - r0), mc = min(NB, n - c0);
    AccF acc;
    accf_zero(acc);
    if (!lp_accumulate<BF16>(acc, buf0, buf1, A, lda, r0, mr, c0, mc, i, j, nt, flags, epoch, err,
                             &s_ok))
      return;
    __syncthreads();
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int r = accf_row(mb), c = accf_col(nb, qq);
          float v;
          if (r < mr && c < mc) v = cload(&A[(long)(r0 + r) + (long)(c0 + c) * lda]) - acc.c[mb][nb][qq];
          else v = (i == j && r == c) ? 1.f : 0.f;
          buf0[c][r] = v;
        }
    __syncthreads();
    if (i == j) {
      factor_tile_lds_f32(buf0, buf1, inv_d, mr, r0, info);
      float* Li = linv_ws + (long)j * NB * NB;
      for (int e = t; e < NB * NB; e += 256) {
        const int r = e & 63, c = e >> 6;
        cstore(&Li[e], buf1[c][r]);
        if (r < mr && c < mr)
          cstore(&A[(long)(r0 + r) + (long)(r0 + c) * lda], (r >= c) ? buf0[c][r] : buf0[r][c]);
      }
    } else {
      if (t == 0 && !lp_wait(&flags[j * nt + j], epoch, err)) s_ok = 0;
      __syncthreads();
      if (!s_ok) return;
      const float* Li = linv_ws + (long)j * NB * NB;
      for (int e = t; e < NB * NB; e += 256) buf1[e >> 6][e & 63] = Li[e];
      __syncthreads();
      accf_zero(acc);
#pragma unroll 4
      for (int ks = 0; ks < NB / 4; ++ks) {
        const int k = ks * 4 + (lane >> 4);
        const float a0 = buf0[k][wr * 32 + (lane & 15)];
        const float a1 = buf0[k][wr * 32 + 16 + (lane & 15)];
        const float b0 = buf1[k][wc * 32 + (lane & 15)];
        const float b1 = buf1[k][wc * 32 + 16 + (lane & 15)];
        acc.c[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(b0, a0, acc.c[0][0], 0, 0, 0);
        acc.c[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(b1, a0, acc.c[0][1], 0, 0, 0);
        acc.c[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(b0, a1, acc.c[1][0], 0, 0, 0);
        acc.c[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(b1, a1, acc.c[1][1], 0, 0, 0);
      }
      __syncthreads();
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) buf0[accf_col(nb, qq)][accf_row(mb)] = acc.c[mb][nb][qq];
      __syncthreads();
      for (int e = t; e < NB * NB; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (r < mr) cstore(&A[(long)(r0 + r) + (long)(c0 + c) * lda], buf0[c][r]);
        if (c < mr) cstore(&A[(long)(c0 + r) + (long)(r0 + c) * lda], buf0[r][c]);   // L^T copy
      }
    }
    lp_publish(&flags[i * nt + j], epoch);
  }
}

void potrf_dataflow_lp(float* A, int lda, int n, float* linv_ws, int* flags, unsigned* ticket,
                       int* info, int* err, int n_wg, bool bf16, hipStream_t st) {
  const int nt = (n + NB - 1) / NB;
  const int ntask = nt * (nt + 1) / 2;
  k_reset_counter_lp<<<1, 1, 0, st>>>(ticket);
  if (bf16)
    k_potrf_dataflow_lp<true><<<std::min(ntask, n_wg), 256, 0, st>>>(A, lda, n, nt, linv_ws, flags,
                                                                     ticket, info, err);
  else
    k_potrf_dataflow_lp<false><<<std::min(ntask, n_wg), 256, 0, st>>>(A, lda, n, nt, linv_ws, flags,
                                                                      ticket, info, err);
}

// ---------------------------------------------------------------------------
// d[i] = 1 / sqrt(H[i, i])  (Jacobi equilibration of the SPD system)
__global__ void k_diag_rsqrt(const double* H, int ld, int n, double* d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = 1.0 / sqrt(H[(long)i + (long)i * ld]);
}

// H32 = float(D H D) on the lower tiles (diagonal tiles full).
__global__ __launch_bounds__(256) void k_scale_convert_lower(const double* H, int ld, int n,
                                                             const double* d, float* H32,
                                                             int ld32) {
  const int nt = (n + NB - 1) / NB;
  (void)nt;
  int b = blockIdx.x;
  int i = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= b) ++i;
  while (i * (i + 1) / 2 > b) --i;
  const int j = b - i * (i + 1) / 2;
  const int r0 = i * NB, c0 = j * NB;
  const int mr = min(NB, n - r0), mc = min(NB, n - c0);
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e & 63, c = e >> 6;
    if (r < mr && c < mc) {
      const long o = (long)(r0 + r) + (long)(c0 + c) * ld;
      H32[(long)(r0 + r) + (long)(c0 + c) * ld32] = (float)(H[o] * d[r0 + r] * d[c0 + c]);
    }
  }
}

void equilibrate_convert(const double* H, int ld, int n, double* d, float* H32, int ld32,
                         hipStream_t st) {
  const int nt = (n + NB - 1) / NB;
  k_diag_rsqrt<<<(n + 255) / 256, 256, 0, st>>>(H, ld, n, d);
  k_scale_convert_lower<<<nt * (nt + 1) / 2, 256, 0, st>>>(H, ld, n, d, H32, ld32);
}

// ---------------------------------------------------------------------------
// Triangular solves with the FP32 factor of D H D, three right-hand sides:
//   forward:  y = L^-1 (D r)           (r FP64 in, y FP32 out)
//   backward: x (+)= D L^-T y          (FP64 out, accumulate or overwrite)
// Same ticket/epoch dataflow as the FP64 solves.
constexpr long LPS_SPIN = 1L << 24;

__device__ inline float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(256) void k_trsv3_fwd_lp(const float* __restrict__ L, int ld, int n,
                                                      int nt, const float* __restrict__ linv,
                                                      const double* __restrict__ r,
                                                      const double* __restrict__ d, float* y,
                                                      unsigned long long* ticket, int* flags,
                                                      int* err) {
  __shared__ int s_row, s_epoch, s_ok;
  __shared__ float ys[3][NB];
  __shared__ float part[4][3][NB];
  __shared__ float Ls[NB][NB + 1];
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
  const int rr = t & 63, cg = t >> 6;
  {
    const float* Li = linv + (long)i * NB * NB;
    for (int e = t; e < NB * NB; e += 256) Ls[e >> 6][e & 63] = Li[e];
  }
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
  float lv[16];
  if (i > 0) {
#pragma unroll
    for (int q = 0; q < 16; ++q) lv[q] = (rr < mr) ? L[(long)(r0 + rr) + (long)(cg * 16 + q) * ld] : 0.f;
  }
  for (int p = 0; p < i; ++p) {
    if (t == 0 && !lp_wait(&flags[p], epoch, err)) s_ok = 0;
    __syncthreads();
    if (!s_ok) return;
    if (t < 3 * NB) ys[t >> 6][t & 63] = cload(&y[(long)(t >> 6) * n + p * NB + (t & 63)]);
    __syncthreads();
    float cur[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) cur[q] = lv[q];
    if (p + 1 < i) {
#pragma unroll
      for (int q = 0; q < 16; ++q)
        lv[q] = (rr < mr) ? L[(long)(r0 + rr) + (long)((p + 1) * NB + cg * 16 + q) * ld] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = cg * 16 + q;
      a0 += cur[q] * ys[0][c];
      a1 += cur[q] * ys[1][c];
      a2 += cur[q] * ys[2][c];
    }
    __syncthreads();
  }
  part[cg][0][rr] = a0;
  part[cg][1][rr] = a1;
  part[cg][2][rr] = a2;
  __syncthreads();
  if (t < 3 * NB) {
    const int v = t >> 6, q = t & 63;
    const float b = (q < mr) ? (float)(r[(long)v * n + r0 + q] * d[r0 + q]) : 0.f;
    ys[v][q] = b - (part[0][v][q] + part[1][v][q] + part[2][v][q] + part[3][v][q]);
  }
  __syncthreads();
  if (t < 3 * NB) {
    const int v = t >> 6, q = t & 63;
    float s = 0.f;
    for (int c = 0; c <= q; ++c) s += Ls[c][q] * ys[v][c];
    if (q < mr) cstore(&y[(long)v * n + r0 + q], s);
  }
  lp_publish(&flags[i], epoch);
}

// L^T x = y with L^T read from the upper triangle.
__global__ __launch_bounds__(256) void k_trsv3_bwd_lp(const float* __restrict__ L, int ld, int n,
                                                      int nt, const float* __restrict__ linv,
                                                      const float* __restrict__ y,
                                                      const double* __restrict__ d, float* xs,
                                                      double* x, int accumulate,
                                                      unsigned long long* ticket, int* flags,
                                                      int* err) {
  __shared__ int s_row, s_epoch, s_ok;
  __shared__ float xsh[3][NB];
  __shared__ float part[4][3][NB];
  __shared__ float Ls[NB][NB + 1];
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
  const int rr = t & 63, cg = t >> 6;
  {
    const float* Li = linv + (long)i * NB * NB;
    for (int e = t; e < NB * NB; e += 256) Ls[e >> 6][e & 63] = Li[e];
  }
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
  float lv[16];
  auto load_tile = [&](int p) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int col = p * NB + cg * 16 + q;
      lv[q] = (rr < mr && col < n) ? L[(long)(r0 + rr) + (long)col * ld] : 0.f;
    }
  };
  if (i < nt - 1) load_tile(nt - 1);
  for (int p = nt - 1; p > i; --p) {
    const int pr0 = p * NB, pmr = min(NB, n - pr0);
    if (t == 0 && !lp_wait(&flags[p], epoch, err)) s_ok = 0;
    __syncthreads();
    if (!s_ok) return;
    if (t < 3 * NB) {
      const int v = t >> 6, cc = t & 63;
      xsh[v][cc] = (cc < pmr) ? cload(&xs[(long)v * n + pr0 + cc]) : 0.f;
    }
    __syncthreads();
    float cur[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) cur[q] = lv[q];
    if (p - 1 > i) load_tile(p - 1);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = cg * 16 + q;
      a0 += cur[q] * xsh[0][c];
      a1 += cur[q] * xsh[1][c];
      a2 += cur[q] * xsh[2][c];
    }
    __syncthreads();
  }
  part[cg][0][rr] = a0;
  part[cg][1][rr] = a1;
  part[cg][2][rr] = a2;
  __syncthreads();
  if (t < 3 * NB) {
    const int v = t >> 6, q = t & 63;
    const float b = (q < mr) ? y[(long)v * n + r0 + q] : 0.f;
    xsh[v][q] = b - (part[0][v][q] + part[1][v][q] + part[2][v][q] + part[3][v][q]);
  }
  __syncthreads();
  if (t < 3 * NB) {
    const int v = t >> 6, q = t & 63;
    float s = 0.f;
    for (int c = q; c < NB; ++c) s += Ls[q][c] * xsh[v][c];
    if (q < mr) {
      cstore(&xs[(long)v * n + r0 + q], s);
      const double val = (double)s * d[r0 + q];
      const long o = (long)v * n + r0 + q;
      x[o] = accumulate ? x[o] + val : val;
    }
  }
  lp_publish(&flags[i], epoch);
}

void trsv3_lp_solve(const float* L, int ld, int n, const float* linv_ws, const double* d,
                    const double* r, float* y, float* xs, double* x, int accumulate,
                    unsigned long long* tickets, int* flags, int* err, hipStream_t st) {
  const int nt = (n + NB - 1) / NB;
  k_trsv3_fwd_lp<<<nt, 256, 0, st>>>(L, ld, n, nt, linv_ws, r, d, y, tickets, flags, err);
  k_trsv3_bwd_lp<<<nt, 256, 0, st>>>(L, ld, n, nt, linv_ws, y, d, xs, x, accumulate, tickets + 1,
                                     flags + nt, err);
}

}  // namespace pdk
