// Low-precision factorization of the Schur system for the refined solve:
// the equilibrated matrix D (S + P) D is factored in FP32, with the O(n^3)
// tile products on the FP32 matrix cores (v_mfma_f32_16x16x4f32) or with
// BF16 operands and FP32 accumulation (v_mfma_f32_16x16x32_bf16); diagonal
// tiles and panel solves stay in FP32.  Triangular solves run in FP32 on
// FP64 inputs/outputs; the refinement residual is computed in FP64 elsewhere.
#include <algorithm>
#include "common.h"
#include "tile_factor_f64.h"
#include "df_schedule.h"

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
                              int i, int j, int kend, int nt, const int* flags, int epoch,
                              int* err, int* s_ok, const int* mark) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int r = t & 63, kq = t >> 6;
  if (kend == 0) return true;
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
  int fi = 0, fj = 0, fm = 0;
  if (t == 0) {
    if (!lp_wait(&flags[i * nt], epoch, err) || !lp_wait(&flags[j * nt], epoch, err)) *s_ok = 0;
  }
  __syncthreads();
  if (!*s_ok) return false;
  load_tile(0);
  if (t == 0 && kend > 1) {
    fi = __hip_atomic_load(&flags[i * nt + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    fj = __hip_atomic_load(&flags[j * nt + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  for (int k = 0; k < kend; ++k) {
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
    const bool nxt = k + 1 < kend;
    if (t == 0 && fm == epoch) cu_pause(mark, epoch);
    if (t == 0 && nxt && (fi != epoch || fj != epoch)) {
      if (!lp_wait(&flags[i * nt + k + 1], epoch, err) || !lp_wait(&flags[j * nt + k + 1], epoch, err))
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

// T[e >> 6][e & 63] = src[e] for the 4096 elements of a float tile.
__device__ inline void stage_tile_f(float (*T)[LP_LD], const float* __restrict__ src) {
  const int t = threadIdx.x;
  float v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = src[t + 256 * q];
#pragma unroll
  for (int q = 0; q < 16; ++q) T[(t >> 6) + 4 * q][t & 63] = v[q];
}

// acc(r, c) += sum_kk As[kk][r] Bs[kk][c] over one 64-deep block (FP32 matrix cores).
__device__ inline void lds_product_f(AccF& acc, float (*As)[LP_LD], float (*Bs)[LP_LD]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
#pragma unroll 4
  for (int ks = 0; ks < NB / 4; ++ks) {
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

// T[c][r] = sign * acc(r, c)
__device__ inline void accf_to_lds(const AccF& acc, float (*T)[LP_LD], float sign) {
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) T[accf_col(nb, qq)][accf_row(mb)] = sign * acc.c[mb][nb][qq];
}

// Dataflow Cholesky of a float matrix, on the schedule of the FP64 kernel:
//  * diagonal (j, j): accumulates k < j - 1, finishes the sub-diagonal tile
//    L_{j,j-1} = (A_{j,j-1} - S_j) Linv_{j-1}^T from the partial sum S_j of
//    the task below, adds its last product, then factors and inverts the tile
//    in FP64 (the blocked tile factor of the FP64 kernel) and rounds L and
//    Linv to FP32;
//  * sub-diagonal (j + 1, j): S_{j+1} = sum_{k<j} L_{j+1,k} L_{j,k}^T (FP32)
//    into sbuf, published with its own flag;
//  * (i, j), i >= j + 2: accumulates k < j, waits for Linv_jj, forms
//    L_ij = (A_ij - acc) Linv_jj^T.
// The k < j products use FP32 operands or BF16 operands (FP32 accumulation);
// the finishing products are FP32.  Flags: nt x nt tile flags, then nt unused,
// then nt partial-sum flags (the layout of the FP64 kernel).
template <bool BF16>
__global__ __launch_bounds__(256, 2) void k_potrf_dataflow_lp(float* A, int lda, int n, int nt,
                                                              float* linv_ws, float* sbuf,
                                                              int* flags, unsigned* ticket,
                                                              int* info, int* err, int* cu_marks) {
  const int epoch = (int)ticket[1];
  int* sflags = flags + (nt + 1) * nt;
  int* const mark = cu_marks ? cu_marks + cu_slot() : nullptr;
  // FP64 tile and inverse of the diagonal factor; the float operand tiles of
  // the products live in the same memory
  __shared__ double Tf[NB][LDS_LD];
  __shared__ double Xf[NB][LDS_LD];
  __shared__ int s_task, s_ok;
  float (*buf0)[LP_LD] = reinterpret_cast<float (*)[LP_LD]>(&Tf[0][0]);
  float (*buf1)[LP_LD] = reinterpret_cast<float (*)[LP_LD]>(&Xf[0][0]);
  const int t = threadIdx.x;
  const int ntask = df_task_count(nt, 0);
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
    df_task_of_ticket(q, nt, 0, i, j);
    const bool diag = (i == j), sub = (i == j + 1);
    const bool critical = diag || sub;
    const int r0 = i * NB, c0 = j * NB;
    const int mr = min(NB, n - r0), mc = min(NB, n - c0);
    if (critical) __builtin_amdgcn_s_setprio(2);
    // acc <- -A_ij (identity padding on the diagonal tile), or 0 for the partial sum
    AccF acc;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int r = accf_row(mb), c = accf_col(nb, qq);
          acc.c[mb][nb][qq] = sub ? 0.f
                            : (r < mr && c < mc) ? -cload(&A[(long)(r0 + r) + (long)(c0 + c) * lda])
                                                 : ((diag && r == c) ? -1.f : 0.f);
        }
    const int kend = df_task_kend(i, j);
    if (!lp_accumulate<BF16>(acc, buf0, buf1, A, lda, r0, mr, c0, mc, i, j, kend, nt, flags, epoch,
                             err, &s_ok, critical ? nullptr : mark))
      return;
    if (sub) {
      float* Sb = sbuf + (long)i * NB * NB;
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq)
            cstore(&Sb[accf_row(mb) + NB * accf_col(nb, qq)], acc.c[mb][nb][qq]);
      lp_publish(&sflags[i], epoch);
      __builtin_amdgcn_s_setprio(0);
      continue;
    }
    if (diag && j > 0) {
      const int cs = (j - 1) * NB;
      __syncthreads();                             // last products done with buf0
      {
        const int r = t & 63;
        float v[16];
#pragma unroll
        for (int qq = 0; qq < 16; ++qq)
          v[qq] = (r < mr) ? cload(&A[(long)(r0 + r) + (long)(cs + (t >> 6) + 4 * qq) * lda]) : 0.f;
#pragma unroll
        for (int qq = 0; qq < 16; ++qq) buf0[(t >> 6) + 4 * qq][r] = v[qq];
      }
      if (t == 0 && (!lp_wait(&sflags[j], epoch, err) ||
                     !lp_wait(&flags[(j - 1) * nt + (j - 1)], epoch, err)))
        s_ok = 0;
      __syncthreads();
      if (!s_ok) return;
      if (t == 0 && mark) __hip_atomic_store(mark, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      stage_tile_f(buf1, linv_ws + (long)(j - 1) * NB * NB);   // buf1[kk][c] = Linv(c, kk)
      {
        const float* Sb = sbuf + (long)j * NB * NB;
        float v[16];
#pragma unroll
        for (int qq = 0; qq < 16; ++qq) v[qq] = Sb[t + 256 * qq];
#pragma unroll
        for (int qq = 0; qq < 16; ++qq) buf0[(t >> 6) + 4 * qq][t & 63] -= v[qq];
      }
      __syncthreads();
      AccF l;
      accf_zero(l);
      lds_product_f(l, buf0, buf1);                // L = (A - S) Linv^T
      __syncthreads();
      accf_to_lds(l, buf0, 1.f);
      __syncthreads();
      for (int e = t; e < NB * NB; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (r < mr) cstore(&A[(long)(r0 + r) + (long)(cs + c) * lda], buf0[c][r]);
      }
      lds_product_f(acc, buf0, buf0);              // acc += L L^T, while the stores drain
      lp_publish(&flags[j * nt + (j - 1)], epoch);
      // transposed copy, read only by the backward solve after this launch
      for (int e = t; e < NB * NB; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (c < mr) A[(long)(cs + r) + (long)(r0 + c) * lda] = buf0[r][c];
      }
    }
    __syncthreads();
    if (diag) {
      // C = A_jj - sum_k L_jk L_jk^T = -acc, factored in FP64
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq)
            Tf[accf_col(nb, qq)][accf_row(mb)] = -(double)acc.c[mb][nb][qq];
      __syncthreads();
      if (j == 0 && t == 0 && mark)
        __hip_atomic_store(mark, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      factor_tile_blocked(Tf, Xf, mr, r0, info);
      float* Li = linv_ws + (long)j * NB * NB;
      for (int e = t; e < NB * NB; e += 256) cstore(&Li[e], (float)Xf[e >> 6][e & 63]);
      if (t == 0 && mark) __hip_atomic_store(mark, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      lp_publish(&flags[i * nt + j], epoch);
      for (int e = t; e < NB * NB; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (r < mr && c < mr)
          A[(long)(r0 + r) + (long)(r0 + c) * lda] = (float)((r >= c) ? Tf[c][r] : Tf[r][c]);
      }
    } else {
      accf_to_lds(acc, buf0, -1.f);                // C = A_ij - sum_k L_ik L_jk^T
      if (t == 0 && !lp_wait(&flags[j * nt + j], epoch, err)) s_ok = 0;
      __syncthreads();
      if (!s_ok) return;
      stage_tile_f(buf1, linv_ws + (long)j * NB * NB);
      __syncthreads();
      accf_zero(acc);
      lds_product_f(acc, buf0, buf1);
      __syncthreads();
      accf_to_lds(acc, buf0, 1.f);
      __syncthreads();
      for (int e = t; e < NB * NB; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (r < mr && c < mc) cstore(&A[(long)(r0 + r) + (long)(c0 + c) * lda], buf0[c][r]);
      }
      lp_publish(&flags[i * nt + j], epoch);
      for (int e = t; e < NB * NB; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (c < mr && r < mc) A[(long)(c0 + r) + (long)(r0 + c) * lda] = buf0[r][c];
      }
    }
    if (critical) __builtin_amdgcn_s_setprio(0);
  }
}

void potrf_dataflow_lp(float* A, int lda, int n, float* linv_ws, float* sbuf, int* flags,
                       unsigned* ticket, int* info, int* err, int n_wg, bool bf16, hipStream_t st,
                       int* cu_marks) {
  const int nt = (n + NB - 1) / NB;
  const int ntask = nt * (nt + 1) / 2;
  k_reset_counter_lp<<<1, 1, 0, st>>>(ticket);
  if (bf16)
    k_potrf_dataflow_lp<true><<<std::min(ntask, n_wg), 256, 0, st>>>(
        A, lda, n, nt, linv_ws, sbuf, flags, ticket, info, err, cu_marks);
  else
    k_potrf_dataflow_lp<false><<<std::min(ntask, n_wg), 256, 0, st>>>(
        A, lda, n, nt, linv_ws, sbuf, flags, ticket, info, err, cu_marks);
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
//   b = D r,  L y = b,  L^T z = y,  x (+)= D z
// (the float-factor instances of the FP64 solve kernels: FP64 vectors and
// arithmetic, FP32 matrix reads).
__global__ void k_scale3(int n, const double* __restrict__ d, const double* __restrict__ r,
                         double* __restrict__ b) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * n) return;
  b[e] = r[e] * d[e % n];
}
__global__ void k_unscale3(int n, const double* __restrict__ d, const double* __restrict__ z,
                           double* __restrict__ x, int accumulate) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * n) return;
  const double v = z[e] * d[e % n];
  x[e] = accumulate ? x[e] + v : v;
}

void trsv3_lp_solve(const float* L, int ld, int n, const float* linv_ws, const double* d,
                    const double* r, double* b, double* y, double* x, int accumulate,
                    unsigned long long* tickets, int* err, hipStream_t st) {
  const int g = (3 * n + 255) / 256;
  k_scale3<<<g, 256, 0, st>>>(n, d, r, b);
  // the forward solve puts the sentinel into b as it reads it; z into b
  trsv3_forward(L, ld, n, linv_ws, b, n, y, n, tickets, err, b, n, st);
  trsv3_backward(L, ld, n, linv_ws, y, n, b, n, tickets + 1, err, st);
  k_unscale3<<<g, 256, 0, st>>>(n, d, b, x, accumulate);
}

// ---------------------------------------------------------------------------
// Preconditioned conjugate gradients on H u = g (three independent columns),
// the low-precision factor as preconditioner and H applied in FP64.
// The scalars live in device memory so that no iteration waits for the host.

// out[v] = sum_i a[v][i] b[v][i], one workgroup per column, fixed order.
__global__ __launch_bounds__(256) void k_dot3(int n, const double* __restrict__ a,
                                              const double* __restrict__ b,
                                              double* __restrict__ out) {
  __shared__ double part[256];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += a[(long)v * n + i] * b[(long)v * n + i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = part[0];
}

// With nq = -H p and pnq[v] = p_v . nq_v (= -p_v^T H p_v):
//   alpha_v = rz[v] / (p_v^T H p_v);  u_v += alpha_v p_v;  r_v += alpha_v nq_v.
// A column whose curvature is not positive (converged to exactly zero, or
// broken down) is left unchanged.
__global__ void k_cg_update(int n, const double* __restrict__ rz, const double* __restrict__ pnq,
                            const double* __restrict__ p, const double* __restrict__ nq,
                            double* __restrict__ u, double* __restrict__ r) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * n) return;
  const int v = e / n;
  const double curv = -pnq[v];
  if (!(curv > 0.0)) return;
  const double alpha = rz[v] / curv;
  u[e] += alpha * p[e];
  r[e] += alpha * nq[e];
}

// beta_v = rz_new[v] / rz_old[v] (0 when rz_old is 0);  p_v = z_v + beta_v p_v.
__global__ void k_cg_direction(int n, const double* __restrict__ rz_new,
                               const double* __restrict__ rz_old, const double* __restrict__ z,
                               double* __restrict__ p) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * n) return;
  const int v = e / n;
  const double beta = rz_old[v] != 0.0 ? rz_new[v] / rz_old[v] : 0.0;
  p[e] = z[e] + beta * p[e];
}

void dot3(int n, const double* a, const double* b, double* out, hipStream_t st) {
  k_dot3<<<3, 256, 0, st>>>(n, a, b, out);
}

void cg_update(int n, const double* rz, const double* pnq, const double* p, const double* nq,
               double* u, double* r, hipStream_t st) {
  if (n > 0) k_cg_update<<<(3 * n + 255) / 256, 256, 0, st>>>(n, rz, pnq, p, nq, u, r);
}

void cg_direction(int n, const double* rz_new, const double* rz_old, const double* z, double* p,
                  hipStream_t st) {
  if (n > 0) k_cg_direction<<<(3 * n + 255) / 256, 256, 0, st>>>(n, rz_new, rz_old, z, p);
}

}  // namespace pdk
