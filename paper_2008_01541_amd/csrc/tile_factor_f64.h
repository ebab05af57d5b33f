// Device-side building blocks shared by the dataflow Cholesky kernels: the
// factor and inverse of a 64 x 64 diagonal tile held in LDS (FP64, matrix
// cores for the blocked updates, DPP row broadcasts for the 16 x 16 diagonal
// blocks), and the per-compute-unit marks by which tasks off the critical
// path yield to the diagonal task.  Header-only: included by each kernel file.
#pragma once
#include "common.h"
#include "publish.h"

namespace pdk {

constexpr int LDS_LD = NB + 4;   // padded LDS row (doubles)

// DPP row broadcast (row_newbcast: every lane of a row of 16 lanes reads lane
// S of that row), as volatile asm; s_nop 1 covers the two wait states a DPP
// read needs after a VALU write of its source.
template <int S>
__device__ __forceinline__ double row_bcast(double v) {
  double o;
  asm volatile("s_nop 1\n\tv_mov_b64_dpp %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0xf"
               : "=v"(o)
               : "v"(v), "i"(S));
  return o;
}
// Per-step update blocks of the 16 x 16 diagonal-block Cholesky:
// chol16_a_updates<C>(a) -> next pivot, chol16_x_updates<C>(a, x).
#include "chol16_steps.inc"

// 1/sqrt(d): the hardware estimate (relative error up to about 5e-8 on this
// chip) refined by one third-order step, y <- y (1 + e/2 + 3 e^2/8) with
// e = 1 - d y^2: four dependent operations for an error of about 2.4 ulp (two
// Newton steps reach the same accuracy in six).
__device__ __forceinline__ double rsqrt_newton(double d) {
  const double y = __builtin_amdgcn_rsq(d);
  const double e = fma(-(d * y), y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}

// Right-looking elimination of one 16 x 16 block, one pivot per step C: lane
// r (mod 16) holds row r of the block in a[] and column r of the inverse in
// x[] (initially the identity); the multipliers L(S, C) are broadcast along
// each row of 16 lanes (one asm block of DPP operands per step and array).
// The pivot of step C + 1 is broadcast as soon as its own update is done, so
// that its square root can overlap the rest of step C.
template <int C>
__device__ __forceinline__ void chol16_step(double (&a)[16], double (&x)[16], double d, int r,
                                            int& bad) {
  if constexpr (C < 16) {
    const bool ok = d > 0.0;
    bad = (!ok && bad == 0) ? C + 1 : bad;
    const double y = ok ? rsqrt_newton(d) : 1.0;
    // column C of L, d y on the diagonal and a y below; the lanes above the
    // diagonal (r < C) only carry values of the upper part, which no later
    // step reads into the lower part, and are cleared after the last step
    a[C] *= y;
    x[C] *= y;
    double dn = 0.0;
    if constexpr (C + 1 < 16) {
      dn = chol16_a_updates<C>(a);
      chol16_x_updates<C>(a, x);
    }
    chol16_step<C + 1>(a, x, dn, r, bad);
  }
}

// Cholesky factor and inverse of the 16 x 16 diagonal block at (b0, b0) of the
// LDS tile T, by one wave (the four rows of 16 lanes work redundantly), into
// registers: lane r (mod 16) ends with row r of L in a[] (zeros above the
// diagonal) and column r of its inverse in x[].  The first non-positive pivot
// j of the block (inside the first mr rows) is reported in *info as
// gbase + b0 + j + 1, and its reciprocal square root is taken as 1.
__device__ __forceinline__ void chol16_factor(double (*T)[LDS_LD], int b0, int mr, int gbase,
                                              int* info, double (&a)[16], double (&x)[16]) {
  const int lane = threadIdx.x & 63, r = lane & 15;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    a[c] = T[b0 + c][b0 + r];
    x[c] = (c == r) ? 1.0 : 0.0;
  }
  int bad = 0;          // first non-positive pivot of the block, 1-based; 0: none
  chol16_step<0>(a, x, row_bcast<0>(a[0]), r, bad);
  if (lane == 0 && bad > 0 && b0 + bad - 1 < mr) atomicCAS(info, 0, gbase + b0 + bad);
#pragma unroll
  for (int c = 0; c < 16; ++c) a[c] = (r >= c) ? a[c] : 0.0;
}

// L replaces the lower part of the block (zeros above), its inverse goes to
// the same block of X (zeros above).
__device__ __forceinline__ void chol16_store(double (*T)[LDS_LD], double (*X)[LDS_LD], int b0,
                                             const double (&a)[16], const double (&x)[16]) {
  const int lane = threadIdx.x & 63, r = lane & 15;
  if (lane < 16) {
#pragma unroll
    for (int c = 0; c < 16; ++c) T[b0 + c][b0 + r] = a[c];
#pragma unroll
    for (int i = 0; i < 16; ++i) X[b0 + r][b0 + i] = x[i];
  }
}

__device__ __forceinline__ void chol16_inverse(double (*T)[LDS_LD], double (*X)[LDS_LD], int b0,
                                               int mr, int gbase, int* info) {
  double a[16], x[16];
  chol16_factor(T, b0, mr, gbase, info, a, x);
  chol16_store(T, X, b0, a, x);
}

// C(m, n) += sum_k A(m, k) B(n, k) over one 16-deep block, m, n, k < 16, for
// operands in LDS tiles (Ts[c][r] = tile(r, c)): A(m, k) = As[ak + k][am + m],
// B(n, k) = Bs[bk + k][bn + n] (BT = false) or Bs[bn + n][bk + k] (BT = true).
// Result: lane l, register q holds C(l % 16, l / 16 + 4 q).
template <bool BT>
__device__ inline void mma16(double4_t& acc, double (*As)[LDS_LD], int am, int ak,
                             double (*Bs)[LDS_LD], int bn, int bk) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = 4 * s + (lane >> 4);
    const double av = As[ak + k][am + (lane & 15)];
    const double bv = BT ? Bs[bn + (lane & 15)][bk + k] : Bs[bk + k][bn + (lane & 15)];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bv, av, acc, 0, 0, 0);
  }
}

// Cholesky of a 64 x 64 tile held in LDS (T[c][r] = tile(r, c), lower part
// valid, rows/cols >= mr padded with the identity) and the inverse of the
// factor into X (X[c][r] = inverse(r, c), zero above the diagonal).  Right-
// looking over 16-wide block columns: wave 0 factors and inverts the diagonal
// block, the panel below becomes P Dinv^T and the trailing blocks are updated
// on the matrix cores.  The off-diagonal blocks of the inverse follow from
// X_ij = -X_ii Y_ij, Y_ij = sum_{p=j}^{i-1} L_ip X_pj; wave 1 + j owns block
// column j of the inverse and does that work while wave 0 factors the next
// diagonal block (the staged Y_ij waits in the X_ij slot until X_ii exists),
// so only the last block row is left after the final diagonal block.  A
// non-positive pivot stores its 1-based global index gbase + j + 1 in *info
// (first one wins) and its reciprocal square root is taken as 1 so that the
// factorization stays finite.  Only the lower triangle of T is meaningful on return.
//
// With lflag != NULL, X enters holding a 64 x 64 tile B (X[k][r] = B(r, k))
// and the tile factored is T - B B^T: wave 0 subtracts B B^T from the first
// diagonal block and factors it at once, while waves 1-3 update the nine other
// lower blocks; once B has been read by every wave, *lflag = epoch is
// published (after this workgroup's earlier global stores have drained) and X
// is reused for the inverse.  The last rank-64 update of a diagonal tile thus
// overlaps the factorization of its first block.
__device__ __forceinline__ void factor_tile_blocked(double (*T)[LDS_LD], double (*X)[LDS_LD], int mr, int gbase,
                                    int* info, int* lflag = nullptr, int epoch = 0) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // zero the six strictly upper 16 x 16 blocks of X: X[16 jb + c][16 ib + r], ib < jb
  const auto zero_upper_x = [&]() {
    for (int e = t; e < 6 * 256; e += 256) {
      const int blk = e >> 8, r = e & 15, c = (e >> 4) & 15;
      const int ib = blk < 3 ? 0 : (blk < 5 ? 1 : 2);
      const int jb = blk < 3 ? blk + 1 : (blk < 5 ? blk - 1 : 3);
      X[16 * jb + c][16 * ib + r] = 0.0;
    }
  };
  // Y_ij into the X_ij slot / X_ij = -X_ii Y_ij in place (one wave each)
  const auto inv_stage = [&](int i, int j) {
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int p = j; p < i; ++p) mma16<true>(acc, T, 16 * i, 16 * p, X, 16 * j, 16 * p);
#pragma unroll
    for (int q = 0; q < 4; ++q) X[16 * j + (lane >> 4) + 4 * q][16 * i + (lane & 15)] = acc[q];
  };
  const auto inv_finish = [&](int i, int j) {
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    mma16<true>(acc, X, 16 * i, 16 * i, X, 16 * j, 16 * i);
    __builtin_amdgcn_wave_barrier();      // all lanes have read Y before X_ij overwrites it
#pragma unroll
    for (int q = 0; q < 4; ++q) X[16 * j + (lane >> 4) + 4 * q][16 * i + (lane & 15)] = -acc[q];
  };
  if (lflag) {
    // T block (ib, jb) -= sum_{k < 64} B(16 ib + m, k) B(16 jb + n, k)
    const auto b_update = [&](int ib, int jb) {
      double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) mma16<false>(acc, X, 16 * ib, 16 * s, X, 16 * jb, 16 * s);
#pragma unroll
      for (int q = 0; q < 4; ++q) T[16 * jb + (lane >> 4) + 4 * q][16 * ib + (lane & 15)] -= acc[q];
    };
    if (w == 0) {
      b_update(0, 0);
      // the block just written by other lanes of this wave is read below
      __builtin_amdgcn_wave_barrier();
      double a[16], x[16];
      chol16_factor(T, 0, mr, gbase, info, a, x);
      // L_00 in place; its inverse waits in the unused upper block (0, 1) of
      // T, in the layout of X (T[16 + c][r] = inverse(r, c)), until B has
      // been read
      chol16_store(T, T + 16, 0, a, x);
    } else {
      // lower blocks of block rows 1..3 in row order, three per wave:
      // (1,0) (1,1) (2,0) | (2,1) (2,2) (3,0) | (3,1) (3,2) (3,3)
      for (int u = 0; u < 3; ++u) {
        const int idx = 3 * (w - 1) + u;
        const int ib = idx < 2 ? 1 : (idx < 5 ? 2 : 3);
        const int jb = idx - (ib == 1 ? 0 : (ib == 2 ? 2 : 5));
        b_update(ib, jb);
      }
    }
    publish_flag(lflag, epoch);           // B read by every wave: X is free
    zero_upper_x();
    X[t >> 4][t & 15] = T[16 + (t >> 4)][t & 15];   // X_00 (256 threads, one element each)
  } else {
    zero_upper_x();
    if (w == 0) chol16_inverse(T, X, 0, mr, gbase, info);
  }
  __syncthreads();
  for (int kb = 0; kb < 3; ++kb) {
    const int b0 = 16 * kb;
    // panel: block row ib = kb + 1 + w becomes P Dinv^T
    if (kb + 1 + w <= 3) {
      const int ib = kb + 1 + w;
      double4_t acc = {0.0, 0.0, 0.0, 0.0};
      mma16<false>(acc, T, 16 * ib, b0, X, b0, b0);
#pragma unroll
      for (int q = 0; q < 4; ++q) T[b0 + (lane >> 4) + 4 * q][16 * ib + (lane & 15)] = acc[q];
    }
    __syncthreads();
    // trailing blocks (ib, jb), kb < jb <= ib <= 3; wave 0 takes the next
    // diagonal block and goes straight on to factor it
    const int R = 3 - kb, nblk = R * (R + 1) / 2;
    for (int bi = (w == 0 ? 0 : w); bi < nblk; bi += (w == 0 ? nblk : 3)) {
      int jb = kb + 1, rem = bi;
      while (rem >= 4 - jb) { rem -= 4 - jb; ++jb; }
      const int ib = jb + rem;
      double4_t acc = {0.0, 0.0, 0.0, 0.0};
      mma16<false>(acc, T, 16 * ib, b0, T, 16 * jb, b0);
#pragma unroll
      for (int q = 0; q < 4; ++q) T[16 * jb + (lane >> 4) + 4 * q][16 * ib + (lane & 15)] -= acc[q];
    }
    if (w == 0) {
      chol16_inverse(T, X, b0 + 16, mr, gbase, info);
    } else {
      // meanwhile, block column j = w - 1 of the inverse: finish row kb,
      // stage row kb + 1 (the panels up to kb and X_kk are final)
      const int j = w - 1;
      if (j < kb) inv_finish(kb, j);
      // X_{kb,j} just written by other lanes of this wave is read below: the
      // wave barrier keeps the compiler from moving loads across those stores
      __builtin_amdgcn_wave_barrier();
      if (j <= kb) inv_stage(kb + 1, j);
    }
    __syncthreads();
  }
  // last block row of the inverse: X_3j = -X_33 Y_3j
  if (w >= 1) inv_finish(3, w - 1);
  __syncthreads();
}

// Compute-unit courtesy.  The diagonal tasks form the critical path of the
// factorization; their local phase (finishing the sub-diagonal tile, the tile
// factor, the inverse) runs on one compute unit and, with two workgroups per
// unit, shares its FP64 pipes with the other one's products.  A diagonal task
// marks its unit busy (slot cu_slot(), value = launch epoch) for that phase;
// tasks off the critical path that find their unit marked sleep at their next
// k-step until the mark is cleared.  The diagonal task waits for nothing while
// marked, so the pause is short; it is bounded anyway, and the marks only
// steer timing, never results.
constexpr int CU_SLOTS = 2048;
__device__ inline int cu_slot() {
  const unsigned hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);    // HW_ID: SE, SH, CU in bits 15:8
  const unsigned xcc = __builtin_amdgcn_s_getreg((31 << 11) | 20);  // XCC_ID
  return (int)(((xcc & 7u) << 8) | ((hw >> 8) & 0xffu));
}
__device__ inline void cu_pause(const int* mark, int epoch) {
  for (int s = 0; s < 4096; ++s) {                                   // at most ~0.5 ms
    __builtin_amdgcn_s_sleep(8);
    if (__hip_atomic_load(mark, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) return;
  }
}

}  // namespace pdk
