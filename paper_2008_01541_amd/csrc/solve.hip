// Three-right-hand-side triangular solves with the tiled factor of the
// dataflow Cholesky (Alg. 1 step 4.5: the forward and backward substitution
// of the region system, one factor for the x, y and z columns).
#include <algorithm>
#include "common.h"
#include "publish.h"

namespace pdk {

// ---------------------------------------------------------------------------
// Three-right-hand-side triangular solves with the tiled factor.  One
// workgroup per block row; rows are claimed in dependency order through a
// ticket counter, so every claimed row only waits on rows claimed earlier by
// running workgroups.  Row completion is published with a per-call epoch.

constexpr long SPIN_LIMIT = 1L << 24;

__device__ inline bool wait_flag(int* f, int epoch, int* err) {
  long spins = 0;
  while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(1);
    if (++spins > SPIN_LIMIT) {
      atomicExch(err, 1);
      return false;
    }
  }
  return true;
}

// Two tile rows per workgroup ("super-row" s: tile rows TR s and TR s + 1), so
// that one cross-workgroup hand-off covers 128 rows of the solve.  Thread
// t works on row r = t & 63 of a tile and on the 16 columns cg = t >> 6 of it;
// the four column groups are added through LDS.
constexpr int TR = 2;

// sums the four column-group partials of part (3 x 64 per group) into out[v][rr]
// = base[v][rr] - sum; base may be null (then out = sum).
__device__ inline void trsv_reduce(double (*part)[3][NB], const double* base, int ldb, int r0,
                                   int mr, double (*out)[NB], bool negate) {
  const int t = threadIdx.x;
  if (t < 3 * NB) {
    const int v = t >> 6, rr = t & 63;
    const double sum = part[0][v][rr] + part[1][v][rr] + part[2][v][rr] + part[3][v][rr];
    const double b = (base && rr < mr) ? base[(long)v * ldb + r0 + rr] : 0.0;
    out[v][rr] = negate ? b - sum : sum;
  }
}

// Loads of a column panel of a column-major matrix through a buffer
// descriptor: the row goes in the lane offset, the column (relative to the
// panel's first one) in the scalar offset, so that a load needs no 64-bit
// address registers.  Byte offsets stay below 2^32 within a panel.
template <typename T>
__device__ inline __amdgpu_buffer_rsrc_t panel_rsrc(const T* L, long ld, int col0, int ncol) {
  const unsigned long long b = reinterpret_cast<unsigned long long>(L + (long)col0 * ld);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  const unsigned long long bytes = (unsigned long long)ncol * ld * sizeof(T);
  const unsigned nrec = bytes < 0xffffffffull ? (unsigned)bytes : 0xffffffffu;
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((unsigned long long)hi << 32) | lo),
                                           0, (int)__builtin_amdgcn_readfirstlane(nrec), 0x00020000);
}
template <typename T>
__device__ inline T panel_load(__amdgpu_buffer_rsrc_t rs, int voff, int soff);
template <>
__device__ inline double panel_load<double>(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
}
template <>
__device__ inline float panel_load<float>(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}

// L y = g.  Tile row i: y_i = Linv_ii (g_i - sum_{p<i} L_ip y_p).
// With fflags, the factor is still being computed by a dataflow Cholesky
// launch on another stream (its tile flags and its ticket[2], whose epoch
// ticket[1] that launch uses): each super-row first waits until the diagonal
// tile of its last row is published, which implies that every tile of its
// rows and both tile inverses are final.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_trsv3_fwd(const T* __restrict__ L, int ld, int n,
                                                   int nt, const T* __restrict__ linv,
                                                   const double* __restrict__ g, int ldg,
                                                   double* y, int ldy,
                                                   unsigned long long* ticket, int* flags,
                                                   int* err, const int* fflags,
                                                   const unsigned* fticket) {
  __shared__ int s_row, s_epoch, s_ok;
  __shared__ double Ls[TR][NB][NB + 1];     // Ls[u][c][r] = Linv_{i_u}(r, c)
  __shared__ double ys[3][TR * NB];         // y of a finished super-row / of this one
  __shared__ double part[4][3][NB];
  __shared__ double zs[3][NB];
  const int t = threadIdx.x;
  const int ns = (nt + TR - 1) / TR;
  if (t == 0) {
    const unsigned long long tk = atomicAdd(ticket, 1ull);
    s_row = (int)(tk % (unsigned long long)ns);
    s_epoch = (int)(tk / (unsigned long long)ns) + 1;
    s_ok = 1;
  }
  __syncthreads();
  const int sr = s_row, epoch = s_epoch;
  const int r = t & 63, cg = t >> 6;
  const int cgs = __builtin_amdgcn_readfirstlane(cg);    // cg is uniform per wave
  const int i0 = TR * sr, nu = min(TR, nt - i0);
  if (fflags) {
    if (t == 0) {
      const int fe = (int)__hip_atomic_load(&fticket[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int il = i0 + nu - 1;
      if (!df_wait(&fflags[il * nt + il], fe, err)) s_ok = 0;
    }
    __syncthreads();
    if (!s_ok) return;
  }
  for (int u = 0; u < nu; ++u) {
    const T* Li = linv + (long)(i0 + u) * NB * NB;
    double v16[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v16[q] = Li[t + 256 * q];
#pragma unroll
    for (int q = 0; q < 16; ++q) Ls[u][(t >> 6) + 4 * q][t & 63] = v16[q];
  }
  // the coupling tile L_{i0+1, i0} (this thread's row and 16 columns), read
  // now so that its latency is off the path when the super-row finishes
  static_assert(TR == 2, "the coupling prefetch assumes two tile rows per super-row");
  T lc[16];
  {
    const int r1 = (i0 + 1) * NB + r;
    const bool ok = nu > 1 && r1 < n;
    const T* Lr = ok ? L + r1 + (long)(i0 * NB + cg * 16) * ld : L;
    const long cs = ok ? (long)ld : 0;
#pragma unroll
    for (int c = 0; c < 16; ++c) lc[c] = Lr[c * cs] * (ok ? T(1) : T(0));
  }
  double acc[TR][3];
#pragma unroll
  for (int u = 0; u < TR; ++u) acc[u][0] = acc[u][1] = acc[u][2] = 0.0;
  for (int q = 0; q < sr; ++q) {
    // the four operand tiles L_{i_u, TR q + u'} (16 columns each) load while the flag is awaited
    // unconditional loads from a clamped row, then a select: no branch per
    // load, so all of them are in flight together
    // (rows past the edge re-read row 0 and are masked by a multiply, so no
    // load is put under a branch)
    T lv[TR][TR][16];
    const __amdgpu_buffer_rsrc_t prs = panel_rsrc(L, ld, TR * q * NB, TR * NB);
#pragma unroll
    for (int u = 0; u < TR; ++u) {
      const int ru = (i0 + u) * NB + r;
      const bool ok = u < nu && ru < n;
      const int voff = (ok ? ru : 0) * (int)sizeof(T);
#pragma unroll
      for (int w = 0; w < TR; ++w)
#pragma unroll
        for (int c = 0; c < 16; ++c)
          lv[u][w][c] = panel_load<T>(prs, voff, (w * NB + cgs * 16 + c) * ld * (int)sizeof(T)) *
                        (ok ? T(1) : T(0));
    }
    if (t == 0 && !wait_flag(&flags[q], epoch, err)) s_ok = 0;
    __syncthreads();
    if (!s_ok) return;
    for (int e = t; e < 3 * TR * NB; e += 256) {
      const int v = e / (TR * NB), cc = e - v * TR * NB;
      ys[v][cc] = coherent_load(&y[(long)v * ldy + TR * q * NB + cc]);
    }
    __syncthreads();
    // each operand of ys is read once and used for every tile row; four
    // columns at a time, so that the operands are not all held at once
#pragma unroll
    for (int w = 0; w < TR; ++w)
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int col = w * NB + cg * 16 + c;
        const double y0 = ys[0][col], y1 = ys[1][col], y2 = ys[2][col];
#pragma unroll
        for (int u = 0; u < TR; ++u) {
          acc[u][0] += (double)lv[u][w][c] * y0;
          acc[u][1] += (double)lv[u][w][c] * y1;
          acc[u][2] += (double)lv[u][w][c] * y2;
        }
        if ((c & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    __syncthreads();
  }
  // finish the tile rows of this super-row in order
  for (int u = 0; u < nu; ++u) {
    const int i = i0 + u, r0 = i * NB, mr = min(NB, n - r0);
    if (u > 0) {           // coupling to the row finished above in this super-row
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int col = cg * 16 + c;
        const double l = (double)lc[c];
        acc[u][0] += l * ys[0][col];
        acc[u][1] += l * ys[1][col];
        acc[u][2] += l * ys[2][col];
      }
    }
    part[cg][0][r] = acc[u][0];
    part[cg][1][r] = acc[u][1];
    part[cg][2][r] = acc[u][2];
    __syncthreads();
    trsv_reduce(part, g, ldg, r0, mr, zs, true);        // zs = g_i - sum
    __syncthreads();
    // y_i = Linv_ii zs: column group cg adds columns 16 cg .. 16 cg + 15
    {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int col = cg * 16 + c;
        const double l = Ls[u][col][r];
        s0 += l * zs[0][col];
        s1 += l * zs[1][col];
        s2 += l * zs[2][col];
      }
      part[cg][0][r] = s0;
      part[cg][1][r] = s1;
      part[cg][2][r] = s2;
    }
    __syncthreads();
    if (t < 3 * NB) {
      const int v = t >> 6, rr = t & 63;
      const double yv = part[0][v][rr] + part[1][v][rr] + part[2][v][rr] + part[3][v][rr];
      ys[v][u * NB + rr] = yv;
      if (rr < mr) coherent_store(&y[(long)v * ldy + r0 + rr], yv);
    }
    __syncthreads();
  }
  publish_flag(&flags[sr], epoch);
}

// L^T x = y, reading L^T from the upper triangle (U(r, c) = L(c, r) for c > r):
// x_i = Linv_ii^T (y_i - sum_{p>i} U_ip x_p).  Super-rows from the bottom.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_trsv3_bwd(const T* __restrict__ L, int ld, int n,
                                                   int nt, const T* __restrict__ linv,
                                                   const double* __restrict__ y, int ldy,
                                                   double* x, int ldx,
                                                   unsigned long long* ticket, int* flags,
                                                   int* err) {
  __shared__ int s_row, s_epoch, s_ok;
  __shared__ double Ls[TR][NB][NB + 1];     // Ls[u][c][r] = Linv_{i_u}(r, c)
  __shared__ double xs[3][TR * NB];
  __shared__ double part[4][3][NB];
  __shared__ double zs[3][NB];
  const int t = threadIdx.x;
  const int ns = (nt + TR - 1) / TR;
  if (t == 0) {
    const unsigned long long tk = atomicAdd(ticket, 1ull);
    s_row = ns - 1 - (int)(tk % (unsigned long long)ns);
    s_epoch = (int)(tk / (unsigned long long)ns) + 1;
    s_ok = 1;
  }
  __syncthreads();
  const int sr = s_row, epoch = s_epoch;
  const int r = t & 63, cg = t >> 6;
  const int cgs = __builtin_amdgcn_readfirstlane(cg);    // cg is uniform per wave
  const int i0 = TR * sr, nu = min(TR, nt - i0);
  for (int u = 0; u < nu; ++u) {
    const T* Li = linv + (long)(i0 + u) * NB * NB;
    double v16[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v16[q] = Li[t + 256 * q];
#pragma unroll
    for (int q = 0; q < 16; ++q) Ls[u][(t >> 6) + 4 * q][t & 63] = v16[q];
  }
  // the coupling tile U_{i0, i0+1} (this thread's row of tile row i0, 16
  // columns of tile i0 + 1), read now so that its latency is off the path
  static_assert(TR == 2, "the coupling prefetch assumes two tile rows per super-row");
  T lc[16];
  {
    const int wn = nu > 1 ? min(NB, n - (i0 + 1) * NB) : 0;
    const int rr0 = i0 * NB + r;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int col = cg * 16 + c;
      const bool ok = col < wn;
      const T* p = ok ? L + rr0 + (long)((i0 + 1) * NB + col) * ld : L;
      lc[c] = *p * (ok ? T(1) : T(0));
    }
  }
  double acc[TR][3];
#pragma unroll
  for (int u = 0; u < TR; ++u) acc[u][0] = acc[u][1] = acc[u][2] = 0.0;
  for (int q = ns - 1; q > sr; --q) {
    T lv[TR][TR][16];
    const int pc0 = TR * q * NB;
    const __amdgpu_buffer_rsrc_t prs = panel_rsrc(L, ld, pc0, min(TR * NB, n - pc0));
#pragma unroll
    for (int u = 0; u < TR; ++u) {
      const int ru = (i0 + u) * NB + r;
      const bool okr = u < nu && ru < n;
      const int voff = (okr ? ru : 0) * (int)sizeof(T);
#pragma unroll
      for (int w = 0; w < TR; ++w)
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const int col = (TR * q + w) * NB + cgs * 16 + c;
          // columns past the edge re-read the last one; a multiply, not a
          // select, masks them, so that the load is not put under a branch
          lv[u][w][c] = panel_load<T>(prs, voff, (min(col, n - 1) - pc0) * ld * (int)sizeof(T)) *
                        ((okr && col < n) ? T(1) : T(0));
        }
    }
    if (t == 0 && !wait_flag(&flags[q], epoch, err)) s_ok = 0;
    __syncthreads();
    if (!s_ok) return;
    const int qn = min(TR * NB, n - TR * q * NB);
    for (int e = t; e < 3 * TR * NB; e += 256) {
      const int v = e / (TR * NB), cc = e - v * TR * NB;
      xs[v][cc] = (cc < qn) ? coherent_load(&x[(long)v * ldx + TR * q * NB + cc]) : 0.0;
    }
    __syncthreads();
    // each operand of xs is read once and used for every tile row; four
    // columns at a time, so that the operands are not all held at once
#pragma unroll
    for (int w = 0; w < TR; ++w)
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int col = w * NB + cg * 16 + c;
        const double y0 = xs[0][col], y1 = xs[1][col], y2 = xs[2][col];
#pragma unroll
        for (int u = 0; u < TR; ++u) {
          acc[u][0] += (double)lv[u][w][c] * y0;
          acc[u][1] += (double)lv[u][w][c] * y1;
          acc[u][2] += (double)lv[u][w][c] * y2;
        }
        if ((c & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    __syncthreads();
  }
  for (int u = nu - 1; u >= 0; --u) {
    const int i = i0 + u, r0 = i * NB, mr = min(NB, n - r0);
    if (u + 1 < nu) {      // coupling to the row finished below in this super-row
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int col = cg * 16 + c;
        const double l = (double)lc[c];
        acc[u][0] += l * xs[0][NB + col];
        acc[u][1] += l * xs[1][NB + col];
        acc[u][2] += l * xs[2][NB + col];
      }
    }
    part[cg][0][r] = acc[u][0];
    part[cg][1][r] = acc[u][1];
    part[cg][2][r] = acc[u][2];
    __syncthreads();
    trsv_reduce(part, y, ldy, r0, mr, zs, true);        // zs = y_i - sum
    __syncthreads();
    // x_i = Linv_ii^T zs: (Linv^T z)(rr) = sum_c Linv(c, rr) z(c) = sum_c Ls[rr][c] z(c);
    // thread (r, cg) adds c = 16 cg .. 16 cg + 15 for output row r
    {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int col = cg * 16 + c;
        const double l = Ls[u][r][col];
        s0 += l * zs[0][col];
        s1 += l * zs[1][col];
        s2 += l * zs[2][col];
      }
      part[cg][0][r] = s0;
      part[cg][1][r] = s1;
      part[cg][2][r] = s2;
    }
    __syncthreads();
    if (t < 3 * NB) {
      const int v = t >> 6, rr = t & 63;
      const double xv = part[0][v][rr] + part[1][v][rr] + part[2][v][rr] + part[3][v][rr];
      xs[v][u * NB + rr] = xv;
      if (rr < mr) coherent_store(&x[(long)v * ldx + r0 + rr], xv);
    }
    __syncthreads();
  }
  publish_flag(&flags[sr], epoch);
}

void trsv3_forward(const double* L, int ld, int n, const double* linv_ws, const double* g,
                   int ldg, double* y, int ldy, unsigned long long* ticket, int* flags,
                   int* err, hipStream_t st, const int* fflags, const unsigned* fticket) {
  const int nt = (n + NB - 1) / NB, ns = (nt + TR - 1) / TR;
  k_trsv3_fwd<double><<<ns, 256, 0, st>>>(L, ld, n, nt, linv_ws, g, ldg, y, ldy, ticket, flags, err,
                                          fflags, fticket);
}

void trsv3_backward(const double* L, int ld, int n, const double* linv_ws, const double* y,
                    int ldy, double* x, int ldx, unsigned long long* ticket, int* flags,
                    int* err, hipStream_t st) {
  const int nt = (n + NB - 1) / NB, ns = (nt + TR - 1) / TR;
  k_trsv3_bwd<double><<<ns, 256, 0, st>>>(L, ld, n, nt, linv_ws, y, ldy, x, ldx, ticket, flags, err);
}

// The same solves with a float factor (FP64 vectors and arithmetic).
void trsv3_forward(const float* L, int ld, int n, const float* linv_ws, const double* g, int ldg,
                   double* y, int ldy, unsigned long long* ticket, int* flags, int* err,
                   hipStream_t st) {
  const int nt = (n + NB - 1) / NB, ns = (nt + TR - 1) / TR;
  k_trsv3_fwd<float><<<ns, 256, 0, st>>>(L, ld, n, nt, linv_ws, g, ldg, y, ldy, ticket, flags, err,
                                         nullptr, nullptr);
}
void trsv3_backward(const float* L, int ld, int n, const float* linv_ws, const double* y, int ldy,
                    double* x, int ldx, unsigned long long* ticket, int* flags, int* err,
                    hipStream_t st) {
  const int nt = (n + NB - 1) / NB, ns = (nt + TR - 1) / TR;
  k_trsv3_bwd<float><<<ns, 256, 0, st>>>(L, ld, n, nt, linv_ws, y, ldy, x, ldx, ticket, flags, err);
}

}  // namespace pdk
