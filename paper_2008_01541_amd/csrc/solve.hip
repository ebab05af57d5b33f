// Three-right-hand-side triangular solves with the tiled factor of the
// dataflow Cholesky (Alg. 1 step 4.5: the forward and backward substitution
// of the region system, one factor for the x, y and z columns).
#include <algorithm>
#include "common.h"
#include "publish.h"

namespace pdk {

// ---------------------------------------------------------------------------
// Three-right-hand-side triangular solves with the tiled factor.  One
// workgroup per pair of block rows; rows are claimed in dependency order
// through a ticket counter, so every claimed row only waits on rows claimed
// earlier by running workgroups.
//
// Publication by value: the vector a solve produces (y of the forward solve,
// x of the backward one) holds a sentinel before the solve (a signalling NaN
// bit pattern, which no arithmetic produces: every NaN an operation returns
// is quiet); each value is published by its own agent-coherent 8-byte store,
// and a consumer polls the values of a block row with coherent loads until
// none is the sentinel.  This takes one round trip per hand-off instead of a
// flag (stores drained, flag stored, flag polled, data loaded).  The
// sentinels are written by the solve that consumes the previous content:
// the forward solve puts them into x as it reads each value of its right-hand
// side (so x may alias the right-hand side), the backward solve puts them
// back into y as it reads y, and sentinel_fill() prepares a vector once.

constexpr long SPIN_LIMIT = 1L << 24;
constexpr unsigned long long SENTINEL = 0x7FF0DEAD00000001ull;   // signalling NaN

__device__ inline bool is_sentinel(double v) {
  return __builtin_bit_cast(unsigned long long, v) == SENTINEL;
}

__global__ void k_sentinel_fill(long n, double* p) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = __builtin_bit_cast(double, SENTINEL);
}
void sentinel_fill(long n, double* p, hipStream_t st) {
  if (n > 0) k_sentinel_fill<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, p);
}

// Workgroup barrier for data exchanged through LDS only: waits for this
// wave's LDS operations, not for its global loads and stores in flight (the
// barrier of __syncthreads also waits for those, which puts the latency of
// every write-through store of a published value on the chain).
__device__ inline void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Polls the cnt values v[0 .. cnt - 1] of the three columns (v[c * ldv + e])
// into out[c][e] until none is the sentinel; false (and *err set) after the
// spin limit or when another workgroup has set *err.  Uniform over the block.
template <int CAP>
__device__ inline bool poll_block(const double* v, int ldv, int cnt, double (*out)[CAP],
                                  int (*s_miss)[4], int* err) {
  const int t = threadIdx.x;
  long spins = 0;
  for (int it = 0;; it ^= 1) {
    int miss = 0;
    for (int e = t; e < 3 * CAP; e += 256) {
      const int c = e / CAP, cc = e - c * CAP;
      double val = 0.0;
      if (cc < cnt) {
        val = coherent_load(&v[(long)c * ldv + cc]);
        miss |= is_sentinel(val) ? 1 : 0;
      }
      out[c][cc] = val;
    }
    // one slot per wave, two sets used alternately so that a slot is not
    // rewritten before every wave has read it
    const bool wmiss = __ballot(miss) != 0;
    if ((t & 63) == 0) s_miss[it][t >> 6] = wmiss ? 1 : 0;
    lds_barrier();
    if (!(s_miss[it][0] | s_miss[it][1] | s_miss[it][2] | s_miss[it][3])) return true;
    if (++spins > SPIN_LIMIT ||
        __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
      if (t == 0) atomicExch(err, 1);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Two tile rows per workgroup ("super-row" s: tile rows TR s and TR s + 1), so
// that one cross-workgroup hand-off covers 128 rows of the solve.  Thread
// t works on row r = t & 63 of a tile and on the 16 columns cg = t >> 6 of it;
// the four column groups are added through LDS.
constexpr int TR = 2;

// sums the four column-group partials of part (3 x 64 per group) into out[v][rr]
// = base[v][rr] - sum; base may be null (then out = sum).
// out[v][rr] = b - (sum of the four column-group partials of part) for
// thread t = 64 v + rr < 192, b = this thread's right-hand-side value.
__device__ inline void trsv_reduce(double (*part)[3][NB], double b, double (*out)[NB]) {
  const int t = threadIdx.x;
  if (t < 3 * NB) {
    const int v = t >> 6, rr = t & 63;
    const double sum = part[0][v][rr] + part[1][v][rr] + part[2][v][rr] + part[3][v][rr];
    out[v][rr] = b - sum;
  }
}

// The right-hand-side values of the TR tile rows from i0 on, one per thread
// t = 64 v + rr < 192 (rows past n: 0), read at the start so that their
// latency is off the chain; fill (may alias base) gets the sentinel at each
// value once it is read, by the thread that read it.
template <int R>
__device__ inline void load_rhs(const double* base, int ldb, int i0, int nu, int n, double* fill,
                                int ldf, double (&b)[R]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int u = 0; u < R; ++u) b[u] = 0.0;
  if (t < 3 * NB) {
    const int v = t >> 6, rr = t & 63;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int row = (i0 + u) * NB + rr;
      if (u < nu && row < n) {
        b[u] = base[(long)v * ldb + row];
        if (fill) fill[(long)v * ldf + row] = __builtin_bit_cast(double, SENTINEL);
      }
    }
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
                                                   const double* g, int ldg,
                                                   double* y, int ldy,
                                                   unsigned long long* ticket, int* err,
                                                   const int* fflags, const unsigned* fticket,
                                                   double* xfill, int ldxf) {
  __shared__ int s_row, s_ok;
  __shared__ double Ls[TR][NB][NB + 1];     // Ls[u][c][r] = Linv_{i_u}(r, c)
  __shared__ double ys[3][TR * NB];         // y of a finished super-row / of this one
  __shared__ int s_miss[2][4];
  __shared__ double part[4][3][NB];
  __shared__ double zs[3][NB];
  const int t = threadIdx.x;
  const int ns = (nt + TR - 1) / TR;
  if (t == 0) {
    const unsigned long long tk = atomicAdd(ticket, 1ull);
    s_row = (int)(tk % (unsigned long long)ns);
    s_ok = 1;
  }
  lds_barrier();
  const int sr = s_row;
  const int r = t & 63, cg = t >> 6;
  const int cgs = __builtin_amdgcn_readfirstlane(cg);    // cg is uniform per wave
  const int i0 = TR * sr, nu = min(TR, nt - i0);
  double rhs[TR];
  load_rhs<TR>(g, ldg, i0, nu, n, xfill, ldxf, rhs);
  if (fflags) {
    if (t == 0) {
      const int fe = (int)__hip_atomic_load(&fticket[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int il = i0 + nu - 1;
      if (!df_wait(&fflags[il * nt + il], fe, err)) s_ok = 0;
    }
    lds_barrier();
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
    if (!poll_block<TR * NB>(y + (long)TR * q * NB, ldy, TR * NB, ys, s_miss, err)) return;
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
    lds_barrier();
  }
  // finish the tile rows of this super-row in order (unrolled, so that the
  // accumulators acc[u] are indexed at compile time, not through register
  // indexing)
#pragma unroll
  for (int u = 0; u < TR; ++u) {
    if (u >= nu) break;
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
    lds_barrier();
    trsv_reduce(part, rhs[u], zs);                      // zs = g_i - sum
    lds_barrier();
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
    lds_barrier();
    if (t < 3 * NB) {
      const int v = t >> 6, rr = t & 63;
      const double yv = part[0][v][rr] + part[1][v][rr] + part[2][v][rr] + part[3][v][rr];
      ys[v][u * NB + rr] = yv;
      if (rr < mr) coherent_store(&y[(long)v * ldy + r0 + rr], yv);   // published
    }
    lds_barrier();
  }
}

// L^T x = y, reading L^T from the upper triangle (U(r, c) = L(c, r) for c > r):
// x_i = Linv_ii^T (y_i - sum_{p>i} U_ip x_p).  Super-rows from the bottom.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_trsv3_bwd(const T* __restrict__ L, int ld, int n,
                                                   int nt, const T* __restrict__ linv,
                                                   double* y, int ldy,
                                                   double* x, int ldx,
                                                   unsigned long long* ticket, int* err) {
  __shared__ int s_row, s_ok;
  __shared__ double Ls[TR][NB][NB + 1];     // Ls[u][c][r] = Linv_{i_u}(r, c)
  __shared__ double xs[3][TR * NB];
  __shared__ int s_miss[2][4];
  __shared__ double part[4][3][NB];
  __shared__ double zs[3][NB];
  const int t = threadIdx.x;
  const int ns = (nt + TR - 1) / TR;
  if (t == 0) {
    const unsigned long long tk = atomicAdd(ticket, 1ull);
    s_row = ns - 1 - (int)(tk % (unsigned long long)ns);
    s_ok = 1;
  }
  lds_barrier();
  const int sr = s_row;
  const int r = t & 63, cg = t >> 6;
  const int cgs = __builtin_amdgcn_readfirstlane(cg);    // cg is uniform per wave
  const int i0 = TR * sr, nu = min(TR, nt - i0);
  double rhs[TR];
  load_rhs<TR>(y, ldy, i0, nu, n, y, ldy, rhs);        // y refilled with the sentinel
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
    const int qn = min(TR * NB, n - TR * q * NB);
    if (!poll_block<TR * NB>(x + (long)TR * q * NB, ldx, qn, xs, s_miss, err)) return;
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
    lds_barrier();
  }
  // (unrolled, so that the accumulators acc[u] are indexed at compile time)
#pragma unroll
  for (int uu = 0; uu < TR; ++uu) {
    const int u = TR - 1 - uu;
    if (u >= nu) continue;
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
    lds_barrier();
    trsv_reduce(part, rhs[u], zs);                      // zs = y_i - sum
    lds_barrier();
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
    lds_barrier();
    if (t < 3 * NB) {
      const int v = t >> 6, rr = t & 63;
      const double xv = part[0][v][rr] + part[1][v][rr] + part[2][v][rr] + part[3][v][rr];
      xs[v][u * NB + rr] = xv;
      if (rr < mr) coherent_store(&x[(long)v * ldx + r0 + rr], xv);   // published
    }
    lds_barrier();
  }
}

void trsv3_forward(const double* L, int ld, int n, const double* linv_ws, const double* g,
                   int ldg, double* y, int ldy, unsigned long long* ticket, int* err,
                   double* xfill, int ldxf, hipStream_t st, const int* fflags,
                   const unsigned* fticket) {
  const int nt = (n + NB - 1) / NB, ns = (nt + TR - 1) / TR;
  k_trsv3_fwd<double><<<ns, 256, 0, st>>>(L, ld, n, nt, linv_ws, g, ldg, y, ldy, ticket, err,
                                          fflags, fticket, xfill, ldxf);
}

void trsv3_backward(const double* L, int ld, int n, const double* linv_ws, double* y, int ldy,
                    double* x, int ldx, unsigned long long* ticket, int* err, hipStream_t st) {
  const int nt = (n + NB - 1) / NB, ns = (nt + TR - 1) / TR;
  k_trsv3_bwd<double><<<ns, 256, 0, st>>>(L, ld, n, nt, linv_ws, y, ldy, x, ldx, ticket, err);
}

// The same solves with a float factor (FP64 vectors and arithmetic).
void trsv3_forward(const float* L, int ld, int n, const float* linv_ws, const double* g, int ldg,
                   double* y, int ldy, unsigned long long* ticket, int* err, double* xfill,
                   int ldxf, hipStream_t st) {
  const int nt = (n + NB - 1) / NB, ns = (nt + TR - 1) / TR;
  k_trsv3_fwd<float><<<ns, 256, 0, st>>>(L, ld, n, nt, linv_ws, g, ldg, y, ldy, ticket, err,
                                         nullptr, nullptr, xfill, ldxf);
}
void trsv3_backward(const float* L, int ld, int n, const float* linv_ws, double* y, int ldy,
                    double* x, int ldx, unsigned long long* ticket, int* err, hipStream_t st) {
  const int nt = (n + NB - 1) / NB, ns = (nt + TR - 1) / TR;
  k_trsv3_bwd<float><<<ns, 256, 0, st>>>(L, ld, n, nt, linv_ws, y, ldy, x, ldx, ticket, err);
}

}  // namespace pdk
