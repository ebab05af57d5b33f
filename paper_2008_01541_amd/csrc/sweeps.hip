// Condensation sweeps through the interior factor as single cooperative
// launches.  The level chain is sequential (level k+1 needs all of level k),
// so one persistent grid walks the levels with grid-wide barriers between the
// dense symmetric products (Z_k times three columns) and the sparse coupling
// updates, instead of two launches per level.
#include <algorithm>
#include "common.h"

namespace pdk {

namespace {

constexpr long SW_SPIN_LIMIT = 1L << 24;

__device__ inline double cld(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void cst(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Grid barrier number b (0, 1, ...) on a counter that starts at zero.
__device__ inline bool grid_barrier(unsigned* cnt, unsigned target, int* err) {
  __builtin_amdgcn_s_waitcnt(0x0F70);     // own stores complete
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    ok = 1;
    atomicAdd(cnt, 1u);
    long spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) { ok = 0; break; }
      __builtin_amdgcn_s_sleep(1);
      if (++spins > SW_SPIN_LIMIT) {
        atomicExch(err, 1);
        ok = 0;
        break;
      }
    }
  }
  __syncthreads();
  return ok != 0;
}

// y[col] (=|+=) alpha * (Z[:, col] . v) for 8-column groups owned by this
// workgroup (group g = blockIdx.x, blockIdx.x + gridDim.x, ...).  v is read
// with coherent loads (it may have been written earlier in this launch).
__device__ void level_symv(const double* __restrict__ Z, long ldz, int w, const double* v, long ldv,
                           double alpha, bool accumulate, double* y, long ldy, double (*vs)[512]) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int ngroups = (w + 7) / 8;
  for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const int c0 = g * 8 + wv * 2;
    const double* a0 = Z + (long)min(c0, w - 1) * ldz;
    const double* a1 = Z + (long)min(c0 + 1, w - 1) * ldz;
    double s[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int j0 = 0; j0 < w; j0 += 512) {
      const int cnt = min(512, w - j0);
      __syncthreads();
      for (int e = t; e < 3 * 512; e += 256) {
        const int vv = e >> 9, jj = e & 511;
        vs[vv][jj] = (jj < cnt) ? cld(&v[(long)vv * ldv + j0 + jj]) : 0.0;
      }
      __syncthreads();
      if (cnt == 512 && ((ldz & 1) == 0)) {
#pragma unroll
        for (int it = 0; it < 4; ++it) {
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
      for (int vv = 0; vv < 3; ++vv) s[cc][vv] = wsum(s[cc][vv]);
    if (lane == 0) {
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const int col = c0 + cc;
        if (col >= w) continue;
#pragma unroll
        for (int vv = 0; vv < 3; ++vv) {
          double* yo = y + (long)vv * ldy + col;
          cst(yo, accumulate ? cld(yo) + alpha * s[cc][vv] : alpha * s[cc][vv]);
        }
      }
    }
  }
}

// y[r] = base[r] + alpha * sum_e val[e] v[col[e]] for rows r of a CSR block,
// rows spread over the whole grid; v and base read coherently.
__device__ void level_spmv(int rows, const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                           const double* __restrict__ val, const double* v, long ldv, double alpha,
                           double* y, long ldy, bool has_base) {
  const long nthr = (long)gridDim.x * blockDim.x;
  for (long r = (long)blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += nthr) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int32_t e = ptr[r]; e < ptr[r + 1]; ++e) {
      const double a = val[e];
      const long c = col[e];
      s0 += a * cld(&v[c]);
      s1 += a * cld(&v[ldv + c]);
      s2 += a * cld(&v[2 * ldv + c]);
    }
    const double b0 = has_base ? cld(&y[r]) : 0.0;
    const double b1 = has_base ? cld(&y[ldy + r]) : 0.0;
    const double b2 = has_base ? cld(&y[2 * ldy + r]) : 0.0;
    cst(&y[r], b0 + alpha * s0);
    cst(&y[ldy + r], b1 + alpha * s1);
    cst(&y[2 * ldy + r], b2 + alpha * s2);
  }
}

}  // namespace

// Forward sweep: for k = 0..K-1: v_k = Z_k fhat_k;
//   fhat_{k+1} -= B_k v_k  (k+1 < K)   or   y2 -= B_{K-1} v_{K-1}.
// fhat and y2 hold the gathered forces on entry.
__global__ __launch_bounds__(256) void k_sweep_forward(const SweepDesc d, double* fhat, double* v,
                                                       double* y2, unsigned* bar, int* err) {
  __shared__ double vs[3][512];
  unsigned b = 0;
  const unsigned G = gridDim.x;
  for (int k = 0; k < d.K; ++k) {
    const long off = d.lev_off[k];
    const int w = (int)(d.lev_off[k + 1] - off);
    level_symv(d.levmat + d.mat_off[k], d.ldw[k], w, fhat + off, d.n1, 1.0, false, v + off, d.n1, vs);
    if (!grid_barrier(bar, G * ++b, err)) return;
    const int32_t* bp = d.Bptr + d.B_ptr_off[k];
    const int32_t* bc = d.Bcol + d.B_nnz_off[k];
    const double* bv = d.Bval + d.B_nnz_off[k];
    if (k + 1 < d.K) {
      const long off2 = d.lev_off[k + 1];
      const int w2 = (int)(d.lev_off[k + 2] - off2);
      level_spmv(w2, bp, bc, bv, v + off, d.n1, -1.0, fhat + off2, d.n1, true);
    } else {
      level_spmv(d.m, bp, bc, bv, v + off, d.n1, -1.0, y2, d.m, true);
    }
    if (!grid_barrier(bar, G * ++b, err)) return;
  }
}

// Backward sweep: xs = v; for k = K-1..0: tmp = B_k^T x_{k+1} (x_K = delta2);
//   xs_k -= Z_k tmp.
__global__ __launch_bounds__(256) void k_sweep_backward(const SweepDesc d, const double* v,
                                                        const double* delta2, double* xs,
                                                        double* tmp, unsigned* bar, int* err) {
  __shared__ double vs[3][512];
  unsigned b = 0;
  const unsigned G = gridDim.x;
  {
    const long nthr = (long)G * blockDim.x;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < 3L * d.n1; e += nthr)
      cst(&xs[e], v[e]);
  }
  if (!grid_barrier(bar, G * ++b, err)) return;
  for (int k = d.K - 1; k >= 0; --k) {
    const long off = d.lev_off[k];
    const int w = (int)(d.lev_off[k + 1] - off);
    const int32_t* tp = d.Btptr + d.Bt_ptr_off[k];
    const int32_t* tc = d.Btcol + d.Bt_nnz_off[k];
    const double* tv = d.Btval + d.Bt_nnz_off[k];
    const double* xn = (k + 1 < d.K) ? xs + d.lev_off[k + 1] : delta2;
    const long ldxn = (k + 1 < d.K) ? d.n1 : d.m;
    level_spmv(w, tp, tc, tv, xn, ldxn, 1.0, tmp, d.maxw, false);
    if (!grid_barrier(bar, G * ++b, err)) return;
    level_symv(d.levmat + d.mat_off[k], d.ldw[k], w, tmp, d.maxw, -1.0, true, xs + off, d.n1, vs);
    if (!grid_barrier(bar, G * ++b, err)) return;
  }
}

__global__ void k_zero_u32(unsigned* p) { *p = 0u; }

static int sweep_grid(const void* kernel) {
  static int cached = 0;
  if (cached) return cached;
  int dev = 0, ncu = 256, per = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0) != hipSuccess || per < 1) per = 1;
  cached = ncu * std::min(per, 2);
  return cached;
}

hipError_t sweep_forward(const SweepDesc& d, double* fhat, double* v, double* y2, unsigned* bar,
                         int* err, hipStream_t st) {
  if (d.K == 0) return hipSuccess;
  k_zero_u32<<<1, 1, 0, st>>>(bar);
  const int G = sweep_grid((const void*)k_sweep_forward);
  SweepDesc dd = d;
  void* args[] = {(void*)&dd, (void*)&fhat, (void*)&v, (void*)&y2, (void*)&bar, (void*)&err};
  return hipLaunchCooperativeKernel((const void*)k_sweep_forward, dim3(G), dim3(256), args, 0, st);
}

hipError_t sweep_backward(const SweepDesc& d, const double* v, const double* delta2, double* xs,
                          double* tmp, unsigned* bar, int* err, hipStream_t st) {
  if (d.K == 0) return hipSuccess;
  k_zero_u32<<<1, 1, 0, st>>>(bar);
  const int G = sweep_grid((const void*)k_sweep_backward);
  SweepDesc dd = d;
  void* args[] = {(void*)&dd, (void*)&v, (void*)&delta2, (void*)&xs, (void*)&tmp, (void*)&bar,
                  (void*)&err};
  return hipLaunchCooperativeKernel((const void*)k_sweep_backward, dim3(G), dim3(256), args, 0, st);
}

}  // namespace pdk
