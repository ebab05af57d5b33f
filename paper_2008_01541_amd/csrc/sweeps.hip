// Condensation sweeps through the interior factor (one-way dissection in
// breadth-first levels, Z_k = S_k^-1 dense and symmetric, B_k the sparse
// coupling of level k to level k+1 or to the region).  The level chain is
// sequential, so each level is two launches: a dense product with Z_k, and a
// sparse coupling update that also finishes the dense product.
//
// Dense product: (Z_k x)[c] = Z_k[:, c] . x (Z_k symmetric, full storage,
// column-major).  One wave owns 4 columns over one chunk of about 800 rows and
// streams them with 16-byte loads, two row blocks in flight; the chunk
// results (one partial sum per chunk, column and right-hand side) go to a
// small workspace P[chunk][rhs][column], and the coupling launch adds them in
// chunk order, so results do not depend on scheduling.
#include <algorithm>
#include "common.h"

namespace pdk {

namespace {

constexpr int SW_CW = 4;     // columns per wave
constexpr int SW_U = 2;      // row blocks (128 rows each) in flight per wave

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// P[(r * 3 + v) * w + c] = sum over rows j of chunk r of Z[j + c ldz] x[v ldx + j]
__global__ __launch_bounds__(256) void k_sweep_symv(const double* __restrict__ Z, long ldz, int w,
                                                    int R, int chunk, const double* __restrict__ x,
                                                    long ldx, double* __restrict__ P) {
  const int lane = threadIdx.x & 63;
  const int u = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ngroups = (w + SW_CW - 1) / SW_CW;
  if (u >= ngroups * R) return;
  const int g = u / R, r = u - g * R, c0 = g * SW_CW;
  const int j0 = r * chunk, j1 = min(w, j0 + chunk);
  double s[SW_CW][3];
  const double* col[SW_CW];
#pragma unroll
  for (int cc = 0; cc < SW_CW; ++cc) {
    s[cc][0] = s[cc][1] = s[cc][2] = 0.0;
    col[cc] = Z + (long)min(c0 + cc, w - 1) * ldz;   // columns past w repeat the last one
  }
  const double* x0 = x;
  const double* x1 = x + ldx;
  const double* x2 = x + 2 * ldx;
  int j = j0 + 2 * lane;                   // rows j, j + 1 (column starts are 16-byte aligned)
  for (; j + 128 * (SW_U - 1) + 1 < j1; j += 128 * SW_U) {
    double2 z[SW_U][SW_CW];
    double xv[SW_U][3][2];
#pragma unroll
    for (int q = 0; q < SW_U; ++q) {
      const int jj = j + 128 * q;
#pragma unroll
      for (int cc = 0; cc < SW_CW; ++cc) z[q][cc] = *(const double2*)(col[cc] + jj);
      xv[q][0][0] = x0[jj]; xv[q][0][1] = x0[jj + 1];
      xv[q][1][0] = x1[jj]; xv[q][1][1] = x1[jj + 1];
      xv[q][2][0] = x2[jj]; xv[q][2][1] = x2[jj + 1];
    }
#pragma unroll
    for (int q = 0; q < SW_U; ++q)
#pragma unroll
      for (int cc = 0; cc < SW_CW; ++cc)
#pragma unroll
        for (int vv = 0; vv < 3; ++vv)
          s[cc][vv] += z[q][cc].x * xv[q][vv][0] + z[q][cc].y * xv[q][vv][1];
  }
  for (; j < j1; j += 128) {
    const bool two = j + 1 < j1;
#pragma unroll
    for (int cc = 0; cc < SW_CW; ++cc) {
      const double za = col[cc][j], zb = two ? col[cc][j + 1] : 0.0;
      s[cc][0] += za * x0[j] + (two ? zb * x0[j + 1] : 0.0);
      s[cc][1] += za * x1[j] + (two ? zb * x1[j + 1] : 0.0);
      s[cc][2] += za * x2[j] + (two ? zb * x2[j + 1] : 0.0);
    }
  }
#pragma unroll
  for (int cc = 0; cc < SW_CW; ++cc)
#pragma unroll
    for (int vv = 0; vv < 3; ++vv) s[cc][vv] = wave_sum(s[cc][vv]);
  if (lane == 0) {
#pragma unroll
    for (int cc = 0; cc < SW_CW; ++cc)
      if (c0 + cc < w)
#pragma unroll
        for (int vv = 0; vv < 3; ++vv) P[(long)(r * 3 + vv) * w + c0 + cc] = s[cc][vv];
  }
}

// One thread per (row, right-hand side): v[vv][c] = (Z_k x)[c] from the chunk
// sums of P (c < w); xn[vv][t] -= sum_e B(t, e) v[vv][col(e)] (t < rows).  The
// neighbour loop is unrolled so that its loads are in flight together.
__global__ void k_sweep_fwd_couple(int w, int R, const double* __restrict__ P, double* __restrict__ v,
                                   long ldv, int rows, const int32_t* __restrict__ ptr,
                                   const int32_t* __restrict__ col, const double* __restrict__ val,
                                   double* __restrict__ xn, long ldn) {
  const int n = max(w, rows);
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int vv = gt / n, t = gt - vv * n;
  if (vv >= 3) return;
  const double* Pv = P + (long)vv * w;
  const long ldp = 3L * w;
  if (t < w) {
    double s = 0.0;
    for (int r = 0; r < R; ++r) s += Pv[r * ldp + t];
    v[(long)vv * ldv + t] = s;
  }
  if (t < rows) {
    double acc = 0.0;
    const int e1 = ptr[t + 1];
#pragma unroll 4
    for (int e = ptr[t]; e < e1; ++e) {
      const int c = col[e];
      double s = 0.0;
      for (int r = 0; r < R; ++r) s += Pv[r * ldp + c];
      acc += val[e] * s;
    }
    xn[(long)vv * ldn + t] -= acc;
  }
}

// Next level (k + 1) finished: xs_n = v_n - Z_n tmp_n from the chunk sums Q of
// Z_n tmp_n (t < wn); then tmp[t] = sum_e B^T(t, e) x_n[col(e)] for t < rows,
// with x_n = xs_n, or x_n = delta2 when Q is null (level k is the last one).
// One thread per (row, right-hand side).
__global__ void k_sweep_bwd_couple(int wn, int R, const double* __restrict__ Q,
                                   const double* __restrict__ vn, double* __restrict__ xsn, long ldv,
                                   const double* __restrict__ delta2, long ldd, int rows,
                                   const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                   const double* __restrict__ val, double* __restrict__ tmp,
                                   long ldt) {
  const int n = max(Q ? wn : 0, rows);
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int vv = gt / n, t = gt - vv * n;
  if (vv >= 3) return;
  const long ldq = 3L * wn;
  const double* Qv = Q ? Q + (long)vv * wn : nullptr;
  const double* vnv = vn ? vn + (long)vv * ldv : nullptr;
  if (Q && t < wn) {
    double s = 0.0;
    for (int r = 0; r < R; ++r) s += Qv[r * ldq + t];
    xsn[(long)vv * ldv + t] = vnv[t] - s;
  }
  if (t < rows) {
    double acc = 0.0;
    const int e1 = ptr[t + 1];
    if (Q) {
#pragma unroll 4
      for (int e = ptr[t]; e < e1; ++e) {
        const int c = col[e];
        double s = 0.0;
        for (int r = 0; r < R; ++r) s += Qv[r * ldq + c];
        acc += val[e] * (vnv[c] - s);
      }
    } else {
      const double* d2 = delta2 + (long)vv * ldd;
#pragma unroll 4
      for (int e = ptr[t]; e < e1; ++e) acc += val[e] * d2[col[e]];
    }
    tmp[(long)vv * ldt + t] = acc;
  }
}

}  // namespace

void sweep_split(int64_t w, int* R, int* chunk) {
  const int r0 = (int)std::min<int64_t>(8, std::max<int64_t>(1, (w + 400) / 800));
  const int64_t ch = ((w + r0 - 1) / r0 + 127) / 128 * 128;
  *chunk = (int)std::max<int64_t>(128, ch);
  *R = (int)std::max<int64_t>(1, (w + *chunk - 1) / *chunk);
}

void sweep_symv(const double* Z, long ldz, int w, const double* x, long ldx, double* P,
                hipStream_t st) {
  if (w <= 0) return;
  int R, chunk;
  sweep_split(w, &R, &chunk);
  const int units = (w + SW_CW - 1) / SW_CW * R;
  k_sweep_symv<<<(units + 3) / 4, 256, 0, st>>>(Z, ldz, w, R, chunk, x, ldx, P);
}

void sweep_fwd_couple(int w, const double* P, double* v, long ldv, int rows, const int32_t* ptr,
                      const int32_t* col, const double* val, double* xn, long ldn, hipStream_t st) {
  const int n = std::max(w, rows);
  if (n <= 0) return;
  int R, chunk;
  sweep_split(w, &R, &chunk);
  k_sweep_fwd_couple<<<(3 * n + 255) / 256, 256, 0, st>>>(w, R, P, v, ldv, rows, ptr, col, val, xn,
                                                         ldn);
}

void sweep_bwd_couple(int wn, const double* Q, const double* vn, double* xsn, long ldv,
                      const double* delta2, long ldd, int rows, const int32_t* ptr,
                      const int32_t* col, const double* val, double* tmp, long ldt,
                      hipStream_t st) {
  const int n = std::max(Q ? wn : 0, rows);
  if (n <= 0) return;
  int R = 1, chunk;
  if (Q) sweep_split(wn, &R, &chunk);
  k_sweep_bwd_couple<<<(3 * n + 255) / 256, 256, 0, st>>>(wn, R, Q, vn, xsn, ldv, delta2, ldd,
                                                          rows, ptr, col, val, tmp, ldt);
}

}  // namespace pdk
