// Kernels of the nested-dissection (multifrontal) interior factor: extend-add
// of a child's update matrix into its parent's front, and the batched
// matrix-vector products of the two sweeps through the supernodes (three
// right-hand sides).  Supernode s holds X_s = L_ss^-1 (n_s x n_s, lower) and
// L_Bs (b_s x n_s, the rows of its boundary), column-major.  Sums run in a
// fixed order, so the sweeps are bitwise reproducible.
#include "common.h"

namespace pdk {

// Lower entries (r >= c) of a child's b x b update matrix U into its parent's
// front.  The map is increasing, so i = map[r] >= j = map[c]: columns j < ns
// go to the front's first ns columns P (F_ss entries also to their mirror,
// which the dense factorization may read inside a diagonal tile), the rest to
// the trailing update block Uo at (i - ns, j - ns), mirrored when asked.
// Distinct (r, c) give distinct destinations, and the children of one front
// are added one launch after another, so no two threads add into one entry.
__global__ void k_nd_extend_add(const double* __restrict__ U, long ldu, int b,
                                const int32_t* __restrict__ map, int ns, double* __restrict__ P,
                                long ldp, double* __restrict__ Uo, long lduo, int mirror) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)b * b) return;
  const int r = (int)(e % b), c = (int)(e / b);
  if (r < c) return;
  const double v = U[r + (long)c * ldu];
  const int i = map[r], j = map[c];
  if (j < ns) {
    P[(long)i + (long)j * ldp] += v;
    if (i < ns && i != j) P[(long)j + (long)i * ldp] += v;
  } else {
    Uo[(long)(i - ns) + (long)(j - ns) * lduo] += v;
    if (mirror && i != j) Uo[(long)(j - ns) + (long)(i - ns) * lduo] += v;
  }
}
void nd_extend_add(const double* U, long ldu, int b, const int32_t* map, int ns, double* P,
                   long ldp, double* Uo, long lduo, int mirror, hipStream_t st) {
  const long cnt = (long)b * b;
  if (cnt > 0)
    k_nd_extend_add<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>(U, ldu, b, map, ns, P, ldp, Uo,
                                                                   lduo, mirror);
}

// dst[v][o] = f[v][node_of[t]] - sum_{e in [ptr[t], ptr[t+1])} contrib[v][slot[e]]
// for the cnt targets t listed in tlist: t < n1 is an elimination position
// (o = t), t >= n1 the region node t - n1 (o = t - n1).  The contributions
// of a target are subtracted in the order of its slot list.
__global__ void k_nd_gather_rhs(int cnt, const int32_t* __restrict__ tlist, int n1,
                                const int32_t* __restrict__ node_of, const double* __restrict__ f,
                                long ldf, const int32_t* __restrict__ ptr,
                                const int32_t* __restrict__ slot, const double* __restrict__ contrib,
                                long ldc, double* __restrict__ dst, long ldd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int t = tlist[i];
  const long node = node_of[t];
  const int out = t < n1 ? t : t - n1;
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    double s = f[v * ldf + node];
    for (int e = ptr[t]; e < ptr[t + 1]; ++e) s -= contrib[v * ldc + slot[e]];
    dst[v * ldd + out] = s;
  }
}
void nd_gather_rhs(int cnt, const int32_t* tlist, int n1, const int32_t* node_of, const double* f,
                   long ldf, const int32_t* ptr, const int32_t* slot, const double* contrib,
                   long ldc, double* dst, long ldd, hipStream_t st) {
  if (cnt > 0)
    k_nd_gather_rhs<<<(cnt + 255) / 256, 256, 0, st>>>(cnt, tlist, n1, node_of, f, ldf, ptr, slot,
                                                       contrib, ldc, dst, ldd);
}

// y[yoff + row0 + r] = sum_c M(row0 + r, c) x[xoff + c] (three columns of x
// and y, strides ldx / ldy), one workgroup per item of 64 rows; lower: M is
// lower triangular (columns c <= row).  Thread (r, g) adds columns g, g + 4,
// ...; the four partial sums are added in a fixed order through LDS.
__global__ __launch_bounds__(256) void k_nd_gemv_n(const NdItem* __restrict__ items,
                                                   const double* __restrict__ Mb,
                                                   const double* __restrict__ x, long ldx,
                                                   double* __restrict__ y, long ldy, int lower) {
  __shared__ double part[4][3][64];
  const NdItem it = items[blockIdx.x];
  if (it.rows <= 0) return;
  const int t = threadIdx.x, r = t & 63, g = t >> 6;
  const int row = it.row0 + r;
  const int rr = min(row, it.rows - 1);
  const int cend = lower ? min(it.cols, it.row0 + 64) : it.cols;
  const double* M = Mb + it.moff + rr;
  const double* xv = x + it.xoff;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int c = g; c < cend; c += 4) {
    const double m = (lower && c > rr) ? 0.0 : M[(long)c * it.ldm];
    s0 += m * xv[c];
    s1 += m * xv[ldx + c];
    s2 += m * xv[2 * ldx + c];
  }
  part[g][0][r] = s0;
  part[g][1][r] = s1;
  part[g][2][r] = s2;
  __syncthreads();
  if (t < 192) {
    const int v = t >> 6, q = t & 63;
    if (it.row0 + q < it.rows)
      y[v * ldy + it.yoff + it.row0 + q] =
          (part[0][v][q] + part[1][v][q]) + (part[2][v][q] + part[3][v][q]);
  }
}
void nd_gemv_n(int nitems, const NdItem* items, const double* M, const double* x, long ldx,
               double* y, long ldy, int lower, hipStream_t st) {
  if (nitems > 0) k_nd_gemv_n<<<nitems, 256, 0, st>>>(items, M, x, ldx, y, ldy, lower);
}

__device__ inline double nd_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// y[yoff + c] = sum_r M(r, c) (xa - xb)[xoff + r] for the four columns
// c = col0 + w of an item (one wave each; xb may be null); lower: rows r >= c
// only.  Each wave walks its column in 64-row steps and adds up across lanes.
__global__ __launch_bounds__(256) void k_nd_gemv_t(const NdItem* __restrict__ items,
                                                   const double* __restrict__ Mb,
                                                   const double* __restrict__ xa,
                                                   const double* __restrict__ xb, long ldx,
                                                   double* __restrict__ y, long ldy, int lower) {
  const NdItem it = items[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = it.row0 + w;                  // row0 holds the first column of the item
  if (c >= it.cols) return;
  const double* M = Mb + it.moff + (long)c * it.ldm;
  const double* a = xa + it.xoff;
  const double* b = xb ? xb + it.xoff : nullptr;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int r = (lower ? c : 0) + lane; r < it.rows; r += 64) {
    const double m = M[r];
    double v0 = a[r], v1 = a[ldx + r], v2 = a[2 * ldx + r];
    if (b) {
      v0 -= b[r];
      v1 -= b[ldx + r];
      v2 -= b[2 * ldx + r];
    }
    s0 += m * v0;
    s1 += m * v1;
    s2 += m * v2;
  }
  s0 = nd_wave_sum(s0);
  s1 = nd_wave_sum(s1);
  s2 = nd_wave_sum(s2);
  if (lane == 0) {
    y[it.yoff + c] = s0;
    y[ldy + it.yoff + c] = s1;
    y[2 * ldy + it.yoff + c] = s2;
  }
}
void nd_gemv_t(int nitems, const NdItem* items, const double* M, const double* xa, const double* xb,
               long ldx, double* y, long ldy, int lower, hipStream_t st) {
  if (nitems > 0) k_nd_gemv_t<<<nitems, 256, 0, st>>>(items, M, xa, xb, ldx, y, ldy, lower);
}

// zb[v][e] = (t < n1) ? z[v][t] : d2[v][t - n1] with t = key[e], for the
// cnt boundary entries e listed in elist.
__global__ void k_nd_gather_zb(int cnt, const int32_t* __restrict__ elist,
                               const int32_t* __restrict__ key, int n1,
                               const double* __restrict__ z, long ldz,
                               const double* __restrict__ d2, long ldd2, double* __restrict__ zb,
                               long ldzb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int e = elist[i], t = key[e];
#pragma unroll
  for (int v = 0; v < 3; ++v)
    zb[v * ldzb + e] = t < n1 ? z[v * ldz + t] : d2[v * ldd2 + (t - n1)];
}
void nd_gather_zb(int cnt, const int32_t* elist, const int32_t* key, int n1, const double* z,
                  long ldz, const double* d2, long ldd2, double* zb, long ldzb, hipStream_t st) {
  if (cnt > 0)
    k_nd_gather_zb<<<(cnt + 255) / 256, 256, 0, st>>>(cnt, elist, key, n1, z, ldz, d2, ldd2,
                                                      zb, ldzb);
}

}  // namespace pdk
