// Kernels of the nested-dissection (multifrontal) interior factor: extend-add
// of a child's update matrix into its parent's front, and the batched
// matrix-vector products of the two sweeps through the supernodes (three
// right-hand sides).  Supernode s keeps Z_s = A_ss^-1 (n_s x n_s, symmetric)
// stacked above W_s = F_Bs Z_s (b_s x n_s), and W_s^T, all column-major, so
// that every product of a sweep sums down contiguous columns: the forward
// sweep reads W_s^T (contributions W_s r_s to the boundary), the backward
// sweep the stacked block (x_s = Z_s r_s - W_s^T zb_s).  Sums run in a fixed
// order, so the sweeps are bitwise reproducible.
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

// dst[v][out] = f[v][node] - sum_{c0 <= e < c1} contrib[v][e] for the cnt
// targets of trec (the forward products store their contributions
// target-major, so each target's are contiguous).  Eight lanes share a
// target: lane k adds entries k, k + 8, ..., then the eight partial sums are
// combined by a fixed butterfly, so loads of different entries are in flight
// together and the result does not depend on timing.  A target costs two
// dependent loads: its record, then its contributions and force.
__global__ __launch_bounds__(256) void k_nd_gather_rhs(int cnt, const NdTarget* __restrict__ trec,
                                                       const double* __restrict__ f, long ldf,
                                                       const double* __restrict__ contrib,
                                                       long ldc, double* __restrict__ dst,
                                                       long ldd) {
  const int g = (int)((blockIdx.x * (long)blockDim.x + threadIdx.x) >> 3);
  const int k = threadIdx.x & 7;
  const bool on = g < cnt;
  const NdTarget tr = on ? trec[g] : NdTarget{0, 0, 0, 0};
  const double fv = (on && k < 3) ? f[k * ldf + tr.node] : 0.0;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int e = tr.c0 + k; e < tr.c1; e += 8) {
    s0 += contrib[e];
    s1 += contrib[ldc + e];
    s2 += contrib[2 * ldc + e];
  }
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, 64);
    s1 += __shfl_xor(s1, o, 64);
    s2 += __shfl_xor(s2, o, 64);
  }
  if (on && k < 3) dst[k * ldd + tr.out] = fv - (k == 0 ? s0 : (k == 1 ? s1 : s2));
}
void nd_gather_rhs(int cnt, const NdTarget* trec, const double* f, long ldf,
                   const double* contrib, long ldc, double* dst, long ldd, hipStream_t st) {
  if (cnt > 0)
    k_nd_gather_rhs<<<(cnt + 31) / 32, 256, 0, st>>>(cnt, trec, f, ldf, contrib, ldc, dst, ldd);
}

// Partner exchange of a transposed reduction: the lanes with bit hi set keep
// value b and give a away, the others keep a and give b; returns kept +
// the partner's given, i.e. the pair's sum of the value this lane keeps.
__device__ inline double nd_xchg(double a, double b, bool hi, int mask) {
  const double give = hi ? a : b, keep = hi ? b : a;
  return keep + __shfl_xor(give, mask, 64);
}

// Wave sums of the twelve values s[0..11]: every exchange halves the values
// a lane still carries (6 -> 3 -> 2 -> 1, then two plain rounds), 14
// exchanges instead of 72.  Value idx = 6 b5 + 3 b4 + 2 b3 + b2 (bits of the
// lane; b3 = b2 = 1 carries padding) ends, summed over the wave in a fixed
// order, in the four lanes with those bits.
__device__ inline double nd_wave_sum12(const double (&s)[12], int& idx) {
  const int lane = threadIdx.x & 63;
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
  double t[6], u[3];
#pragma unroll
  for (int k = 0; k < 6; ++k) t[k] = nd_xchg(s[k], s[6 + k], b5, 32);
#pragma unroll
  for (int k = 0; k < 3; ++k) u[k] = nd_xchg(t[k], t[3 + k], b4, 16);
  const double w0 = nd_xchg(u[0], u[2], b3, 8);
  const double w1 = nd_xchg(u[1], 0.0, b3, 8);
  double x = nd_xchg(w0, w1, b2, 4);
  x += __shfl_xor(x, 2, 64);
  x += __shfl_xor(x, 1, 64);
  idx = (b5 ? 6 : 0) + (b4 ? 3 : 0) + (b3 ? 2 : 0) + (b2 ? 1 : 0);
  return x;
}

// The same for three values: value idx = 2 b5 + b4 (b5 = b4 = 1: padding)
// ends in the sixteen lanes with those bits.
__device__ inline double nd_wave_sum3(double s0, double s1, double s2, int& idx) {
  const int lane = threadIdx.x & 63;
  const bool b5 = lane & 32, b4 = lane & 16;
  const double w0 = nd_xchg(s0, s2, b5, 32);
  const double w1 = nd_xchg(s1, 0.0, b5, 32);
  double x = nd_xchg(w0, w1, b4, 16);
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  idx = (b5 ? 2 : 0) + (b4 ? 1 : 0);
  return x;
}

// s += sign * sum_{r < n} M[r] x[r] (three columns of x, stride ldx) over
// this lane's rows lane, lane + 64, ...: four rows per step, loads guarded
// rather than branched around, so that a short column takes one step with
// all its loads in flight.
template <int SIGN>
__device__ __forceinline__ void nd_dot(const double* __restrict__ M, const double* __restrict__ x,
                                       long ldx, int n, double& s0, double& s1, double& s2) {
  const int lane = threadIdx.x & 63;
  for (int r = lane; r < n; r += 256) {
    double m[4], v0[4], v1[4], v2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = r + 64 * u;
      const bool ok = q < n;
      m[u] = ok ? M[q] : 0.0;
      v0[u] = ok ? x[q] : 0.0;
      v1[u] = ok ? x[ldx + q] : 0.0;
      v2[u] = ok ? x[2 * ldx + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (SIGN > 0) {
        s0 += m[u] * v0[u];
        s1 += m[u] * v1[u];
        s2 += m[u] * v2[u];
      } else {
        s0 -= m[u] * v0[u];
        s1 -= m[u] * v1[u];
        s2 -= m[u] * v2[u];
      }
    }
  }
}

// The same for four columns M, M + ldm, M + 2 ldm, M + 3 ldm at once (nc of
// them valid): the vector entries are loaded once for the four, two rows
// per lane and step.
template <int SIGN>
__device__ __forceinline__ void nd_dot4(const double* __restrict__ M, long ldm, int nc,
                                        const double* __restrict__ x, long ldx, int n,
                                        double (&s)[4][3]) {
  const int lane = threadIdx.x & 63;
  for (int r = lane; r < n; r += 128) {
    double m[2][4], v[2][3];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = r + 64 * u;
      const bool ok = q < n;
#pragma unroll
      for (int k = 0; k < 3; ++k) v[u][k] = ok ? x[k * ldx + q] : 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) m[u][c] = (ok && c < nc) ? M[c * ldm + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if (SIGN > 0) s[c][k] += m[u][c] * v[u][k];
          else s[c][k] -= m[u][c] * v[u][k];
        }
  }
}

// y[q] (q = yoff + c, or ymap[q]) = sum_{r < split} M(r, c) xa[xoff + r] -
// sum_{split <= r < rows} M(r, c) xb[x2off + r - split] for the columns of an
// item (three right-hand sides): cpw = 1, one column per wave (columns
// col0 + w); cpw = 4, four per wave (col0 + 4 w .. + 3), for short columns,
// whose loads are then shared.  The lanes' sums are added across the wave at
// the end (fixed order); the storing lanes read their output index first.
__global__ __launch_bounds__(256) void k_nd_gemv(const NdItem* __restrict__ items,
                                                 const double* __restrict__ Mb,
                                                 const double* __restrict__ xa, long ldxa,
                                                 const double* __restrict__ xb, long ldxb,
                                                 double* __restrict__ y, long ldy,
                                                 const int32_t* __restrict__ ymap) {
  const NdItem it = items[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (it.cpw == 1) {
    const int c = it.col0 + w;
    if (c >= it.cols) return;
    // lanes 0, 16, 32 store the three sums (nd_wave_sum3)
    const bool store = (lane & 15) == 0 && (lane >> 4) < 3;
    const int o = store ? (ymap ? ymap[it.yoff + c] : it.yoff + c) : 0;
    const double* M = Mb + it.moff + (long)c * it.ldm;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    nd_dot<1>(M, xa + it.xoff, ldxa, it.split, s0, s1, s2);
    if (it.rows > it.split)
      nd_dot<-1>(M + it.split, xb + it.x2off, ldxb, it.rows - it.split, s0, s1, s2);
    int k;
    const double v = nd_wave_sum3(s0, s1, s2, k);
    if (store) y[k * ldy + o] = v;
    return;
  }
  const int c0 = it.col0 + 4 * w;
  if (c0 >= it.cols) return;
  const int nc = min(4, it.cols - c0);
  // the lane that stores sum idx (nd_wave_sum12): column idx / 3, component idx % 3
  const int sidx = ((lane & 32) ? 6 : 0) + ((lane & 16) ? 3 : 0) + ((lane & 8) ? 2 : 0) +
                   ((lane & 4) ? 1 : 0);
  const int sc = sidx / 3;
  const bool store = (lane & 3) == 0 && (lane & 12) != 12 && sc < nc;
  const int o = store ? (ymap ? ymap[it.yoff + c0 + sc] : it.yoff + c0 + sc) : 0;
  const double* M = Mb + it.moff + (long)c0 * it.ldm;
  double s[4][3];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int k = 0; k < 3; ++k) s[c][k] = 0.0;
  nd_dot4<1>(M, it.ldm, nc, xa + it.xoff, ldxa, it.split, s);
  if (it.rows > it.split)
    nd_dot4<-1>(M + it.split, it.ldm, nc, xb + it.x2off, ldxb, it.rows - it.split, s);
  double sf[12];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int k = 0; k < 3; ++k) sf[3 * c + k] = s[c][k];
  int idx;
  const double v = nd_wave_sum12(sf, idx);
  if (store) y[(idx - 3 * sc) * ldy + o] = v;
}
void nd_gemv(int nitems, const NdItem* items, const double* M, const double* xa, long ldxa,
             const double* xb, long ldxb, double* y, long ldy, const int32_t* ymap,
             hipStream_t st) {
  if (nitems > 0) k_nd_gemv<<<nitems, 256, 0, st>>>(items, M, xa, ldxa, xb, ldxb, y, ldy, ymap);
}

// dst (cols x rows, leading dimension ldd) = transpose of src (rows x cols,
// leading dimension lds), through a 32 x 32 LDS tile.
__global__ __launch_bounds__(256) void k_nd_transpose(const double* __restrict__ src, long lds,
                                                      int rows, int cols,
                                                      double* __restrict__ dst, long ldd) {
  __shared__ double T[32][33];
  const int tr = blockIdx.x * 32, tc = blockIdx.y * 32;
  const int x = threadIdx.x & 31, yy = threadIdx.x >> 5;
  for (int k = yy; k < 32; k += 8)
    if (tr + x < rows && tc + k < cols) T[k][x] = src[(long)(tr + x) + (long)(tc + k) * lds];
  __syncthreads();
  for (int k = yy; k < 32; k += 8)
    if (tc + x < cols && tr + k < rows) dst[(long)(tc + x) + (long)(tr + k) * ldd] = T[x][k];
}
void nd_transpose(const double* src, long lds, int rows, int cols, double* dst, long ldd,
                  hipStream_t st) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid((rows + 31) / 32, (cols + 31) / 32);
  k_nd_transpose<<<grid, 256, 0, st>>>(src, lds, rows, cols, dst, ldd);
}

// zb[v][e] = (key < n1) ? z[v][key] : d2[v][key - n1] for the cnt entries
// (e, key) of erec.
__global__ void k_nd_gather_zb(int cnt, const NdEntry* __restrict__ erec, int n1,
                               const double* __restrict__ z, long ldz,
                               const double* __restrict__ d2, long ldd2, double* __restrict__ zb,
                               long ldzb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const NdEntry en = erec[i];
  const int t = en.key;
#pragma unroll
  for (int v = 0; v < 3; ++v)
    zb[v * ldzb + en.e] = t < n1 ? z[v * ldz + t] : d2[v * ldd2 + (t - n1)];
}
void nd_gather_zb(int cnt, const NdEntry* erec, int n1, const double* z, long ldz,
                  const double* d2, long ldd2, double* zb, long ldzb, hipStream_t st) {
  if (cnt > 0)
    k_nd_gather_zb<<<(cnt + 255) / 256, 256, 0, st>>>(cnt, erec, n1, z, ldz, d2, ldd2, zb, ldzb);
}

}  // namespace pdk
