// Condensation sweeps through the interior factor (one-way dissection in
// breadth-first levels, Z_k = S_k^-1 dense and symmetric, B_k the sparse
// coupling of level k to level k+1 or to the region).  The level chain is
// sequential; each level is a dense product with Z_k, the assembly of its
// result, and a sparse coupling update (csr_spmv3).
//
// Dense product y = Z_k x with only the lower triangle read: Z_k is stored in
// full (column-major), but the kernels walk the lower 64 x 64 tiles (I, J),
// J <= I, once each, computing
//   row part  Z_IJ x_J      (I > J), and
//   col part  Z_IJ^T x_I,
// each into the tile's slot of a workspace.  y_I is then the sum of the row
// parts of tiles (I, J < I) and the col parts of tiles (I' >= I, I), taken
// in that fixed order by the assembly kernel, so results do not depend on
// scheduling.  HBM traffic is half the full matrix.
#include <algorithm>
#include "common.h"

namespace pdk {

namespace {

constexpr int TS = 64;                 // tile size of the level products
constexpr int SLOT = 3 * TS;           // doubles per part slot: [rhs][64]

// One workgroup per lower tile (I, J), wave w owning columns 16 w .. 16 w + 15:
// the wave loads its 64 x 16 block into registers (lane = row, sixteen
// coalesced column loads in flight), adds its share of the row part Z_IJ x_J
// in-lane, and forms the col part Z_IJ^T x_I of its sixteen columns through a
// wave-private LDS transpose, 32 rows at a time (lane = (column, row group),
// then two cross-lane additions).  The four row-part shares are added in wave
// order.  Row parts go to slot t(I, J) of Prow (off-diagonal tiles), col parts
// to slot t(I, J) of Pcol.  26 KB of LDS per workgroup, so that the products
// still find room next to a running factorization.
__global__ __launch_bounds__(256) void k_sweep_symv(const double* __restrict__ Z, long ldz, int w,
                                                    int nb, const double* __restrict__ x, long ldx,
                                                    double* __restrict__ Prow,
                                                    double* __restrict__ Pcol) {
  __shared__ double Ts[4][TS / 2][17];     // per wave: 32 rows x 16 columns (+1 pad)
  __shared__ double xs[2][3][TS];          // x_J, x_I
  __shared__ double rp[4][3][TS];          // per-wave shares of the row part
  const int t = threadIdx.x, lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int tt = blockIdx.x;
  int I = (int)((sqrt(8.0 * (double)tt + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= tt) ++I;
  while (I * (I + 1) / 2 > tt) --I;
  I = __builtin_amdgcn_readfirstlane(I);
  const int J = tt - I * (I + 1) / 2;
  const int i0 = I * TS, j0 = J * TS;
  const int nr = min(TS, w - i0), nc = min(TS, w - j0);
  const int c0 = 16 * wv;                  // first column of this wave
  const int ncw = max(0, min(16, nc - c0));
  // buffer loads: one 32-bit lane offset (the row) for all sixteen columns, the
  // column offset in a scalar register; lanes past the last row get an offset
  // beyond the buffer's range and read zero
  // (base and size are wave-uniform; readfirstlane keeps the descriptor scalar)
  const unsigned long long zb = reinterpret_cast<unsigned long long>(
      Z + (long)(j0 + (ncw > 0 ? c0 : 0)) * ldz);
  const unsigned zlo = __builtin_amdgcn_readfirstlane((unsigned)zb);
  const unsigned zhi = __builtin_amdgcn_readfirstlane((unsigned)(zb >> 32));
  const int zbytes = __builtin_amdgcn_readfirstlane((int)(max(ncw, 1) * ldz * (long)sizeof(double)));
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      reinterpret_cast<void*>(((unsigned long long)zhi << 32) | zlo), 0, zbytes, 0x00020000);
  const int voff = lane < nr ? (i0 + lane) * (int)sizeof(double) : 0x7ffffff0;
  // x_J and x_I: two loads per thread (t and t + 256 of the 384 entries),
  // issued before the tile so that waiting for them does not wait for it
  double xv[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int e = t + 256 * k;
    const int h = e >= 3 * TS ? 1 : 0, v = (e / TS) % 3, r = e % TS;
    const int base = h ? i0 : j0, lim = h ? nr : nc;
    const bool ok = e < 2 * 3 * TS && r < lim;
    xv[k] = x[ok ? (long)v * ldx + base + r : 0] * (ok ? 1.0 : 0.0);
  }
  // columns past the last one (ragged tile) re-read the last column, so every
  // address stays inside the matrix: they meet zeros of x_J in the row part,
  // and their col parts are never read
  const int clast = __builtin_amdgcn_readfirstlane(max(ncw, 1) - 1);
  double z[16];
#pragma unroll
  for (int c = 0; c < 16; ++c)
    z[c] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                          rs, voff, min(c, clast) * (int)(ldz * sizeof(double)), 0));
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int e = t + 256 * k;
    if (e < 2 * 3 * TS) (&xs[0][0][0])[e] = xv[k];
  }
  __syncthreads();
  // this wave's share of the row part, lane = row
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    s0 += z[c] * xs[0][0][c0 + c];
    s1 += z[c] * xs[0][1][c0 + c];
    s2 += z[c] * xs[0][2][c0 + c];
    // four columns at a time: keeps the scheduler from loading all 48
    // operands of the row part into registers at once
    if ((c & 3) == 3) __builtin_amdgcn_sched_barrier(0);
  }
  rp[wv][0][lane] = s0;
  rp[wv][1][lane] = s1;
  rp[wv][2][lane] = s2;
  // col part of the sixteen columns, 32 rows at a time: lane = (cc = lane & 15, rg = lane >> 4)
  const int cc = lane & 15, rg = lane >> 4;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    // the transpose goes through wave-private LDS: the wave barriers keep the
    // compiler from moving a lane's loads across other lanes' stores
    __builtin_amdgcn_wave_barrier();
    if ((lane >> 5) == h) {
#pragma unroll
      for (int c = 0; c < 16; ++c) Ts[wv][lane & 31][c] = z[c];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = 8 * rg + q;
      const double zz = Ts[wv][r][cc];
      a0 += zz * xs[1][0][32 * h + r];
      a1 += zz * xs[1][1][32 * h + r];
      a2 += zz * xs[1][2][32 * h + r];
      if ((q & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  }
  a0 += __shfl_xor(a0, 16, 64);
  a1 += __shfl_xor(a1, 16, 64);
  a2 += __shfl_xor(a2, 16, 64);
  a0 += __shfl_xor(a0, 32, 64);
  a1 += __shfl_xor(a1, 32, 64);
  a2 += __shfl_xor(a2, 32, 64);
  double* pc = Pcol + (long)tt * SLOT;
  if (lane < 16) {
    pc[c0 + lane] = a0;
    pc[TS + c0 + lane] = a1;
    pc[2 * TS + c0 + lane] = a2;
  }
  if (I > J) {
    __syncthreads();
    if (t < 3 * TS) {
      const int v = t >> 6, r = t & 63;
      Prow[(long)tt * SLOT + v * TS + r] = ((rp[0][v][r] + rp[1][v][r]) + rp[2][v][r]) + rp[3][v][r];
    }
  }
}

// out[v][g] = s or base[v][g] - s, s = (Z x)[v][g].  Output row g of block I
// has nb terms k = 0 .. nb - 1: the row part of tile (I, k) for k < I and the
// col part of tile (k, I) for k >= I.  Four lanes share an output, lane q
// adding terms k = q, q + 4, ...; the four partial sums are combined as
// (s0 + s1) + (s2 + s3), so the result does not depend on scheduling.
__global__ void k_sweep_assemble(int w, int nb, const double* __restrict__ Prow,
                                 const double* __restrict__ Pcol, const double* __restrict__ base,
                                 long ldb, double* __restrict__ out, long ldo) {
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = gt & 3, o = gt >> 2;
  const int v = o / w, g = o - v * w;
  const bool live = v < 3;
  double s = 0.0;
  if (live) {
    const int I = g / TS, r = g - I * TS;
    const double* row = Prow + (long)(I * (I + 1) / 2) * SLOT + v * TS + r;
    const double* col = Pcol + v * TS + r;
#pragma unroll 4
    for (int k = q; k < nb; k += 4)
      s += (k < I) ? row[(long)k * SLOT] : col[(long)(k * (k + 1) / 2 + I) * SLOT];
  }
  const double s1 = __shfl_xor(s, 1, 64);
  const double pair = (q & 1) ? s1 + s : s + s1;           // (s0 + s1) or (s2 + s3)
  const double other = __shfl_xor(pair, 2, 64);
  const double tot = (q & 2) ? other + pair : pair + other;
  if (live && q == 0) out[(long)v * ldo + g] = base ? base[(long)v * ldb + g] - tot : tot;
}

}  // namespace

int64_t sweep_workspace(int64_t maxw) {
  const int64_t nb = (maxw + TS - 1) / TS;
  return std::max<int64_t>(1, nb * (nb + 1) / 2) * 2 * SLOT;
}

void sweep_symv(const double* Z, long ldz, int w, const double* x, long ldx, double* P,
                hipStream_t st) {
  if (w <= 0) return;
  const int nb = (w + TS - 1) / TS, ntiles = nb * (nb + 1) / 2;
  k_sweep_symv<<<ntiles, 256, 0, st>>>(Z, ldz, w, nb, x, ldx, P, P + (long)ntiles * SLOT);
}

void sweep_assemble(int w, const double* P, const double* base, long ldb, double* out, long ldo,
                    hipStream_t st) {
  if (w <= 0) return;
  const int nb = (w + TS - 1) / TS, ntiles = nb * (nb + 1) / 2;
  k_sweep_assemble<<<(12 * w + 255) / 256, 256, 0, st>>>(w, nb, P, P + (long)ntiles * SLOT, base,
                                                         ldb, out, ldo);
}

}  // namespace pdk
