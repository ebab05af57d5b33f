// Warm-start MLP kernels: BF16-operand GEMMs with FP32 accumulation on the
// matrix cores (v_mfma_f32_16x16x32_bf16), fused epilogues, loss, bias
// gradients and Adam.  Activations and gradients are FP32 in memory and are
// rounded to BF16 (round to nearest even) when staged as GEMM operands;
// weights keep an FP32 master copy and a BF16 copy used by the products.
#include <algorithm>
#include "common.h"

namespace pdk {

typedef __bf16 bf16x8m_t __attribute__((ext_vector_type(8)));
constexpr int MT = 64;          // output tile
constexpr int MKC = 32;         // K chunk
constexpr int MLD = MKC + 8;    // LDS row (bf16), 16-byte aligned

__device__ inline float ld_as_float(const float* p) { return *p; }
__device__ inline float ld_as_float(const __bf16* p) { return (float)*p; }

// Stage a 64 x 32 operand chunk into LDS as S[row][k] (bf16).  KCONTIG: the
// element (row, k) is at G[row * ld + k]; otherwise at G[k * ld + row].
template <typename T, bool KCONTIG>
__device__ inline void stage(__bf16 (*S)[MLD], const T* __restrict__ G, long ld, int row0, int nrow,
                             int k0, int kend) {
  const int t = threadIdx.x;
  if (KCONTIG) {
    const int row = t >> 2, kq = (t & 3) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + kq + e;
      float v = 0.f;
      if (row0 + row < nrow && k < kend) v = ld_as_float(G + (long)(row0 + row) * ld + k);
      S[row][kq + e] = (__bf16)v;
    }
  } else {
    const int row = t & 63, kq = (t >> 6) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + kq + e;
      float v = 0.f;
      if (row0 + row < nrow && k < kend) v = ld_as_float(G + (long)k * ld + row0 + row);
      S[row][kq + e] = (__bf16)v;
    }
  }
}

// C[z][m][n] = sum_{k in split z} opA(m, k) opB(n, k)   (FP32 out, row-major, ldc = N)
template <typename TA, bool AK, typename TB, bool BK>
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const TA* __restrict__ A,
                                                   long lda, const TB* __restrict__ B, long ldb,
                                                   float* __restrict__ C, int ksplit) {
  __shared__ __bf16 As[MT][MLD];
  __shared__ __bf16 Bs[MT][MLD];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int m0 = blockIdx.y * MT, n0 = blockIdx.x * MT;
  const int z = blockIdx.z;
  const int kbeg = z * ksplit, kend = min(K, kbeg + ksplit);
  float4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += MKC) {
    __syncthreads();
    stage<TA, AK>(As, A, lda, m0, M, k0, kend);
    stage<TB, BK>(Bs, B, ldb, n0, N, k0, kend);
    __syncthreads();
    const int ko = 8 * (lane >> 4);
    const bf16x8m_t a0 = *(const bf16x8m_t*)&As[wr * 32 + (lane & 15)][ko];
    const bf16x8m_t a1 = *(const bf16x8m_t*)&As[wr * 32 + 16 + (lane & 15)][ko];
    const bf16x8m_t b0 = *(const bf16x8m_t*)&Bs[wc * 32 + (lane & 15)][ko];
    const bf16x8m_t b1 = *(const bf16x8m_t*)&Bs[wc * 32 + 16 + (lane & 15)][ko];
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b0, a0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b1, a0, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b0, a1, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b1, a1, acc[1][1], 0, 0, 0);
  }
  float* Cz = C + (long)z * M * N;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wr * 32 + mb * 16 + (lane & 15);
        const int n = n0 + wc * 32 + nb * 16 + 4 * (lane >> 4) + q;
        if (m < M && n < N) Cz[(long)m * N + n] = acc[mb][nb][q];
      }
}

// out[m][n] = sum_z part[z][m][n] (+ bias[n]) (relu)   (fixed summation order)
__global__ void k_split_reduce(int M, int N, int nsplit, const float* __restrict__ part,
                               const float* __restrict__ bias, int relu, float* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)M * N) return;
  float s = 0.f;
  for (int z = 0; z < nsplit; ++z) s += part[(long)z * M * N + e];
  if (bias) s += bias[e % N];
  if (relu) s = fmaxf(s, 0.f);
  out[e] = s;
}

void mlp_gemm(int M, int N, int K, const void* A, bool a_bf16, bool a_kcontig, long lda,
              const void* B, bool b_bf16, bool b_kcontig, long ldb, float* part, int nsplit,
              hipStream_t st) {
  const int ks = ((K + nsplit - 1) / nsplit + MKC - 1) / MKC * MKC;
  const int nz = (K + ks - 1) / ks;
  dim3 g((N + MT - 1) / MT, (M + MT - 1) / MT, nz);
#define LAUNCH(TA, AKC, TB, BKC) \
  k_gemm_bf16<TA, AKC, TB, BKC><<<g, 256, 0, st>>>(M, N, K, (const TA*)A, lda, (const TB*)B, ldb, part, ks)
  if (!a_bf16 && a_kcontig && b_bf16 && b_kcontig) LAUNCH(float, true, __bf16, true);
  else if (!a_bf16 && a_kcontig && b_bf16 && !b_kcontig) LAUNCH(float, true, __bf16, false);
  else if (!a_bf16 && !a_kcontig && !b_bf16 && !b_kcontig) LAUNCH(float, false, float, false);
  else LAUNCH(float, true, float, true);
#undef LAUNCH
}

int mlp_gemm_nsplit(int M, int N, int K, int nsplit) {
  const int ks = ((K + nsplit - 1) / nsplit + MKC - 1) / MKC * MKC;
  return (K + ks - 1) / ks;
}

void mlp_split_reduce(int M, int N, int nsplit, const float* part, const float* bias, int relu,
                      float* out, hipStream_t st) {
  const long n = (long)M * N;
  k_split_reduce<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(M, N, nsplit, part, bias, relu, out);
}

// dY = (Y - T) / (B n); partial loss sums per block (fixed order)
__global__ __launch_bounds__(256) void k_loss_grad(long total, float scale, const float* __restrict__ Y,
                                                   const float* __restrict__ T, float* __restrict__ dY,
                                                   double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const float d = Y[e] - T[e];
    dY[e] = d * scale;
    s += (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_parts(int n, const double* part, double scale, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s * scale;
  }
}

void mlp_loss_grad(long total, int n_out_times_b, const float* Y, const float* T, float* dY,
                   double* part, double* loss, hipStream_t st) {
  const int nb = 256;
  k_loss_grad<<<nb, 256, 0, st>>>(total, 1.f / (float)n_out_times_b, Y, T, dY, part);
  k_sum_parts<<<1, 1, 0, st>>>(nb, part, 0.5 / (double)n_out_times_b, loss);
}

// dZ = dA * (H > 0) in place
__global__ void k_relu_back(long n, const float* __restrict__ H, float* __restrict__ dA) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n && !(H[e] > 0.f)) dA[e] = 0.f;
}

void mlp_relu_back(long n, const float* H, float* dA, hipStream_t st) {
  k_relu_back<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, H, dA);
}

// gb[n] = sum_m dZ[m][n]
__global__ void k_colsum(int M, int N, const float* __restrict__ dZ, float* __restrict__ gb) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += dZ[(long)m * N + n];
  gb[n] = s;
}

void mlp_colsum(int M, int N, const float* dZ, float* gb, hipStream_t st) {
  k_colsum<<<(N + 255) / 256, 256, 0, st>>>(M, N, dZ, gb);
}

// Adam with bias correction on FP32 master weights; refreshes the BF16 copy.
__global__ void k_adam(long n, float* __restrict__ w, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, __bf16* __restrict__ wb,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float ge = g[e];
  const float me = b1 * m[e] + (1.f - b1) * ge;
  const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
  m[e] = me;
  v[e] = ve;
  const float we = w[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
  w[e] = we;
  if (wb) wb[e] = (__bf16)we;
}

void mlp_adam(long n, float* w, const float* g, float* m, float* v, __bf16* wb, float lr, int step,
              hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  k_adam<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, w, g, m, v, wb, lr, b1, b2, 1e-8f, c1, c2);
}

// dst[b][k] = src[rows[b]][k] * (k < n_scaled ? scale : 1), rows of n_cols floats.
__global__ void k_gather_rows_scaled(int n_cols, const float* __restrict__ src,
                                     const int32_t* __restrict__ rows, int n_scaled, float scale,
                                     float* __restrict__ dst) {
  const int b = blockIdx.y;
  const long r = rows[b];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_cols; k += gridDim.x * blockDim.x) {
    const float v = src[r * n_cols + k];
    dst[(long)b * n_cols + k] = k < n_scaled ? v * scale : v;
  }
}

void mlp_gather_rows_scaled(int B, int n_cols, const float* src, const int32_t* rows, int n_scaled,
                            float scale, float* dst, hipStream_t st) {
  const int gx = std::min((n_cols + 255) / 256, 64);
  k_gather_rows_scaled<<<dim3(gx, B), 256, 0, st>>>(n_cols, src, rows, n_scaled, scale, dst);
}

// out = sum |a| / n over n floats, one workgroup, fixed order.
__global__ __launch_bounds__(1024) void k_abs_mean(long n, const float* __restrict__ a,
                                                   double* __restrict__ out) {
  __shared__ double red[1024];
  double s = 0.0;
  for (long e = threadIdx.x; e < n; e += 1024) s += fabs((double)a[e]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = n > 0 ? red[0] / (double)n : 0.0;
}

void mlp_abs_mean(long n, const float* a, double* out, hipStream_t st) {
  k_abs_mean<<<1, 1024, 0, st>>>(n, a, out);
}

__global__ void k_to_bf16(long n, const float* __restrict__ w, __bf16* __restrict__ wb) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) wb[e] = (__bf16)w[e];
}

void mlp_to_bf16(long n, const float* w, __bf16* wb, hipStream_t st) {
  k_to_bf16<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, w, wb);
}

}  // namespace pdk
