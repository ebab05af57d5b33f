// Per-tet FEM kernels (shape operators, element stiffness, local step and
// forces), gather-based assembly, sparse helpers for the interior level
// elimination, collision detection and penalty terms.  All reductions are
// gathers in a fixed order (no floating-point atomics), so results are
// bitwise reproducible run to run.
#include "common.h"

namespace pdk {

static inline unsigned grid1(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Workgroup b of a launch is dispatched to XCD b % 8 (round robin over the
// eight accelerator dies, each with its own L2).  For kernels whose
// neighbouring blocks share data (node positions of adjacent tets, element
// forces of adjacent nodes), map the dispatch index to a logical block so
// that each XCD works through one contiguous eighth of the blocks and the
// shared lines are fetched into one L2 instead of several.  A bijection on
// [0, nb).
__device__ inline int64_t xcd_contiguous_block(int64_t b, int64_t nb) {
  const int64_t x = b & 7, q = b >> 3, base = nb >> 3, rem = nb & 7;
  return x * base + (x < rem ? x : rem) + q;
}

// ---------------------------------------------------------------------------
// Geometry: D_m = [X1-X0, X2-X0, X3-X0], Bm = D_m^-1 (row-major, SoA [9][T]),
// vol = det(D_m) / 6.
__global__ void k_tet_geometry(const double* __restrict__ rest, int64_t n,
                               const int32_t* __restrict__ tets, int64_t T,
                               double* __restrict__ Bm, double* __restrict__ vol) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T) return;
  double X[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int32_t v = tets[a * T + e];
#pragma unroll
    for (int i = 0; i < 3; ++i) X[a][i] = rest[i * n + v];
  }
  double D[3][3];   // D[i][c] = (X_{c+1} - X_0)_i
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) D[i][c] = X[c + 1][i] - X[0][i];
  const double c00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  const double c01 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
  const double c02 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
  const double det = D[0][0] * c00 + D[0][1] * c01 + D[0][2] * c02;
  const double id = 1.0 / det;
  double I[3][3];
  I[0][0] = c00 * id;
  I[1][0] = c01 * id;
  I[2][0] = c02 * id;
  I[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) * id;
  I[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * id;
  I[2][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) * id;
  I[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) * id;
  I[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * id;
  I[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * id;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Bm[(r * 3 + c) * T + e] = I[r][c];
  vol[e] = det / 6.0;
}

void tet_geometry(const double* rest, int64_t n, const int32_t* tets, int64_t T, double* Bm,
                  double* vol, hipStream_t st) {
  if (T > 0) k_tet_geometry<<<grid1(T), 256, 0, st>>>(rest, n, tets, T, Bm, vol);
}

// Ke[a*4+b][e] = 2 mu vol_e (B_e B_e^T)_ab with B_e row 0 = -(sum of rows of D_m^-1),
// rows 1..3 = rows of D_m^-1.  Computed for a <= b and mirrored (exactly symmetric).
__global__ void k_element_stiffness(const double* __restrict__ Bm, const double* __restrict__ vol,
                                    int64_t T, double mu, double* __restrict__ Ke) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T) return;
  double B[4][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) B[r + 1][c] = Bm[(r * 3 + c) * T + e];
#pragma unroll
  for (int c = 0; c < 3; ++c) B[0][c] = -(B[1][c] + B[2][c] + B[3][c]);
  const double s = 2.0 * mu * vol[e];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
      const double v = s * (B[a][0] * B[b][0] + B[a][1] * B[b][1] + B[a][2] * B[b][2]);
      Ke[(a * 4 + b) * T + e] = v;
      Ke[(b * 4 + a) * T + e] = v;
    }
}

void element_stiffness(const double* Bm, const double* vol, int64_t T, double mu, double* Ke,
                       hipStream_t st) {
  if (T > 0) k_element_stiffness<<<grid1(T), 256, 0, st>>>(Bm, vol, T, mu, Ke);
}

// dst[dst_off[i]] = sum_{e in [ptr[i], ptr[i+1])} vals[src[e]]  (fixed order)
__global__ void k_gather_assign(int64_t count, const int64_t* __restrict__ ptr,
                                const int64_t* __restrict__ src, const double* __restrict__ vals,
                                const int64_t* __restrict__ dst_off, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double s = 0.0;
  for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) s += vals[src[e]];
  dst[dst_off[i]] = s;
}

void gather_assign(int64_t count, const int64_t* ptr, const int64_t* src, const double* vals,
                   const int64_t* dst_off, double* dst, hipStream_t st) {
  if (count > 0) k_gather_assign<<<grid1(count), 256, 0, st>>>(count, ptr, src, vals, dst_off, dst);
}

// ---------------------------------------------------------------------------
// Rotation of the polar decomposition, R = argmin_{R in SO(3)} ||F - R||_F.
// Eigen-decomposition of F^T F by cyclic Jacobi rotations gives V; QR of F V
// by Givens rotations gives U with F V = U diag(s1, s2, s3) (s3 < 0 when F is
// inverted); R = U V^T.  Singular values are sorted in decreasing order, so the
// reflection of an inverted element is put on the smallest one.
template <typename T>
__device__ inline void jacobi_rot(T A[3][3], T V[3][3], int p, int q) {
  const T apq = A[p][q];
  if (apq == T(0)) return;
  const T theta = (A[q][q] - A[p][p]) / (T(2) * apq);
  T t;
  const T at = fabs(theta);
  if (at > T(1e18)) t = T(0.5) / theta;
  else t = (theta >= T(0) ? T(1) : T(-1)) / (at + sqrt(theta * theta + T(1)));
  const T c = T(1) / sqrt(t * t + T(1));
  const T s = t * c;
  const int r = 3 - p - q;
  const T arp = A[r][p], arq = A[r][q];
  A[p][p] -= t * apq;
  A[q][q] += t * apq;
  A[p][q] = A[q][p] = T(0);
  A[r][p] = A[p][r] = c * arp - s * arq;
  A[r][q] = A[q][r] = s * arp + c * arq;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T vp = V[k][p], vq = V[k][q];
    V[k][p] = c * vp - s * vq;
    V[k][q] = s * vp + c * vq;
  }
}

template <typename T>
__device__ inline void givens_rows(T B[3][3], T U[3][3], int p, int q) {
  // zero B[q][p] using rows p and q: B <- G B, U <- U G^T
  const T a = B[p][p], b = B[q][p];
  const T r = sqrt(a * a + b * b);
  if (r == T(0)) return;
  const T c = a / r, s = b / r;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T bp = B[p][k], bq = B[q][k];
    B[p][k] = c * bp + s * bq;
    B[q][k] = -s * bp + c * bq;
    const T up = U[k][p], uq = U[k][q];
    U[k][p] = c * up + s * uq;
    U[k][q] = -s * up + c * uq;
  }
}

// Q: the strain-limited projection of the biphasic material
// (Sec. 5.3): F V = U diag(b) with b_1, b_2 >= 0 and b_3 of either sign, so
// the singular values are |b_i| with left vectors sign(b_i) U e_i, and the
// closest matrix with singular values in [smin, smax] is
// Q = U diag(sign(b_i) clamp(|b_i|)) V^T (computed always: a pointer chosen
// at run time would keep the arrays in private memory; callers that do not
// need Q ignore it).
template <typename T>
__device__ void polar_rotation(const T F[3][3], T R[3][3], T Q[3][3], T smin, T smax) {
  T A[3][3], V[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      A[i][j] = F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j];
      V[i][j] = (i == j) ? T(1) : T(0);
    }
  const T eps = sizeof(T) == 8 ? T(1e-34) : T(1e-16);   // relative off-diagonal^2 target
  for (int sweep = 0; sweep < 12; ++sweep) {
    const T off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const T dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (!(off > eps * dia)) break;
    jacobi_rot(A, V, 0, 1);
    jacobi_rot(A, V, 0, 2);
    jacobi_rot(A, V, 1, 2);
  }
  // sort eigenvalues (squared singular values) in decreasing order
  T ev[3] = {A[0][0], A[1][1], A[2][2]};
#pragma unroll
  for (int pass = 0; pass < 2; ++pass)
#pragma unroll
    for (int i = 0; i < 2; ++i)
      if (ev[i] < ev[i + 1]) {
        const T tmp = ev[i]; ev[i] = ev[i + 1]; ev[i + 1] = tmp;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T tv = V[k][i]; V[k][i] = V[k][i + 1]; V[k][i + 1] = tv;
        }
      }
  const T detV = V[0][0] * (V[1][1] * V[2][2] - V[1][2] * V[2][1]) -
                 V[0][1] * (V[1][0] * V[2][2] - V[1][2] * V[2][0]) +
                 V[0][2] * (V[1][0] * V[2][1] - V[1][1] * V[2][0]);
  if (detV < T(0)) {
#pragma unroll
    for (int k = 0; k < 3; ++k) V[k][2] = -V[k][2];
  }
  T B[3][3], U[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      B[i][j] = F[i][0] * V[0][j] + F[i][1] * V[1][j] + F[i][2] * V[2][j];
      U[i][j] = (i == j) ? T(1) : T(0);
    }
  givens_rows(B, U, 0, 1);
  givens_rows(B, U, 0, 2);
  givens_rows(B, U, 1, 2);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) R[i][j] = U[i][0] * V[j][0] + U[i][1] * V[j][1] + U[i][2] * V[j][2];
  {
    T d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T b = B[k][k];
      const T a = fabs(b);
      const T c = a < smin ? smin : (a > smax ? smax : a);
      d[k] = b < T(0) ? -c : c;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Q[i][j] = U[i][0] * d[0] * V[j][0] + U[i][1] * d[1] * V[j][1] + U[i][2] * d[2] * V[j][2];
  }
}

// Local step and elemental forces for a list of tets:
//   F = D_s D_m^-1, R = polar(F), P = 2 mu (F - R),
//   f_a = -vol P (D_m^-1)^T e_(a-1) for a = 1..3, f_0 = -(f_1 + f_2 + f_3).
// tets [4][ldt] index positions in x ([3][ldx]); fe [12][T] (vertex-major);
// R [9][T] (row-major 3x3 per tet) in FP64 or FP32, or NULL.
//   biphasic material (mu_p > 0, Sec. 5.3): Q = strain-limited projection of F,
//   P += 2 mu_p (F - Q).
__global__ void k_local_step(int64_t T, const int32_t* __restrict__ tets, int64_t ldt,
                             const double* __restrict__ Bm, const double* __restrict__ vol,
                             int64_t ldb, const double* __restrict__ x, int64_t ldx, double mu,
                             double mu_p, double smin, double smax,
                             double* __restrict__ fe, void* Rout, int rot_fp32) {
  const int64_t e = xcd_contiguous_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (e >= T) return;
  double X[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int32_t v = tets[a * ldt + e];
#pragma unroll
    for (int i = 0; i < 3; ++i) X[a][i] = x[i * ldx + v];
  }
  double Dinv[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Dinv[r][c] = Bm[(r * 3 + c) * ldb + e];
  double F[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      F[i][j] = (X[1][i] - X[0][i]) * Dinv[0][j] + (X[2][i] - X[0][i]) * Dinv[1][j] +
                (X[3][i] - X[0][i]) * Dinv[2][j];
  double R[3][3], Q[3][3];
  const bool biphasic = mu_p > 0.0;
  if (rot_fp32) {
    float Ff[3][3], Rf[3][3], Qf[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Ff[i][j] = (float)F[i][j];
    polar_rotation<float>(Ff, Rf, Qf, (float)smin, (float)smax);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        R[i][j] = (double)Rf[i][j];
        Q[i][j] = biphasic ? (double)Qf[i][j] : F[i][j];
      }
  } else {
    polar_rotation<double>(F, R, Q, smin, smax);
    if (!biphasic) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Q[i][j] = F[i][j];
    }
  }
  const double s = -2.0 * mu * vol[e];
  const double rp = biphasic ? mu_p / mu : 0.0;
  double f[4][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double p0 = (F[i][0] - R[i][0]) + rp * (F[i][0] - Q[i][0]);
    const double p1 = (F[i][1] - R[i][1]) + rp * (F[i][1] - Q[i][1]);
    const double p2 = (F[i][2] - R[i][2]) + rp * (F[i][2] - Q[i][2]);
#pragma unroll
    for (int a = 1; a < 4; ++a)
      f[a][i] = s * (p0 * Dinv[a - 1][0] + p1 * Dinv[a - 1][1] + p2 * Dinv[a - 1][2]);
    f[0][i] = -(f[1][i] + f[2][i] + f[3][i]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) fe[(a * 3 + i) * T + e] = f[a][i];
  if (Rout) {
    if (rot_fp32) {
      float* Rf = (float*)Rout;
#pragma unroll
      for (int k = 0; k < 9; ++k) Rf[k * T + e] = (float)R[k / 3][k % 3];
    } else {
      double* Rd = (double*)Rout;
#pragma unroll
      for (int k = 0; k < 9; ++k) Rd[k * T + e] = R[k / 3][k % 3];
    }
  }
}

void local_step(int64_t T, const int32_t* tets, int64_t ldt, const double* Bm, const double* vol,
                int64_t ldb, const double* x, int64_t ldx, double mu, double mu_p, double smin,
                double smax, double* fe, void* R, int rot_fp32, hipStream_t st) {
  if (T > 0)
    k_local_step<<<grid1(T, 128), 128, 0, st>>>(T, tets, ldt, Bm, vol, ldb, x, ldx, mu, mu_p,
                                                smin, smax, fe, R, rot_fp32);
}

// f[i][node_of_row[r]] (+)= sum over incidences e in [ptr[r], ptr[r+1]) of
// fe[(3*(ent%4) + i)][ent/4]  (fixed order).
__global__ void k_node_gather3(int64_t count, const int32_t* __restrict__ ptr,
                               const int32_t* __restrict__ ent, const double* __restrict__ fe,
                               int64_t ldfe, const int32_t* __restrict__ node_of_row,
                               double* __restrict__ f, int64_t ldf, int accumulate) {
  const int64_t r = xcd_contiguous_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (r >= count) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int32_t e = ptr[r]; e < ptr[r + 1]; ++e) {
    const int32_t en = ent[e];
    const int64_t tet = en >> 2, a = en & 3;
    s0 += fe[(a * 3 + 0) * ldfe + tet];
    s1 += fe[(a * 3 + 1) * ldfe + tet];
    s2 += fe[(a * 3 + 2) * ldfe + tet];
  }
  const int64_t node = node_of_row ? node_of_row[r] : r;
  if (accumulate) {
    f[node] += s0;
    f[ldf + node] += s1;
    f[2 * ldf + node] += s2;
  } else {
    f[node] = s0;
    f[ldf + node] = s1;
    f[2 * ldf + node] = s2;
  }
}

void node_gather3(int64_t count, const int32_t* ptr, const int32_t* ent, const double* fe,
                  int64_t ldfe, const int32_t* node_of_row, double* f, int64_t ldf, int accumulate,
                  hipStream_t st) {
  if (count > 0)
    k_node_gather3<<<grid1(count), 256, 0, st>>>(count, ptr, ent, fe, ldfe, node_of_row, f, ldf,
                                                 accumulate);
}

__global__ void k_gather_rows3(int64_t count, const int32_t* __restrict__ ids,
                               const double* __restrict__ src, int64_t lds,
                               double* __restrict__ dst, int64_t ldd) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= count) return;
  const int64_t s = ids[r];
  dst[r] = src[s];
  dst[ldd + r] = src[lds + s];
  dst[2 * ldd + r] = src[2 * lds + s];
}

void gather_rows3(int64_t count, const int32_t* ids, const double* src, int64_t lds, double* dst,
                  int64_t ldd, hipStream_t st) {
  if (count > 0) k_gather_rows3<<<grid1(count), 256, 0, st>>>(count, ids, src, lds, dst, ldd);
}

__global__ void k_scatter_add_rows3(int64_t count, const int32_t* __restrict__ ids,
                                    const double* __restrict__ src, int64_t lds,
                                    double* __restrict__ dst, int64_t ldd) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= count) return;
  const int64_t d = ids[r];
  dst[d] += src[r];
  dst[ldd + d] += src[lds + r];
  dst[2 * ldd + d] += src[2 * lds + r];
}

void scatter_add_rows3(int64_t count, const int32_t* ids, const double* src, int64_t lds,
                       double* dst, int64_t ldd, hipStream_t st) {
  if (count > 0) k_scatter_add_rows3<<<grid1(count), 256, 0, st>>>(count, ids, src, lds, dst, ldd);
}

// y[v][r] = base[v][r] + alpha * sum_j val * v[v][col]   (base may be NULL = 0, may alias y)
__global__ void k_csr_spmv3(int64_t rows, const int32_t* __restrict__ ptr,
                            const int32_t* __restrict__ col, const double* __restrict__ val,
                            const double* __restrict__ v, int64_t ldv, double alpha, double* y,
                            int64_t ldy, const double* base, int64_t ldbase) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int32_t e = ptr[r]; e < ptr[r + 1]; ++e) {
    const double a = val[e];
    const int64_t c = col[e];
    s0 += a * v[c];
    s1 += a * v[ldv + c];
    s2 += a * v[2 * ldv + c];
  }
  double b0 = 0.0, b1 = 0.0, b2 = 0.0;
  if (base) {
    b0 = base[r];
    b1 = base[ldbase + r];
    b2 = base[2 * ldbase + r];
  }
  y[r] = b0 + alpha * s0;
  y[ldy + r] = b1 + alpha * s1;
  y[2 * ldy + r] = b2 + alpha * s2;
}

void csr_spmv3(int64_t rows, const int32_t* ptr, const int32_t* col, const double* val,
               const double* v, int64_t ldv, double alpha, double* y, int64_t ldy,
               const double* base, int64_t ldbase, hipStream_t st) {
  if (rows > 0)
    k_csr_spmv3<<<grid1(rows), 256, 0, st>>>(rows, ptr, col, val, v, ldv, alpha, y, ldy, base,
                                             ldbase);
}

// U[i + jr*w] = sum_{e in row rows[jr] of B} val[e] * Z[i + col[e]*w]   (U = Z B^T on the rows)
__global__ void k_dense_times_sparse_t(const double* __restrict__ Z, int ldz, int w, int nr,
                                       const int32_t* __restrict__ rows,
                                       const int32_t* __restrict__ ptr,
                                       const int32_t* __restrict__ col,
                                       const double* __restrict__ val, double* __restrict__ U) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int jr = blockIdx.y;
  if (i >= w || jr >= nr) return;
  const int rr = rows[jr];
  double s = 0.0;
  for (int32_t e = ptr[rr]; e < ptr[rr + 1]; ++e) s += val[e] * Z[(int64_t)i + (int64_t)col[e] * ldz];
  U[(int64_t)i + (int64_t)jr * w] = s;
}

void dense_times_sparse_t(const double* Z, int ldz, int w, int nr, const int32_t* rows,
                          const int32_t* ptr, const int32_t* col, const double* val, double* U,
                          hipStream_t st) {
  if (w > 0 && nr > 0) {
    dim3 g(grid1(w), nr);
    k_dense_times_sparse_t<<<g, 256, 0, st>>>(Z, ldz, w, nr, rows, ptr, col, val, U);
  }
}

// Next[rows[ir] + rows[jr]*ldn] -= sum_{e in row rows[ir] of B} val[e] * U[col[e] + jr*ldu]
__global__ void k_sub_sparse_times_dense(double* __restrict__ Next, int ldn, int nr,
                                         const int32_t* __restrict__ rows,
                                         const int32_t* __restrict__ ptr,
                                         const int32_t* __restrict__ col,
                                         const double* __restrict__ val,
                                         const double* __restrict__ U, int ldu) {
  const int ir = blockIdx.x * blockDim.x + threadIdx.x;
  const int jr = blockIdx.y;
  if (ir >= nr || jr >= nr) return;
  const int ri = rows[ir];
  double s = 0.0;
  for (int32_t e = ptr[ri]; e < ptr[ri + 1]; ++e) s += val[e] * U[(int64_t)col[e] + (int64_t)jr * ldu];
  Next[(int64_t)ri + (int64_t)rows[jr] * ldn] -= s;
}

void sub_sparse_times_dense(double* Next, int ldn, int nr, const int32_t* rows, const int32_t* ptr,
                            const int32_t* col, const double* val, const double* U, int ldu,
                            hipStream_t st) {
  if (nr > 0) {
    dim3 g(grid1(nr), nr);
    k_sub_sparse_times_dense<<<g, 256, 0, st>>>(Next, ldn, nr, rows, ptr, col, val, U, ldu);
  }
}

// ---------------------------------------------------------------------------
// Sphere detection for conforming proxies.  The in/out decision and the
// projection are computed with separately rounded operations (no fused
// multiply-add), in the order: dist = sqrt((d0*d0 + d1*d1) + d2*d2).
__global__ void k_detect_spheres(int n_prox, const int32_t* __restrict__ prox, int n_sph,
                                 const double* __restrict__ sph, double k,
                                 const double* __restrict__ x2, int m, int32_t* __restrict__ idx,
                                 double* __restrict__ w, double* __restrict__ c,
                                 double* __restrict__ t) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_prox) return;
  const int a = prox[j];
  if (a < 0 || a >= m) {          // not a region node: emit an inactive slot
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      idx[j * 8 + s] = -1;
      w[j * 8 + s] = 0.0;
    }
    c[j] = 0.0;
    t[j] = t[n_prox + j] = t[2 * n_prox + j] = 0.0;
    return;
  }
  const double p0 = x2[a], p1 = x2[m + a], p2 = x2[2 * m + a];
  double best = -INFINITY;
  int hit = -1;
  double t0 = p0, t1 = p1, t2 = p2;
  for (int s = 0; s < n_sph; ++s) {
    const double cx = sph[s], cy = sph[n_sph + s], cz = sph[2 * n_sph + s], r = sph[3 * n_sph + s];
    const double d0 = __dsub_rn(p0, cx), d1 = __dsub_rn(p1, cy), d2 = __dsub_rn(p2, cz);
    const double dist =
        __dsqrt_rn(__dadd_rn(__dadd_rn(__dmul_rn(d0, d0), __dmul_rn(d1, d1)), __dmul_rn(d2, d2)));
    const double depth = __dsub_rn(r, dist);
    if (dist < r && depth > best) {
      best = depth;
      hit = s;
      double u0 = 0.0, u1 = 0.0, u2 = 1.0;
      if (dist > 0.0) {
        u0 = __ddiv_rn(d0, dist);
        u1 = __ddiv_rn(d1, dist);
        u2 = __ddiv_rn(d2, dist);
      }
      t0 = __dadd_rn(cx, __dmul_rn(r, u0));
      t1 = __dadd_rn(cy, __dmul_rn(r, u1));
      t2 = __dadd_rn(cz, __dmul_rn(r, u2));
    }
  }
  idx[j * 8] = a;
  w[j * 8] = 1.0;
#pragma unroll
  for (int s = 1; s < 8; ++s) {
    idx[j * 8 + s] = -1;
    w[j * 8 + s] = 0.0;
  }
  c[j] = (hit >= 0) ? k : 0.0;
  t[j] = t0;
  t[n_prox + j] = t1;
  t[2 * n_prox + j] = t2;
}

void detect_spheres(int n_prox, const int32_t* prox, int n_sph, const double* sph, double k,
                    const double* x2, int m, int32_t* idx, double* w, double* c, double* t,
                    hipStream_t st) {
  if (n_prox > 0)
    k_detect_spheres<<<grid1(n_prox), 256, 0, st>>>(n_prox, prox, n_sph, sph, k, x2, m, idx, w,
                                                     c, t);
}

// Active penalties and their incidence on the region rows, one workgroup
// (block-wide prefix sums; deterministic):
//  * act[0..*cnt) = indices j < n_pen with c[j] != 0, increasing;
//  * ent[rowptr[a] .. rowptr[a + 1]) = keys 8 q + s of the slots s of the
//    active penalties act[q] that name region row a, increasing.
// Counts and cursors live in cursor[] (global; read back with L1-bypassing
// atomic loads after the atomic updates); the fill order of a row is then
// fixed by sorting its keys.
__device__ inline int block_exclusive_scan(int v, int* wsum, int* total) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(x, o, 64);
    if (lane >= o) x += u;
  }
  __syncthreads();                         // wsum may still be read by a previous call
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int off = 0, tot = 0;
  for (int q = 0; q < 16; ++q) {
    if (q < w) off += wsum[q];
    tot += wsum[q];
  }
  *total = tot;
  return off + x - v;
}

__global__ __launch_bounds__(1024) void k_penalty_prepare(int n_pen, int m, const double* __restrict__ c,
                                                          const int32_t* __restrict__ idx,
                                                          int32_t* __restrict__ act,
                                                          int32_t* __restrict__ cnt,
                                                          int32_t* __restrict__ rowptr,
                                                          int32_t* cursor, int32_t* ent) {
  __shared__ int32_t wsum[16];
  const int t = threadIdx.x;
  // active list
  int na = 0;
  for (int j0 = 0; j0 < n_pen; j0 += 1024) {
    const int j = j0 + t;
    const int f = (j < n_pen && c[j] != 0.0) ? 1 : 0;
    int tot;
    const int pos = block_exclusive_scan(f, wsum, &tot);
    if (f) act[na + pos] = j;
    na += tot;
  }
  if (t == 0) *cnt = na;
  // per-row counts
  for (int a = t; a < m; a += 1024) __hip_atomic_store(&cursor[a], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  for (int e = t; e < 8 * na; e += 1024) {
    const int r = idx[(int64_t)act[e >> 3] * 8 + (e & 7)];
    if (r >= 0 && r < m) atomicAdd(&cursor[r], 1);
  }
  __syncthreads();
  // row pointers; the cursors restart at the row starts
  int base = 0;
  for (int a0 = 0; a0 < m; a0 += 1024) {
    const int a = a0 + t;
    const int v = a < m ? __hip_atomic_load(&cursor[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    int tot;
    const int pos = block_exclusive_scan(v, wsum, &tot);
    if (a < m) {
      rowptr[a] = base + pos;
      __hip_atomic_store(&cursor[a], base + pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    base += tot;
  }
  if (t == 0) rowptr[m] = base;
  __syncthreads();
  // fill, then order each row's keys
  for (int e = t; e < 8 * na; e += 1024) {
    const int r = idx[(int64_t)act[e >> 3] * 8 + (e & 7)];
    if (r >= 0 && r < m) ent[atomicAdd(&cursor[r], 1)] = e;
  }
  __syncthreads();
  for (int a = t; a < m; a += 1024) {
    const int e0 = rowptr[a], e1 = rowptr[a + 1];
    for (int i = e0 + 1; i < e1; ++i) {
      const int key = ent[i];
      int k = i - 1;
      while (k >= e0 && ent[k] > key) {
        ent[k + 1] = ent[k];
        --k;
      }
      ent[k + 1] = key;
    }
  }
}

// Two-sided contact of paired region nodes (a = lower lip, b = upper lip):
// active iff z_b < z_a; an active pair is a spring with W row [1, -1] on
// (a, b) and target 0.  One penalty slot per pair.
__global__ void k_detect_pairs(int n_pairs, const int32_t* __restrict__ pairs, double k,
                               const double* __restrict__ x2, int m, int32_t* __restrict__ idx,
                               double* __restrict__ w, double* __restrict__ c,
                               double* __restrict__ t) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_pairs) return;
  const int a = pairs[j], b = pairs[n_pairs + j];
  const bool ok = a >= 0 && a < m && b >= 0 && b < m;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    idx[j * 8 + s] = -1;
    w[j * 8 + s] = 0.0;
  }
  if (ok) {
    idx[j * 8] = a;
    idx[j * 8 + 1] = b;
    w[j * 8] = 1.0;
    w[j * 8 + 1] = -1.0;
  }
  c[j] = (ok && x2[2 * m + b] < x2[2 * m + a]) ? k : 0.0;
  t[j] = t[n_pairs + j] = t[2 * n_pairs + j] = 0.0;
}

void detect_pairs(int n_pairs, const int32_t* pairs, double k, const double* x2, int m,
                  int32_t* idx, double* w, double* c, double* t, hipStream_t st) {
  if (n_pairs > 0)
    k_detect_pairs<<<grid1(n_pairs), 256, 0, st>>>(n_pairs, pairs, k, x2, m, idx, w, c, t);
}

// Penalty terms, one thread per region node a (row a of W^T C W and entry a
// of f_col), over the active slots that name a (its incidence list, in
// increasing penalty order):
//   H[a + b*ldh] += c_j w_ja w_jb  for b <= a   (lower triangle, H may be NULL)
//   fcol[:, a]    = -sum_j c_j w_ja (W_j x2 - tscale t_j)
__global__ __launch_bounds__(64) void k_penalty_apply(int n_pen, const int32_t* __restrict__ act,
                                                      const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ ent,
                                                      const int32_t* __restrict__ idx,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ c,
                                                      const double* __restrict__ t,
                                                      double tscale,
                                                      const double* __restrict__ x2, int m,
                                                      double* H, int ldh, double* fcol) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= m) return;
  double f0 = 0.0, f1 = 0.0, f2 = 0.0;
  const int e1 = rowptr[a + 1];
  for (int e = rowptr[a]; e < e1; ++e) {
    const int key = ent[e];
    const int j = act[key >> 3], s = key & 7;
    const int32_t* ij = idx + (int64_t)j * 8;
    const double* wj = w + (int64_t)j * 8;
    const double coef = c[j] * wj[s];
    if (fcol) {
      double r0 = 0.0, r1 = 0.0, r2 = 0.0;
      for (int sb = 0; sb < 8; ++sb) {
        const int b = ij[sb];
        if (b < 0 || b >= m) continue;
        const double ws = wj[sb];
        r0 += ws * x2[b];
        r1 += ws * x2[m + b];
        r2 += ws * x2[2 * m + b];
      }
      r0 -= tscale * t[j];
      r1 -= tscale * t[n_pen + j];
      r2 -= tscale * t[2 * n_pen + j];
      f0 -= coef * r0;
      f1 -= coef * r1;
      f2 -= coef * r2;
    }
    if (H) {
      for (int sb = 0; sb < 8; ++sb) {
        const int b = ij[sb];
        if (b >= 0 && b <= a) H[(int64_t)a + (int64_t)b * ldh] += coef * wj[sb];
      }
    }
  }
  if (fcol) {
    fcol[a] = f0;
    fcol[m + a] = f1;
    fcol[2 * m + a] = f2;
  }
}

void penalty_prepare(int n_pen, int m, const double* c, const int32_t* idx, int32_t* act,
                     int32_t* cnt, int32_t* rowptr, int32_t* cursor, int32_t* ent, hipStream_t st) {
  k_penalty_prepare<<<1, 1024, 0, st>>>(n_pen, m, c, idx, act, cnt, rowptr, cursor, ent);
}

void penalty_apply(int n_pen, const int32_t* act, const int32_t* rowptr, const int32_t* ent,
                   const int32_t* idx, const double* w, const double* c, const double* t,
                   double tscale, const double* x2, int m, double* H, int ldh, double* fcol,
                   hipStream_t st) {
  if (m > 0)
    k_penalty_apply<<<grid1(m, 64), 64, 0, st>>>(n_pen, act, rowptr, ent, idx, w, c, t, tscale, x2,
                                                 m, H, ldh, fcol);
}

// Sum of squares of each of the three columns of a [3][m], one workgroup per
// column, fixed reduction order.
__global__ __launch_bounds__(256) void k_colnorm2_3(int m, const double* __restrict__ a,
                                                    double* __restrict__ out) {
  __shared__ double part[256];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) {
    const double x = a[(int64_t)v * m + i];
    s += x * x;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = part[0];
}

void colnorm2_3(int m, const double* a, double* out, hipStream_t st) {
  k_colnorm2_3<<<3, 256, 0, st>>>(m, a, out);
}

// out[0] = sum over listed nodes of ||x - xp||^2, out[1] = sum of ||x - X||^2
// (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void k_change_norms(int64_t cnt, const int32_t* __restrict__ ids,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ xp,
                                                       const double* __restrict__ X, int64_t n,
                                                       double* __restrict__ out) {
  __shared__ double r0[1024], r1[1024];
  double a = 0.0, b = 0.0;
  for (int64_t e = threadIdx.x; e < cnt; e += 1024) {
    const int64_t i = ids[e];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const double d = x[v * n + i] - xp[v * n + i];
      const double u = x[v * n + i] - X[v * n + i];
      a += d * d;
      b += u * u;
    }
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      r0[threadIdx.x] += r0[threadIdx.x + o];
      r1[threadIdx.x] += r1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = r0[0];
    out[1] = r1[0];
  }
}

void change_norms(int64_t cnt, const int32_t* ids, const double* x, const double* xp,
                  const double* X, int64_t n, double* out, hipStream_t st) {
  k_change_norms<<<1, 1024, 0, st>>>(cnt, ids, x, xp, X, n, out);
}

// Warm-start input [scale (x2 - x2_prev) (3m) ; active mask (m)] in float32;
// the mask is 1 for region nodes that are proxies with c > 0.
__global__ void k_ws_input(int m, const double* __restrict__ x2, const double* __restrict__ x2p,
                           float scale, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < 3 * (int64_t)m) out[e] = (float)((x2[e] - x2p[e]) * scale);
  if (e < m) out[3 * (int64_t)m + e] = 0.f;
}
__global__ void k_ws_mask(int n_prox, const int32_t* __restrict__ prox, const double* __restrict__ c,
                          int m, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n_prox && prox[j] >= 0 && prox[j] < m && c[j] != 0.0) out[3 * (int64_t)m + prox[j]] = 1.f;
}

void ws_input(int m, const double* x2, const double* x2p, float scale, int n_prox,
              const int32_t* prox, const double* c, float* out, hipStream_t st) {
  k_ws_input<<<grid1(3 * (int64_t)m), 256, 0, st>>>(m, x2, x2p, scale, out);
  if (n_prox > 0) k_ws_mask<<<grid1(n_prox), 256, 0, st>>>(n_prox, prox, c, m, out);
}

// x[:, ids[r]] += scale * d[:, r] for a float32 region increment
__global__ void k_region_add_f32(int64_t count, const int32_t* __restrict__ ids,
                                 const float* __restrict__ d, double scale, double* __restrict__ x,
                                 int64_t ldx) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= count) return;
  const int64_t i = ids[r];
  x[i] += scale * (double)d[r];
  x[ldx + i] += scale * (double)d[count + r];
  x[2 * ldx + i] += scale * (double)d[2 * count + r];
}

void region_add_f32(int64_t count, const int32_t* ids, const float* d, double scale, double* x,
                    int64_t ldx, hipStream_t st) {
  if (count > 0) k_region_add_f32<<<grid1(count), 256, 0, st>>>(count, ids, d, scale, x, ldx);
}

// base[dst[i]] += val[i] (distinct destinations).
__global__ void k_add_at(int64_t count, const int64_t* __restrict__ dst,
                         const double* __restrict__ val, double* __restrict__ base) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) base[dst[i]] += val[i];
}

void add_at(int64_t count, const int64_t* dst, const double* val, double* base, hipStream_t st) {
  if (count > 0) k_add_at<<<grid1(count), 256, 0, st>>>(count, dst, val, base);
}

// Backward-Euler inertia force: f[:, i] -= D_i (x[:, i] - y[:, i]).
__global__ void k_inertia_force(int64_t n, const double* __restrict__ D,
                                const double* __restrict__ x, const double* __restrict__ y,
                                double* __restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = D[i];
#pragma unroll
  for (int v = 0; v < 3; ++v) f[v * n + i] -= d * (x[v * n + i] - y[v * n + i]);
}

void inertia_force(int64_t n, const double* D, const double* x, const double* y, double* f,
                   hipStream_t st) {
  if (n > 0) k_inertia_force<<<grid1(n), 256, 0, st>>>(n, D, x, y, f);
}

// End of a backward-Euler step: v = (x - xp) / dt, xp = x, y = x + dt v.
__global__ void k_time_step_advance(int64_t len, double dt, const double* __restrict__ x,
                                    double* __restrict__ xp, double* __restrict__ v,
                                    double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const double xi = x[i];
  const double vi = (xi - xp[i]) / dt;
  v[i] = vi;
  xp[i] = xi;
  y[i] = xi + dt * vi;
}

void time_step_advance(int64_t len, double dt, const double* x, double* xp, double* v, double* y,
                       hipStream_t st) {
  if (len > 0) k_time_step_advance<<<grid1(len), 256, 0, st>>>(len, dt, x, xp, v, y);
}

// out = scale * d (+ a - b when a and b are given)
__global__ void k_scale_f32_to_f64(int64_t n, const float* __restrict__ d, double scale,
                                   const double* __restrict__ a, const double* __restrict__ b,
                                   double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = scale * (double)d[i];
  if (a) v += a[i] - b[i];
  out[i] = v;
}

void scale_f32_to_f64(int64_t n, const float* d, double scale, const double* a, const double* b,
                      double* out, hipStream_t st) {
  if (n > 0) k_scale_f32_to_f64<<<grid1(n), 256, 0, st>>>(n, d, scale, a, b, out);
}

// out = scale * ((x - xp) - (xp - xpp)), float32
__global__ void k_ws_target(int64_t n, const double* __restrict__ x, const double* __restrict__ xp,
                            const double* __restrict__ xpp, float scale, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)(((x[i] - xp[i]) - (xp[i] - xpp[i])) * scale);
}

void ws_target(int64_t n, const double* x, const double* xp, const double* xpp, float scale,
               float* out, hipStream_t st) {
  if (n > 0) k_ws_target<<<grid1(n), 256, 0, st>>>(n, x, xp, xpp, scale, out);
}

__global__ void k_axpy3_sum(int64_t len, const double* __restrict__ a, const double* b,
                            const double* c, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double s = a[i];
  if (b) s += b[i];
  if (c) s += c[i];
  out[i] = s;
}

void axpy3_sum(int m, const double* a, const double* b, const double* c, double* out,
               hipStream_t st) {
  const int64_t len = 3 * (int64_t)m;
  if (len > 0) k_axpy3_sum<<<grid1(len), 256, 0, st>>>(len, a, b, c, out);
}

__global__ void k_inner_update(int64_t len, const double* __restrict__ u, double* x2, double* d2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const double v = u[i];
  x2[i] += v;
  d2[i] += v;
}

void inner_update(int m, const double* u, double* x2, double* d2, hipStream_t st) {
  const int64_t len = 3 * (int64_t)m;
  if (len > 0) k_inner_update<<<grid1(len), 256, 0, st>>>(len, u, x2, d2);
}

}  // namespace pdk
