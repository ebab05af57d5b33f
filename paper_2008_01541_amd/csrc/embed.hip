// Embedded (non-conforming) collision proxies and rest-pose level-set
// self-collision (Sec. 3.3 eq. p_j_v; Sec. 5.1).
//
// A proxy embedded in the mesh moves with the tetrahedron that contains its
// rest position: p = sum_k w_k x_k over that tet's four region nodes, w its
// barycentric coordinates.  Point location takes the lowest-index candidate
// tet whose four barycentric coordinates are all >= -BARY_TOL.  One
// wavefront serves one query point: the 64 lanes test 64 consecutive
// candidates at a time, and the first batch that holds a hit gives the lowest
// index (ballot, lowest set lane), so the scan stops as early as a serial one.
//
// Level sets: a proxy found inside a tet of another body in the deformed
// configuration is taken back to the rest pose with the same barycentric
// coordinates; the body's rest signed distance phi (linear over the tet,
// phi < 0 inside) decides penetration; the target is the closest rest surface
// point X - phi g / |g|^2 (g = grad phi on that tet), carried to the deformed
// configuration by the rest tet of the same body that contains it.  The
// penalty is a zero-rest-length spring between the proxy and that surface
// point: W row [w over the proxy's nodes, -b' over the surface tet's nodes]
// (a node present twice carries the sum, in its first slot), target 0.
#include "common.h"

namespace pdk {

namespace {

constexpr double BARY_TOL = 1e-12;

inline unsigned grid_waves(long count, int waves_per_block) {
  return (unsigned)((count + waves_per_block - 1) / waves_per_block);
}

// Barycentric coordinates of p in the tet with corners a, b, c, d (Cramer's
// rule on [b - a, c - a, d - a] l = p - a).
__device__ inline void bary(const double p[3], const double a[3], const double b[3],
                            const double c[3], const double d[3], double l[4]) {
  const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  const double e3[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
  const double r[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
  const double c23[3] = {e2[1] * e3[2] - e2[2] * e3[1], e2[2] * e3[0] - e2[0] * e3[2],
                         e2[0] * e3[1] - e2[1] * e3[0]};
  const double det = e1[0] * c23[0] + e1[1] * c23[1] + e1[2] * c23[2];
  const double cr3[3] = {r[1] * e3[2] - r[2] * e3[1], r[2] * e3[0] - r[0] * e3[2],
                         r[0] * e3[1] - r[1] * e3[0]};
  const double c2r[3] = {e2[1] * r[2] - e2[2] * r[1], e2[2] * r[0] - e2[0] * r[2],
                         e2[0] * r[1] - e2[1] * r[0]};
  const double inv = 1.0 / det;
  l[1] = (r[0] * c23[0] + r[1] * c23[1] + r[2] * c23[2]) * inv;
  l[2] = (e1[0] * cr3[0] + e1[1] * cr3[1] + e1[2] * cr3[2]) * inv;
  l[3] = (e1[0] * c2r[0] + e1[1] * c2r[1] + e1[2] * c2r[2]) * inv;
  l[0] = 1.0 - l[1] - l[2] - l[3];
}

__device__ inline void load3(const double* pos, int m, int a, double out[3]) {
  out[0] = pos[a];
  out[1] = pos[m + a];
  out[2] = pos[2 * m + a];
}

// Lowest candidate e (cand: [4][nc] region-local ids into pos [3][m]) that
// contains p, among those whose body equals want_body (mode 1), differs from
// it (mode 2) or any body (mode 0, body may be null), skipping tets that
// share a node with excl[0..3] (excl[0] < 0: none).  Called by all 64 lanes of
// a wavefront with the same arguments; returns e (or -1) and l on every lane.
__device__ int wave_locate(const double p[3], int nc, const int32_t* __restrict__ cand,
                           const int32_t* __restrict__ body, int mode, int want_body,
                           const int32_t excl[4], const double* __restrict__ pos, int m,
                           double l_out[4]) {
  const int lane = threadIdx.x & 63;
  for (int base = 0; base < nc; base += 64) {
    const int e = base + lane;
    bool hit = false;
    double l[4] = {0.0, 0.0, 0.0, 0.0};
    if (e < nc) {
      const int v0 = cand[e], v1 = cand[nc + e], v2 = cand[2 * nc + e], v3 = cand[3 * nc + e];
      bool ok = v0 >= 0 && v0 < m && v1 >= 0 && v1 < m && v2 >= 0 && v2 < m && v3 >= 0 && v3 < m;
      if (ok && mode != 0) {
        const int bd = body[e];
        ok = (mode == 1) ? (bd == want_body) : (bd != want_body);
      }
      if (ok && excl[0] >= 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          ok = ok && v0 != excl[q] && v1 != excl[q] && v2 != excl[q] && v3 != excl[q];
      }
      if (ok) {
        double a[3], b[3], c[3], d[3];
        load3(pos, m, v0, a);
        load3(pos, m, v1, b);
        load3(pos, m, v2, c);
        load3(pos, m, v3, d);
        bary(p, a, b, c, d, l);
        hit = l[0] >= -BARY_TOL && l[1] >= -BARY_TOL && l[2] >= -BARY_TOL && l[3] >= -BARY_TOL;
      }
    }
    const unsigned long long mask = __ballot(hit);
    if (mask) {
      const int src = __ffsll((long long)mask) - 1;
#pragma unroll
      for (int q = 0; q < 4; ++q) l_out[q] = __shfl(l[q], src, 64);
      return base + src;
    }
  }
  return -1;
}

// ---- embedding of rest points -----------------------------------------------
__global__ __launch_bounds__(256) void k_embed_points(int n, const double* __restrict__ pts,
                                                      int nc, const int32_t* __restrict__ cand,
                                                      const double* __restrict__ pos, int m,
                                                      int32_t* __restrict__ tet,
                                                      int32_t* __restrict__ eidx,
                                                      double* __restrict__ ew) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= n) return;
  const double p[3] = {pts[j], pts[n + j], pts[2 * n + j]};
  const int32_t none[4] = {-1, -1, -1, -1};
  double l[4];
  const int e = wave_locate(p, nc, cand, nullptr, 0, 0, none, pos, m, l);
  if (lane == 0) {
    tet[j] = e;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      eidx[4 * j + q] = e >= 0 ? cand[q * nc + e] : -1;
      ew[4 * j + q] = e >= 0 ? l[q] : 0.0;
    }
  }
}

// ---- sphere detection for embedded proxies ----------------------------------
// The sphere rule of the conforming detector applied to p = sum_k w_k x2_k:
// inside iff ||p - c|| < r, deepest sphere wins (ties: lowest index), target
// c + r (p - c) / ||p - c|| (+z at the centre); inactive proxies keep t = p.
__global__ void k_detect_embedded_spheres(int n_prox, const int32_t* __restrict__ eidx,
                                          const double* __restrict__ ew, int n_sph,
                                          const double* __restrict__ sph, double k,
                                          const double* __restrict__ x2, int m,
                                          int32_t* __restrict__ idx, double* __restrict__ w,
                                          double* __restrict__ c, double* __restrict__ t) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_prox) return;
  bool ok = true;
  int nodes[4];
  double wt[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    nodes[q] = eidx[4 * j + q];
    wt[q] = ew[4 * j + q];
    ok = ok && nodes[q] >= 0 && nodes[q] < m;
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    idx[j * 8 + s] = (ok && s < 4) ? nodes[s] : -1;
    w[j * 8 + s] = (ok && s < 4) ? wt[s] : 0.0;
  }
  if (!ok) {
    c[j] = 0.0;
    t[j] = t[n_prox + j] = t[2 * n_prox + j] = 0.0;
    return;
  }
  double p[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) s = __dadd_rn(s, __dmul_rn(x2[v * m + nodes[q]], wt[q]));
    p[v] = s;
  }
  double best = -INFINITY;
  int hit = -1;
  double t0 = p[0], t1 = p[1], t2 = p[2];
  for (int s = 0; s < n_sph; ++s) {
    const double cx = sph[s], cy = sph[n_sph + s], cz = sph[2 * n_sph + s], r = sph[3 * n_sph + s];
    const double d0 = __dsub_rn(p[0], cx), d1 = __dsub_rn(p[1], cy), d2 = __dsub_rn(p[2], cz);
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
  c[j] = hit >= 0 ? k : 0.0;
  t[j] = t0;
  t[n_prox + j] = t1;
  t[2 * n_prox + j] = t2;
}

// ---- rest-pose level-set self-collision ---------------------------------------
__global__ __launch_bounds__(256) void k_detect_levelset(
    int n_prox, const int32_t* __restrict__ eidx, const double* __restrict__ ew,
    const int32_t* __restrict__ prox_body, int nc, const int32_t* __restrict__ cand,
    const double* __restrict__ cand_phi, const int32_t* __restrict__ cand_body,
    const double* __restrict__ rest2, double k, const double* __restrict__ x2, int m,
    int32_t* __restrict__ idx, double* __restrict__ w, double* __restrict__ c,
    double* __restrict__ t) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= n_prox) return;
  int32_t nodes[4];
  double wt[4];
  bool ok = true;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    nodes[q] = eidx[4 * j + q];
    wt[q] = ew[4 * j + q];
    ok = ok && nodes[q] >= 0 && nodes[q] < m;
  }
  // default: the proxy's own row, inactive
  int32_t row_i[8];
  double row_w[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    row_i[s] = (ok && s < 4) ? nodes[s] : -1;
    row_w[s] = (ok && s < 4) ? wt[s] : 0.0;
  }
  double cj = 0.0;
  if (ok) {
    double p[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) s += x2[v * m + nodes[q]] * wt[q];
      p[v] = s;
    }
    double b[4];
    const int pb = prox_body[j];
    const int e = wave_locate(p, nc, cand, cand_body, 2, pb, nodes, x2, m, b);
    if (e >= 0) {
      const int bd = cand_body[e];
      int tn[4];
      double ph4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        tn[q] = cand[q * nc + e];
        ph4[q] = cand_phi[q * nc + e];
      }
      double R[4][3];
#pragma unroll
      for (int q = 0; q < 4; ++q) load3(rest2, m, tn[q], R[q]);
      double X[3], ph = 0.0;
#pragma unroll
      for (int v = 0; v < 3; ++v) X[v] = R[0][v] * b[0] + R[1][v] * b[1] + R[2][v] * b[2] + R[3][v] * b[3];
#pragma unroll
      for (int q = 0; q < 4; ++q) ph += ph4[q] * b[q];
      if (ph < 0.0) {
        // grad phi on the rest tet: D^T g = (phi_q - phi_0)_{q=1..3},
        // D = [R1 - R0, R2 - R0, R3 - R0]; g = D^-T dphi through the adjugate
        double D[3][3];
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int v = 0; v < 3; ++v) D[v][q] = R[q + 1][v] - R[0][v];
        const double dp[3] = {ph4[1] - ph4[0], ph4[2] - ph4[0], ph4[3] - ph4[0]};
        // cofactor matrix C of D: D^-1 = C^T / det, so D^-T = C / det
        double Cf[3][3];
        Cf[0][0] = D[1][1] * D[2][2] - D[1][2] * D[2][1];
        Cf[0][1] = D[1][2] * D[2][0] - D[1][0] * D[2][2];
        Cf[0][2] = D[1][0] * D[2][1] - D[1][1] * D[2][0];
        Cf[1][0] = D[0][2] * D[2][1] - D[0][1] * D[2][2];
        Cf[1][1] = D[0][0] * D[2][2] - D[0][2] * D[2][0];
        Cf[1][2] = D[0][1] * D[2][0] - D[0][0] * D[2][1];
        Cf[2][0] = D[0][1] * D[1][2] - D[0][2] * D[1][1];
        Cf[2][1] = D[0][2] * D[1][0] - D[0][0] * D[1][2];
        Cf[2][2] = D[0][0] * D[1][1] - D[0][1] * D[1][0];
        const double det = D[0][0] * Cf[0][0] + D[0][1] * Cf[0][1] + D[0][2] * Cf[0][2];
        double g[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) g[v] = (Cf[v][0] * dp[0] + Cf[v][1] * dp[1] + Cf[v][2] * dp[2]) / det;
        const double gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        if (gg != 0.0) {
          const double Xs[3] = {X[0] - ph * g[0] / gg, X[1] - ph * g[1] / gg,
                                X[2] - ph * g[2] / gg};
          double b2[4];
          const int e2 = wave_locate(Xs, nc, cand, cand_body, 1, bd, nodes, rest2, m, b2);
          if (e2 >= 0) {
            int cnt = 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int v = cand[q * nc + e2];
              int at = -1;
#pragma unroll
              for (int s = 0; s < 8; ++s)
                if (at < 0 && s < cnt && row_i[s] == v) at = s;
              if (at >= 0) {
                row_w[at] -= b2[q];
              } else {
                // append in the next free slot (cnt < 8 always: 4 + 4 nodes)
#pragma unroll
                for (int s = 4; s < 8; ++s)
                  if (s == cnt) {
                    row_i[s] = v;
                    row_w[s] = -b2[q];
                  }
                ++cnt;
              }
            }
            cj = k;
          }
        }
      }
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      idx[j * 8 + s] = row_i[s];
      w[j * 8 + s] = row_w[s];
    }
    c[j] = cj;
    t[j] = t[n_prox + j] = t[2 * n_prox + j] = 0.0;
  }
}

}  // namespace

void embed_points(int n, const double* pts, int nc, const int32_t* cand, const double* pos, int m,
                  int32_t* tet, int32_t* eidx, double* ew, hipStream_t st) {
  if (n > 0)
    k_embed_points<<<grid_waves(n, 4), 256, 0, st>>>(n, pts, nc, cand, pos, m, tet, eidx, ew);
}

void detect_embedded_spheres(int n_prox, const int32_t* eidx, const double* ew, int n_sph,
                             const double* sph, double k, const double* x2, int m, int32_t* idx,
                             double* w, double* c, double* t, hipStream_t st) {
  if (n_prox > 0)
    k_detect_embedded_spheres<<<(n_prox + 255) / 256, 256, 0, st>>>(n_prox, eidx, ew, n_sph, sph,
                                                                   k, x2, m, idx, w, c, t);
}

void detect_levelset(int n_prox, const int32_t* eidx, const double* ew, const int32_t* prox_body,
                     int nc, const int32_t* cand, const double* cand_phi,
                     const int32_t* cand_body, const double* rest2, double k, const double* x2,
                     int m, int32_t* idx, double* w, double* c, double* t, hipStream_t st) {
  if (n_prox > 0)
    k_detect_levelset<<<grid_waves(n_prox, 4), 256, 0, st>>>(n_prox, eidx, ew, prox_body, nc,
                                                             cand, cand_phi, cand_body, rest2, k,
                                                             x2, m, idx, w, c, t);
}

}  // namespace pdk
