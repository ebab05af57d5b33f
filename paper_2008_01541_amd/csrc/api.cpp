// Host side of the C ABI: validation, partition, breadth-first interior levels,
// assembly plans, the level-by-level elimination that produces the Schur
// complement, and the per-iteration entry points.  All arithmetic on mesh
// data runs in the HIP kernels; the host only builds integer index structures.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <numeric>
#include <string>
#include <vector>

#include "ctx.h"

using namespace pdk;

namespace {

// Records HIP events around one phase of an entry point when timing is on.
struct PhaseTimer {
  pd_ctx* c;
  int phase;
  size_t i0 = 0;
  bool on;
  PhaseTimer(pd_ctx* ctx, int ph) : c(ctx), phase(ph), on(ctx->timing) {
    if (!on) return;
    i0 = c->ev_used;
    hipEvent_t e = c->next_event();
    if (!e) { on = false; return; }
    (void)hipEventRecord(e, c->st);
  }
  ~PhaseTimer() {
    if (!on) return;
    size_t i1 = c->ev_used;
    hipEvent_t e = c->next_event();
    if (!e) return;
    (void)hipEventRecord(e, c->st);
    c->ev_pairs.push_back({phase, {i0, i1}});
  }
};

}  // namespace

pd_status run_plan(pd_ctx* c, const Plan& P, const double* vals, double* dst) {
  if (P.dst.empty()) return PD_OK;
  int64_t *dp, *ds, *dd;
  CK(c->upload(&dp, P.ptr));
  CK(c->upload(&ds, P.src));
  CK(c->upload(&dd, P.dst));
  gather_assign((int64_t)P.dst.size(), dp, ds, vals, dd, dst, c->st);
  CK(c->check("gather_assign"));
  HIPCK(c, hipStreamSynchronize(c->st));
  // free the plan right away (it can be large)
  for (void* p : {(void*)dp, (void*)ds, (void*)dd}) {
    auto it = std::find(c->mem.ptrs.begin(), c->mem.ptrs.end(), p);
    if (it != c->mem.ptrs.end()) c->mem.ptrs.erase(it);
    (void)hipFree(p);
  }
  return PD_OK;
}

void free_now(pd_ctx* c, void* p) {
  auto it = std::find(c->mem.ptrs.begin(), c->mem.ptrs.end(), p);
  if (it != c->mem.ptrs.end()) c->mem.ptrs.erase(it);
  (void)hipFree(p);
}

namespace {

// In-place lower Cholesky of the n x n matrix A (leading dimension lda, a
// multiple of 16 so tiles start on 128-byte lines); tile inverses to d_linv,
// transpose of the factor in the upper triangle.
void cholesky(pd_ctx* c, double* A, int lda, int n, double* Yt = nullptr, int n_wg = 0,
              hipEvent_t after_reset = nullptr) {
  potrf_dataflow(A, lda, n, c->d_linv, c->d_sbuf, c->d_tflags, c->d_tticket, c->d_info, c->d_err,
                 n_wg > 0 ? std::min(n_wg, c->n_wg) : c->n_wg, Yt, c->st, c->d_cumarks,
                 after_reset);
}

inline int pad_to(int64_t v, int q) { return (int)((v + q - 1) / q * q); }

struct CSRBuild {
  std::vector<int32_t> ptr, col;
  std::vector<int64_t> plan_idx;  // position in the plan for each entry
};

pd_status build_impl(pd_ctx* c, const pd_mesh* M) {
  const int64_t n = M->n_nodes, T = M->n_tets;
  c->n = n;
  c->T = T;
  c->mu = M->mu;
  const int32_t* tets = M->tets;
  // ---- validation
  for (int64_t i = 0; i < 4 * T; ++i)
    if (tets[i] < 0 || tets[i] >= n) return c->fail(PD_ERR_INVALID, "tet vertex id out of range");
  for (int64_t e = 0; e < T; ++e)
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b)
        if (tets[a * T + e] == tets[b * T + e])
          return c->fail(PD_ERR_INVALID, "tet %lld repeats a vertex", (long long)e);
  if (!(M->mu > 0.0) || !std::isfinite(M->mu)) return c->fail(PD_ERR_INVALID, "mu must be positive");
  if (!(M->dt >= 0.0) || !std::isfinite(M->dt) ||
      (M->dt > 0.0 && (!(M->density > 0.0) || !std::isfinite(M->density))))
    return c->fail(PD_ERR_INVALID, "backward Euler needs dt > 0 and density > 0 (dt = 0: quasistatic)");
  c->dt = M->dt;
  if (!(M->mu_prime >= 0.0) || !std::isfinite(M->mu_prime) ||
      (M->mu_prime > 0.0 && !(M->sigma_min >= 0.0 && M->sigma_min <= M->sigma_max &&
                              std::isfinite(M->sigma_max))))
    return c->fail(PD_ERR_INVALID,
                   "biphasic material needs mu_prime >= 0 and 0 <= sigma_min <= sigma_max");
  c->mu_p = M->mu_prime;
  c->smin = M->sigma_min;
  c->smax = M->sigma_max;
  if (M->interior_order != 0 && M->interior_order != 1)
    return c->fail(PD_ERR_INVALID, "interior_order must be 0 (levels) or 1 (nested dissection)");
  if (M->nd_leaf < 0 || M->nd_leaf > 8192)
    return c->fail(PD_ERR_INVALID, "nd_leaf must lie in [0, 8192] (0: default)");
  const bool use_nd = M->interior_order == 1;

  // ---- partition (Sec. 4.2): x2 = region & free, x1 = other free nodes
  std::vector<int8_t> cls(n);   // 0 dirichlet, 1 interior (x1), 2 region (x2)
  for (int64_t i = 0; i < n; ++i)
    cls[i] = M->dirichlet[i] ? 0 : (M->region[i] ? 2 : 1);
  for (int64_t i = 0; i < n; ++i)
    if (cls[i] == 2) c->region_ids.push_back((int32_t)i);
  c->m = (int64_t)c->region_ids.size();
  if (c->m == 0) return c->fail(PD_ERR_INVALID, "the collision-prone region has no free node");
  std::vector<int32_t> rloc(n, -1);
  for (int64_t r = 0; r < c->m; ++r) rloc[c->region_ids[r]] = (int32_t)r;

  // E_beta = tets with all four vertices in x2 (Sec. 4.5), E_alpha = the rest
  std::vector<int32_t> alpha, beta;
  for (int64_t e = 0; e < T; ++e) {
    bool all2 = true;
    for (int a = 0; a < 4; ++a) all2 = all2 && cls[tets[a * T + e]] == 2;
    (all2 ? beta : alpha).push_back((int32_t)e);
  }
  c->nalpha = (int64_t)alpha.size();
  c->nbeta = (int64_t)beta.size();

  // ---- free-node adjacency; interior ordering: breadth-first levels of x1
  // from x2, or nested dissection
  std::vector<int64_t> adj_ptr;
  std::vector<int32_t> adj;
  free_adjacency(n, T, tets, cls, adj_ptr, adj);
  if (use_nd) {
    CK(nd_prepare(c, M->rest, cls, rloc, adj_ptr, adj, M->nd_leaf > 0 ? M->nd_leaf : 256));
    c->K = 0;
    c->lev_off.assign(1, c->n1);
  } else {
    std::vector<int32_t> dist(n, -1), frontier, next;
    for (int32_t r : c->region_ids) {
      for (int64_t k = adj_ptr[r]; k < adj_ptr[r + 1]; ++k) {
        const int32_t v = adj[k];
        if (cls[v] == 1 && dist[v] < 0) {
          dist[v] = 1;
          frontier.push_back(v);
        }
      }
    }
    int dmax = frontier.empty() ? 0 : 1;
    while (!frontier.empty()) {
      next.clear();
      for (int32_t u : frontier)
        for (int64_t k = adj_ptr[u]; k < adj_ptr[u + 1]; ++k) {
          const int32_t v = adj[k];
          if (cls[v] == 1 && dist[v] < 0) {
            dist[v] = dist[u] + 1;
            next.push_back(v);
          }
        }
      if (!next.empty()) dmax = dist[next[0]];
      frontier.swap(next);
    }
    // level index: unreachable interior nodes first (level 0, no coupling),
    // then distance dmax .. 1 (far to near)
    bool any_unreach = false;
    for (int64_t i = 0; i < n; ++i)
      if (cls[i] == 1 && dist[i] < 0) any_unreach = true;
    const int base = any_unreach ? 1 : 0;
    c->K = base + dmax;
    std::vector<std::vector<int32_t>> levels(c->K);
    for (int64_t i = 0; i < n; ++i) {
      if (cls[i] != 1) continue;
      const int lv = dist[i] < 0 ? 0 : base + (dmax - dist[i]);
      levels[lv].push_back((int32_t)i);
    }
    c->lev_off.assign(c->K + 1, 0);
    std::vector<int32_t> lev_nodes;
    for (int k = 0; k < c->K; ++k) {
      c->lev_off[k + 1] = c->lev_off[k] + (int64_t)levels[k].size();
      lev_nodes.insert(lev_nodes.end(), levels[k].begin(), levels[k].end());
      c->maxw = std::max<int64_t>(c->maxw, (int64_t)levels[k].size());
    }
    c->n1 = c->lev_off[c->K];
    CK(c->upload(&c->d_lev_nodes, lev_nodes));
  }
  const int K = c->K;
  const int64_t m = c->m;
  // level id and local index of every free node; region = level K
  std::vector<int32_t> lvl(n, -1), loc(n, -1);
  if (!use_nd) {
    std::vector<int32_t> h(c->n1);
    HIPCK(c, hipMemcpy(h.data(), c->d_lev_nodes, c->n1 * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int k = 0; k < K; ++k)
      for (int64_t p = c->lev_off[k]; p < c->lev_off[k + 1]; ++p) {
        lvl[h[p]] = k;
        loc[h[p]] = (int32_t)(p - c->lev_off[k]);
      }
    for (int64_t r = 0; r < m; ++r) {
      lvl[c->region_ids[r]] = K;
      loc[c->region_ids[r]] = (int32_t)r;
    }
  }
  auto width = [&](int k) -> int64_t { return k == K ? m : c->lev_off[k + 1] - c->lev_off[k]; };
  c->ldw.assign(K + 1, 0);
  for (int k = 0; k <= K; ++k) c->ldw[k] = (k == K) ? (int)m : pad_to(width(k), 16);
  for (int k = 0; k < K; ++k) c->maxldw = std::max<int64_t>(c->maxldw, c->ldw[k]);
  c->ldH = pad_to(m, 16);
  c->ldH32 = pad_to(m, 32);
  if (c->maxw > 46340 || m > 46340) return c->fail(PD_ERR_INVALID, "dense block too large");

  // ---- element geometry and stiffness on the GPU
  double *d_rest, *d_Bm, *d_vol, *d_Ke;
  int32_t* d_tets;
  {
    std::vector<double> rest(M->rest, M->rest + 3 * n);
    std::vector<int32_t> tv(tets, tets + 4 * T);
    CK(c->upload(&d_rest, rest));
    CK(c->upload(&d_tets, tv));
  }
  CK(c->alloc(&d_Bm, 9 * T));
  CK(c->alloc(&d_vol, T));
  CK(c->alloc(&d_Ke, 16 * T));
  tet_geometry(d_rest, n, d_tets, T, d_Bm, d_vol, c->st);
  element_stiffness(d_Bm, d_vol, T, c->mu + c->mu_p, d_Ke, c->st);   // mu' joins K (Sec. 5.3)
  CK(c->check("geometry"));
  {
    std::vector<double> vol(T);
    HIPCK(c, hipMemcpyAsync(vol.data(), d_vol, T * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCK(c, hipStreamSynchronize(c->st));
    for (int64_t e = 0; e < T; ++e)
      if (!(vol[e] > 0.0))
        return c->fail(PD_ERR_INVALID, "tet %lld has non-positive rest volume", (long long)e);
    if (c->dt > 0.0) {
      // lumped masses (a quarter of density * Vol_e per node), D = M / dt^2 on
      // the free nodes (zero on prescribed ones)
      std::vector<double> mass(n, 0.0);
      for (int a = 0; a < 4; ++a)
        for (int64_t e = 0; e < T; ++e) mass[tets[a * T + e]] += 0.25 * M->density * vol[e];
      c->h_D.assign(n, 0.0);
      for (int64_t i = 0; i < n; ++i)
        if (cls[i] != 0) c->h_D[i] = mass[i] / (c->dt * c->dt);
      CK(c->upload(&c->d_D, c->h_D));
    }
  }

  // ---- assembly plans: every K entry between free nodes, grouped by (row, col)
  // in the level ordering, with its element-matrix contributions in fixed order.
  struct Contrib {
    int32_t lr, lc;   // level of row / col node
    int32_t r, cc;    // local indices
    int64_t src;
  };
  int64_t lev_mat_total = 0;
  c->lev_mat_off.assign(K, 0);
  for (int k = 0; k < K; ++k) {
    c->lev_mat_off[k] = lev_mat_total;
    lev_mat_total += (int64_t)c->ldw[k] * width(k);
  }
  CK(c->alloc(&c->d_levmat, lev_mat_total));
  CK(c->alloc(&c->d_S, m * m));
  HIPCK(c, hipMemsetAsync(c->d_levmat, 0, lev_mat_total * sizeof(double), c->st));
  HIPCK(c, hipMemsetAsync(c->d_S, 0, m * m * sizeof(double), c->st));
  if (!use_nd) {
    // node-major bucketing of contributions
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t e = 0; e < T; ++e)
      for (int a = 0; a < 4; ++a) {
        const int32_t u = tets[a * T + e];
        if (cls[u] == 0) continue;
        for (int b = 0; b < 4; ++b)
          if (cls[tets[b * T + e]] != 0) cnt[u + 1]++;
      }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    std::vector<std::pair<int32_t, int64_t>> ent(cnt[n]);   // (col node, src)
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t e = 0; e < T; ++e)
      for (int a = 0; a < 4; ++a) {
        const int32_t u = tets[a * T + e];
        if (cls[u] == 0) continue;
        for (int b = 0; b < 4; ++b) {
          const int32_t v = tets[b * T + e];
          if (cls[v] != 0) ent[pos[u]++] = {v, (int64_t)(a * 4 + b) * T + e};
        }
      }
    Plan pl_lev, pl_S, pl_B, pl_Bt;
    // CSR structures of B_k (rows level k+1 -> cols level k) and B_k^T
    std::vector<std::vector<int32_t>> Bptr(K), Bcol(K), Btptr(K), Btcol(K);
    for (int k = 0; k < K; ++k) {
      Bptr[k].assign(width(k + 1) + 1, 0);
      Btptr[k].assign(width(k) + 1, 0);
    }
    // process rows in level order so CSR rows fill sequentially
    std::vector<int32_t> row_nodes;
    {
      std::vector<int32_t> h(c->n1);
      HIPCK(c, hipMemcpy(h.data(), c->d_lev_nodes, c->n1 * sizeof(int32_t), hipMemcpyDeviceToHost));
      row_nodes = h;
      row_nodes.insert(row_nodes.end(), c->region_ids.begin(), c->region_ids.end());
    }
    std::vector<int64_t> Bval_plan_pos, Btval_plan_pos;
    std::vector<std::vector<int64_t>> Bsrc_groups;  // not used
    for (int32_t u : row_nodes) {
      auto b = ent.begin() + cnt[u], e = ent.begin() + cnt[u + 1];
      // sort by (level, local col, src) for a fixed, ordered layout
      std::sort(b, e, [&](const std::pair<int32_t, int64_t>& x, const std::pair<int32_t, int64_t>& y) {
        if (lvl[x.first] != lvl[y.first]) return lvl[x.first] < lvl[y.first];
        if (loc[x.first] != loc[y.first]) return loc[x.first] < loc[y.first];
        return x.second < y.second;
      });
      const int lu = lvl[u];
      const int64_t ru = loc[u];
      for (auto it = b; it != e;) {
        auto jt = it;
        std::vector<int64_t> srcs;
        while (jt != e && jt->first == it->first) srcs.push_back((jt++)->second);
        const int32_t v = it->first;
        const int lv = lvl[v];
        const int64_t cv = loc[v];
        if (lv == lu) {
          if (lu == K) pl_S.add_group(srcs.data(), (int64_t)srcs.size(), ru + cv * m);
          else pl_lev.add_group(srcs.data(), (int64_t)srcs.size(),
                                c->lev_mat_off[lu] + ru + cv * c->ldw[lu]);
        } else if (lv == lu - 1) {   // row in level k+1, col in level k: B_k
          const int k = lv;
          Bcol[k].push_back((int32_t)cv);
          Bptr[k][ru + 1]++;
          pl_B.add_group(srcs.data(), (int64_t)srcs.size(), -1 - k);  // fixed up below
        } else if (lv == lu + 1) {   // row in level k, col in level k+1: B_k^T
          const int k = lu;
          Btcol[k].push_back((int32_t)cv);
          Btptr[k][ru + 1]++;
          pl_Bt.add_group(srcs.data(), (int64_t)srcs.size(), -1 - k);
        } else {
          return c->fail(PD_ERR_INVALID, "internal: coupling across non-adjacent levels");
        }
        it = jt;
      }
    }
    // CSR offsets and plan destinations (entries were appended in row order per level)
    c->B_ptr_off.assign(K + 1, 0);
    c->B_nnz_off.assign(K + 1, 0);
    c->Bt_ptr_off.assign(K + 1, 0);
    c->Bt_nnz_off.assign(K + 1, 0);
    std::vector<int32_t> allBptr, allBcol, allBtptr, allBtcol;
    for (int k = 0; k < K; ++k) {
      for (size_t i = 1; i < Bptr[k].size(); ++i) Bptr[k][i] += Bptr[k][i - 1];
      for (size_t i = 1; i < Btptr[k].size(); ++i) Btptr[k][i] += Btptr[k][i - 1];
      c->B_ptr_off[k + 1] = c->B_ptr_off[k] + (int64_t)Bptr[k].size();
      c->B_nnz_off[k + 1] = c->B_nnz_off[k] + (int64_t)Bcol[k].size();
      c->Bt_ptr_off[k + 1] = c->Bt_ptr_off[k] + (int64_t)Btptr[k].size();
      c->Bt_nnz_off[k + 1] = c->Bt_nnz_off[k] + (int64_t)Btcol[k].size();
      allBptr.insert(allBptr.end(), Bptr[k].begin(), Bptr[k].end());
      allBcol.insert(allBcol.end(), Bcol[k].begin(), Bcol[k].end());
      allBtptr.insert(allBtptr.end(), Btptr[k].begin(), Btptr[k].end());
      allBtcol.insert(allBtcol.end(), Btcol[k].begin(), Btcol[k].end());
    }
    // destinations: entries of B_k appear in the plan in level-major row order,
    // exactly the CSR order, so the j-th entry of level k goes to nnz_off[k] + j.
    {
      std::vector<int64_t> next(K, 0);
      for (auto& d : pl_B.dst) {
        const int k = -1 - (int)d;
        d = c->B_nnz_off[k] + next[k]++;
      }
      std::fill(next.begin(), next.end(), 0);
      for (auto& d : pl_Bt.dst) {
        const int k = -1 - (int)d;
        d = c->Bt_nnz_off[k] + next[k]++;
      }
    }
    // nonempty rows of each B_k (the rows that receive the elimination update)
    std::vector<int32_t> brows;
    c->Brows_off.assign(K + 1, 0);
    c->Brows_cnt.assign(K, 0);
    for (int k = 0; k < K; ++k) {
      c->Brows_off[k] = (int64_t)brows.size();
      for (int64_t r = 0; r + 1 < (int64_t)Bptr[k].size(); ++r)
        if (Bptr[k][r + 1] > Bptr[k][r]) brows.push_back((int32_t)r);
      c->Brows_cnt[k] = (int64_t)brows.size() - c->Brows_off[k];
    }
    c->Brows_off[K] = (int64_t)brows.size();
    CK(c->upload(&c->d_Bptr, allBptr));
    CK(c->upload(&c->d_Bcol, allBcol));
    CK(c->upload(&c->d_Btptr, allBtptr));
    CK(c->upload(&c->d_Btcol, allBtcol));
    CK(c->upload(&c->d_Brows, brows));
    CK(c->alloc(&c->d_Bval, std::max<int64_t>(1, c->B_nnz_off[K])));
    CK(c->alloc(&c->d_Btval, std::max<int64_t>(1, c->Bt_nnz_off[K])));
    CK(run_plan(c, pl_lev, d_Ke, c->d_levmat));
    CK(run_plan(c, pl_S, d_Ke, c->d_S));
    CK(run_plan(c, pl_B, d_Ke, c->d_Bval));
    CK(run_plan(c, pl_Bt, d_Ke, c->d_Btval));
    if (c->dt > 0.0) {
      // inertia diagonal into the diagonal blocks of the levels and of S
      std::vector<int64_t> off_lev, off_S;
      std::vector<double> val_lev, val_S;
      for (int64_t u = 0; u < n; ++u) {
        if (cls[u] == 0) continue;
        const int lu = lvl[u];
        const int64_t r = loc[u];
        if (lu == K) {
          off_S.push_back(r + r * m);
          val_S.push_back(c->h_D[u]);
        } else {
          off_lev.push_back(c->lev_mat_off[lu] + r + r * c->ldw[lu]);
          val_lev.push_back(c->h_D[u]);
        }
      }
      int64_t *d_ol = nullptr, *d_os = nullptr;
      double *d_vl = nullptr, *d_vs = nullptr;
      CK(c->upload(&d_ol, off_lev));
      CK(c->upload(&d_vl, val_lev));
      CK(c->upload(&d_os, off_S));
      CK(c->upload(&d_vs, val_S));
      add_at((int64_t)off_lev.size(), d_ol, d_vl, c->d_levmat, c->st);
      add_at((int64_t)off_S.size(), d_os, d_vs, c->d_S, c->st);
      CK(c->check("inertia diagonal"));
      HIPCK(c, hipStreamSynchronize(c->st));
      for (void* p : {(void*)d_ol, (void*)d_vl, (void*)d_os, (void*)d_vs}) free_now(c, p);
    }
  }

  // ---- A22^(beta): region-local CSR assembled from the E_beta tets only
  {
    std::vector<std::vector<std::pair<int32_t, int64_t>>> rows(m);
    for (int32_t e : beta)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
          rows[rloc[tets[a * T + e]]].push_back({rloc[tets[b * T + e]], (int64_t)(a * 4 + b) * T + e});
    Plan pl;
    std::vector<int32_t> ptr(m + 1, 0), col;
    for (int64_t r = 0; r < m; ++r) {
      auto& R = rows[r];
      std::sort(R.begin(), R.end());
      for (size_t i = 0; i < R.size();) {
        size_t j = i;
        std::vector<int64_t> srcs;
        while (j < R.size() && R[j].first == R[i].first) srcs.push_back(R[j++].second);
        pl.add_group(srcs.data(), (int64_t)srcs.size(), (int64_t)col.size());
        col.push_back(R[i].first);
        i = j;
      }
      ptr[r + 1] = (int32_t)col.size();
    }
    CK(c->upload(&c->d_Abptr, ptr));
    CK(c->upload(&c->d_Abcol, col));
    CK(c->alloc(&c->d_Abval, std::max<size_t>(1, col.size())));
    CK(run_plan(c, pl, d_Ke, c->d_Abval));
  }

  // ---- level-by-level elimination of x1 (one-way dissection in BFS levels):
  //   S_0 = D_0;  Z_k = S_k^-1;  S_{k+1} = D_{k+1} - B_k Z_k B_k^T;  S = S_K.
  c->ntm = (int)((m + NB - 1) / NB);
  const int64_t ntmax = (std::max<int64_t>(c->maxw, m) + NB - 1) / NB;
  CK(c->alloc(&c->d_linv, ntmax * NB * NB));
  CK(c->alloc(&c->d_sbuf, ntmax * NB * NB));
  CK(c->alloc(&c->d_info, 1));
  CK(c->alloc(&c->d_err, 1));
  CK(c->alloc(&c->d_ticket, 4));
  HIPCK(c, hipMemsetAsync(c->d_info, 0, sizeof(int), c->st));
  HIPCK(c, hipMemsetAsync(c->d_err, 0, sizeof(int), c->st));
  HIPCK(c, hipMemsetAsync(c->d_ticket, 0, 4 * sizeof(unsigned long long), c->st));
  {
    const int64_t nt2 = ntmax * (ntmax + 2);
    CK(c->alloc(&c->d_tflags, nt2));
    CK(c->alloc(&c->d_tticket, 4));
    CK(c->alloc(&c->d_cumarks, potrf_cu_slots()));
    HIPCK(c, hipMemsetAsync(c->d_tflags, 0, nt2 * sizeof(int), c->st));
    HIPCK(c, hipMemsetAsync(c->d_cumarks, 0, potrf_cu_slots() * sizeof(int), c->st));
    HIPCK(c, hipMemsetAsync(c->d_tticket, 0, 4 * sizeof(unsigned), c->st));
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      c->n_wg = 2 * ncu;
  }
  if (K > 0) {
    double *d_M, *d_X, *d_U;
    int64_t maxrows = 0;
    for (int k = 0; k < K; ++k) maxrows = std::max(maxrows, c->Brows_cnt[k]);
    CK(c->alloc(&d_M, c->maxldw * c->maxw));
    CK(c->alloc(&d_X, c->maxldw * c->maxw));
    CK(c->alloc(&d_U, c->maxw * std::max<int64_t>(1, maxrows)));
    for (int k = 0; k < K; ++k) {
      const int w = (int)width(k), ld = c->ldw[k];
      double* A = c->d_levmat + c->lev_mat_off[k];
      cholesky(c, A, ld, w);
      trtri_from_factor(A, ld, w, c->d_linv, d_M, d_X, ld, c->st);
      lauum_full(d_X, ld, w, A, ld, c->st);
      double* Nx = (k + 1 < K) ? c->d_levmat + c->lev_mat_off[k + 1] : c->d_S;
      const int ldn = c->ldw[k + 1];
      const int nr = (int)c->Brows_cnt[k];
      const int32_t* rows = c->d_Brows + c->Brows_off[k];
      const int32_t* bp = c->d_Bptr + c->B_ptr_off[k];
      const int32_t* bc = c->d_Bcol + c->B_nnz_off[k];
      const double* bv = c->d_Bval + c->B_nnz_off[k];
      dense_times_sparse_t(A, ld, w, nr, rows, bp, bc, bv, d_U, c->st);
      sub_sparse_times_dense(Nx, ldn, nr, rows, bp, bc, bv, d_U, w, c->st);
      CK(c->check("level elimination"));
    }
    HIPCK(c, hipStreamSynchronize(c->st));
    free_now(c, d_M);
    free_now(c, d_X);
    free_now(c, d_U);
    int info = 0;
    HIPCK(c, hipMemcpy(&info, c->d_info, sizeof(int), hipMemcpyDeviceToHost));
    if (info != 0)
      return c->fail(PD_ERR_NOT_SPD, "interior level block not positive definite (pivot %d)", info);
  }
  if (use_nd) CK(nd_factor(c, tets, T, cls, rloc, d_Ke));

  // ---- per-iteration data: E_alpha / E_beta tets, incidence lists, buffers
  {
    std::vector<int32_t> ta(4 * c->nalpha), tb_g(4 * c->nbeta), tb(4 * c->nbeta);
    for (int64_t s = 0; s < c->nalpha; ++s)
      for (int a = 0; a < 4; ++a) ta[a * c->nalpha + s] = tets[a * T + alpha[s]];
    for (int64_t s = 0; s < c->nbeta; ++s)
      for (int a = 0; a < 4; ++a) {
        tb_g[a * c->nbeta + s] = tets[a * T + beta[s]];
        tb[a * c->nbeta + s] = rloc[tets[a * T + beta[s]]];
      }
    CK(c->upload(&c->d_tets_alpha, ta));
    CK(c->alloc(&c->d_Bm_alpha, 9 * c->nalpha));
    CK(c->alloc(&c->d_vol_alpha, c->nalpha));
    tet_geometry(d_rest, n, c->d_tets_alpha, c->nalpha, c->d_Bm_alpha, c->d_vol_alpha, c->st);
    int32_t* d_tbg;
    CK(c->upload(&d_tbg, tb_g));
    CK(c->alloc(&c->d_Bm_beta, 9 * c->nbeta));
    CK(c->alloc(&c->d_vol_beta, c->nbeta));
    tet_geometry(d_rest, n, d_tbg, c->nbeta, c->d_Bm_beta, c->d_vol_beta, c->st);
    CK(c->upload(&c->d_tets_beta, tb));
    CK(c->check("subset geometry"));
    // incidence lists (node -> slot*4 + vertex), ordered by slot then vertex
    auto incidence = [&](const std::vector<int32_t>& tl, int64_t cnt, int64_t nodes,
                         std::vector<int32_t>& ptr, std::vector<int32_t>& ent) {
      ptr.assign(nodes + 1, 0);
      for (int64_t s = 0; s < cnt; ++s)
        for (int a = 0; a < 4; ++a) ptr[tl[a * cnt + s] + 1]++;
      for (int64_t i = 0; i < nodes; ++i) ptr[i + 1] += ptr[i];
      ent.assign(ptr[nodes], 0);
      std::vector<int32_t> p(ptr.begin(), ptr.end() - 1);
      for (int64_t s = 0; s < cnt; ++s)
        for (int a = 0; a < 4; ++a) ent[p[tl[a * cnt + s]]++] = (int32_t)(s * 4 + a);
    };
    std::vector<int32_t> ptr, ent;
    incidence(ta, c->nalpha, n, ptr, ent);
    CK(c->upload(&c->d_inc_a_ptr, ptr));
    CK(c->upload(&c->d_inc_a, ent));
    incidence(tb, c->nbeta, m, ptr, ent);
    CK(c->upload(&c->d_inc_b_ptr, ptr));
    CK(c->upload(&c->d_inc_b, ent));
    CK(c->upload(&c->d_region_ids, c->region_ids));
    CK(c->alloc(&c->d_fe, 12 * std::max<int64_t>(1, c->nalpha)));
    CK(c->alloc(&c->d_fe_b, 12 * std::max<int64_t>(1, c->nbeta)));
    HIPCK(c, hipStreamSynchronize(c->st));
    free_now(c, d_tbg);
  }
  free_now(c, d_Ke);
  free_now(c, d_Bm);
  free_now(c, d_vol);
  c->d_rest = d_rest;                 // kept for pd_displacement_change
  {
    std::vector<int32_t> fr;
    for (int64_t i = 0; i < n; ++i)
      if (cls[i] != 0) fr.push_back((int32_t)i);
    c->n_free = (int64_t)fr.size();
    CK(c->upload(&c->d_free_ids, fr));
  }
  free_now(c, d_tets);
  CK(c->alloc(&c->d_H, (int64_t)c->ldH * m));
  CK(c->alloc(&c->d_y, 3 * m));
  CK(c->alloc(&c->d_ys, 3 * m));
  sentinel_fill(3 * m, c->d_ys, c->st);
  CK(c->alloc(&c->d_Yt, (int64_t)NB * m));
  CK(c->alloc(&c->d_res, 3 * m));
  CK(c->alloc(&c->d_norms, 8));
  CK(c->alloc(&c->d_fhat, 3 * std::max<int64_t>(1, c->n1)));
  CK(c->alloc(&c->d_v, 3 * std::max<int64_t>(1, c->n1)));
  CK(c->alloc(&c->d_xs, 3 * std::max<int64_t>(1, c->n1)));
  CK(c->alloc(&c->d_tmp, 3 * std::max<int64_t>(1, c->maxw)));
  CK(c->alloc(&c->d_P, std::max(sweep_workspace(c->maxw), sweep_workspace(m))));
  HIPCK(c, hipStreamSynchronize(c->st));
  return PD_OK;
}

pd_status ensure_pen_cap(pd_ctx* c, int32_t n) {
  if (n <= c->pen_cap) return PD_OK;
  int32_t cap = std::max<int32_t>(n, 2 * c->pen_cap);
  for (void* p : {(void*)c->d_pidx, (void*)c->d_pw, (void*)c->d_pc, (void*)c->d_pt,
                  (void*)c->d_pact, (void*)c->d_pent})
    if (p) {
      HIPCK(c, hipStreamSynchronize(c->st));
      free_now(c, p);
    }
  if (!c->d_pnact) CK(c->alloc(&c->d_pnact, 1));
  if (!c->d_prow) CK(c->alloc(&c->d_prow, c->m + 1));
  if (!c->d_pcur) CK(c->alloc(&c->d_pcur, std::max<int64_t>(c->m, 1)));
  CK(c->alloc(&c->d_pent, 8 * (int64_t)cap));
  CK(c->alloc(&c->d_pact, cap));
  CK(c->alloc(&c->d_pidx, 8 * (int64_t)cap));
  CK(c->alloc(&c->d_pw, 8 * (int64_t)cap));
  CK(c->alloc(&c->d_pc, cap));
  CK(c->alloc(&c->d_pt, 3 * (int64_t)cap));
  c->pen_cap = cap;
  return PD_OK;
}

bool bad_ctx(const pd_ctx* c) { return c == nullptr; }

thread_local std::string g_build_error;

}  // namespace


// ===========================================================================
extern "C" {

pd_status pd_schur_build(const pd_mesh* mesh, void* hip_stream, pd_ctx** out) {
  if (!out) return PD_ERR_INVALID;
  *out = nullptr;
  if (!mesh || !mesh->rest || !mesh->tets || !mesh->region || !mesh->dirichlet ||
      mesh->n_nodes <= 0 || mesh->n_tets <= 0 || mesh->n_nodes > INT32_MAX ||
      mesh->n_tets > (INT32_MAX / 4))
    return PD_ERR_INVALID;
  pd_ctx* c = new pd_ctx();
  c->st = (hipStream_t)hip_stream;
  pd_status s = build_impl(c, mesh);
  if (s != PD_OK) {
    (void)hipStreamSynchronize(c->st);
    // keep the message reachable through a static copy, then free the context
    g_build_error = c->err;
    delete c;
    return s;
  }
  *out = c;
  return PD_OK;
}

pd_status pd_query(const pd_ctx* c, int64_t* m, int64_t* n1, int64_t* n_beta, int64_t* n_alpha,
                   int64_t* n_levels) {
  if (bad_ctx(c)) return PD_ERR_INVALID;
  if (m) *m = c->m;
  if (n1) *n1 = c->n1;
  if (n_beta) *n_beta = c->nbeta;
  if (n_alpha) *n_alpha = c->nalpha;
  if (n_levels) *n_levels = c->nd ? nd_height(c) : c->K;
  return PD_OK;
}

pd_status pd_region_nodes(const pd_ctx* c, int32_t* ids) {
  if (bad_ctx(c) || !ids) return PD_ERR_INVALID;
  std::memcpy(ids, c->region_ids.data(), c->m * sizeof(int32_t));
  return PD_OK;
}

pd_status pd_get_schur(pd_ctx* c, double* S) {
  if (bad_ctx(c) || !S) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  HIPCK(c, hipMemcpyAsync(S, c->d_S, c->m * c->m * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  return PD_OK;
}

pd_status pd_region_gather(pd_ctx* c, const double* x, double* x2) {
  if (bad_ctx(c) || !x || !x2) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  gather_rows3(c->m, c->d_region_ids, x, c->n, x2, c->m, c->st);
  return c->check("pd_region_gather");
}

pd_status pd_local_step_full(pd_ctx* c, const double* x, void* R_alpha, double* f, int rot_fp32) {
  if (bad_ctx(c) || !x || !f) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  if (c->dt > 0.0 && !c->d_target)
    return c->fail(PD_ERR_STATE, "backward Euler: pd_set_inertia_target before pd_local_step_full");
  PhaseTimer tm(c, PD_PHASE_LOCAL_FULL);
  local_step(c->nalpha, c->d_tets_alpha, c->nalpha, c->d_Bm_alpha, c->d_vol_alpha, c->nalpha, x,
             c->n, c->mu, c->mu_p, c->smin, c->smax, c->d_fe, R_alpha, rot_fp32 ? 1 : 0, c->st);
  node_gather3(c->n, c->d_inc_a_ptr, c->d_inc_a, c->d_fe, c->nalpha, nullptr, f, c->n, 0, c->st);
  if (c->dt > 0.0) inertia_force(c->n, c->d_D, x, c->d_target, f, c->st);
  return c->check("pd_local_step_full");
}

pd_status pd_set_inertia_target(pd_ctx* c, const double* y) {
  if (bad_ctx(c)) return PD_ERR_INVALID;
  if (!(c->dt > 0.0)) return c->fail(PD_ERR_STATE, "quasistatic context: no inertia target");
  c->d_target = y;
  return PD_OK;
}

pd_status pd_time_step_advance(pd_ctx* c, const double* x, double* x_prev, double* v, double* y) {
  if (bad_ctx(c) || !x || !x_prev || !v || !y) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  if (!(c->dt > 0.0)) return c->fail(PD_ERR_STATE, "quasistatic context: no time step");
  time_step_advance(3 * c->n, c->dt, x, x_prev, v, y, c->st);
  return c->check("pd_time_step_advance");
}

pd_status pd_condense_rhs(pd_ctx* c, const double* f, double* y2) {
  if (bad_ctx(c) || !f || !y2) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  const int64_t n1 = c->n1, m = c->m;
  PhaseTimer tm(c, PD_PHASE_CONDENSE);
  if (c->nd) {
    nd_condense(c, f, y2);
    c->have_condense = true;
    return c->check("pd_condense_rhs");
  }
  gather_rows3(n1, c->d_lev_nodes, f, c->n, c->d_fhat, n1, c->st);
  gather_rows3(m, c->d_region_ids, f, c->n, y2, m, c->st);
  for (int k = 0; k < c->K; ++k) {
    const int64_t off = c->lev_off[k], w = c->lev_off[k + 1] - off;
    sweep_symv(c->d_levmat + c->lev_mat_off[k], c->ldw[k], (int)w, c->d_fhat + off, n1, c->d_P,
               c->st);
    sweep_assemble((int)w, c->d_P, nullptr, 0, c->d_v + off, n1, c->st);     // v_k = Z_k fhat_k
    const int32_t* bp = c->d_Bptr + c->B_ptr_off[k];
    const int32_t* bc = c->d_Bcol + c->B_nnz_off[k];
    const double* bv = c->d_Bval + c->B_nnz_off[k];
    if (k + 1 < c->K) {
      const int64_t off2 = c->lev_off[k + 1], w2 = c->lev_off[k + 2] - off2;
      csr_spmv3(w2, bp, bc, bv, c->d_v + off, n1, -1.0, c->d_fhat + off2, n1, c->d_fhat + off2, n1,
                c->st);
    } else {
      csr_spmv3(m, bp, bc, bv, c->d_v + off, n1, -1.0, y2, m, y2, m, c->st);
    }
  }
  c->have_condense = true;
  return c->check("pd_condense_rhs");
}

// x1 += v - A11^-1 A12 delta2 level by level (v = A11^-1 f1 from the last
// condensation, kept per level in d_v; zero_w: v = 0), then x2 += delta2.
// With the nested-dissection factor the interior part runs its sweep instead.
static void backsub_levels(pd_ctx* c, const double* delta2, double* x, bool zero_w) {
  const int64_t n1 = c->n1, m = c->m;
  if (c->nd) {
    nd_backsub(c, delta2, x, zero_w);
  } else if (n1 > 0) {
    if (zero_w) zero_f64(3 * n1, c->d_v, c->st);
    // level k: tmp = B_k^T x_{k+1} (x_K = delta2), then xs_k = v_k - Z_k tmp
    for (int k = c->K - 1; k >= 0; --k) {
      const int64_t off = c->lev_off[k], w = c->lev_off[k + 1] - off;
      const int32_t* tp = c->d_Btptr + c->Bt_ptr_off[k];
      const int32_t* tc = c->d_Btcol + c->Bt_nnz_off[k];
      const double* tv = c->d_Btval + c->Bt_nnz_off[k];
      const double* xn = (k + 1 < c->K) ? c->d_xs + c->lev_off[k + 1] : delta2;
      const int64_t ldxn = (k + 1 < c->K) ? n1 : m;
      csr_spmv3(w, tp, tc, tv, xn, ldxn, 1.0, c->d_tmp, c->maxw, nullptr, 0, c->st);
      sweep_symv(c->d_levmat + c->lev_mat_off[k], c->ldw[k], (int)w, c->d_tmp, c->maxw, c->d_P,
                 c->st);
      sweep_assemble((int)w, c->d_P, c->d_v + off, n1, c->d_xs + off, n1, c->st);
    }
    scatter_add_rows3(n1, c->d_lev_nodes, c->d_xs, n1, x, c->n, c->st);
  }
  scatter_add_rows3(m, c->d_region_ids, delta2, m, x, c->n, c->st);
}

pd_status pd_backsub(pd_ctx* c, const double* delta2, double* x) {
  if (bad_ctx(c) || !delta2 || !x) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  if (!c->have_condense) return c->fail(PD_ERR_STATE, "pd_backsub needs a preceding pd_condense_rhs");
  PhaseTimer tm(c, PD_PHASE_BACKSUB);
  backsub_levels(c, delta2, x, false);
  return c->check("pd_backsub");
}

pd_status pd_warmstart_apply(pd_ctx* c, const float* d2, double scale, const double* x2_prev1,
                             const double* x2_prev2, double* x) {
  if (bad_ctx(c) || !d2 || !x || !std::isfinite(scale) || (!x2_prev1 != !x2_prev2))
    return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  if (!c->d_ext) CK(c->alloc(&c->d_ext, 3 * std::max<int64_t>(1, c->m)));
  scale_f32_to_f64(3 * c->m, d2, scale, x2_prev1, x2_prev2, c->d_ext, c->st);
  // the elastic response of the interior with f1 = 0
  backsub_levels(c, c->d_ext, x, true);
  c->have_condense = false;           // v no longer holds a condensation
  return c->check("pd_warmstart_apply");
}

pd_status pd_detect_spheres(pd_ctx* c, int32_t n_prox, const int32_t* prox, int32_t n_sph,
                            const double* spheres, double k, const double* x2, int32_t* idx,
                            double* w, double* cc, double* t) {
  if (bad_ctx(c) || n_prox < 0 || n_sph < 0 || (n_prox > 0 && (!prox || !x2 || !idx || !w || !cc || !t)) ||
      (n_sph > 0 && !spheres) || !(k >= 0.0))
    return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  PhaseTimer tm(c, PD_PHASE_DETECT);
  detect_spheres(n_prox, prox, n_sph, spheres, k, x2, (int)c->m, idx, w, cc, t, c->st);
  return c->check("pd_detect_spheres");
}

pd_status pd_detect_pairs(pd_ctx* c, int32_t n_pairs, const int32_t* pairs, double k,
                          const double* x2, int32_t* idx, double* w, double* cc, double* t) {
  if (bad_ctx(c) || n_pairs < 0 || !(k >= 0.0) ||
      (n_pairs > 0 && (!pairs || !x2 || !idx || !w || !cc || !t)))
    return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  PhaseTimer tm(c, PD_PHASE_DETECT);
  detect_pairs(n_pairs, pairs, k, x2, (int)c->m, idx, w, cc, t, c->st);
  return c->check("pd_detect_pairs");
}

pd_status pd_embed_points(pd_ctx* c, int32_t n_pts, const double* pts, int32_t n_cand,
                          const int32_t* cand, const double* pos, int32_t* tet, int32_t* eidx,
                          double* ew) {
  if (bad_ctx(c) || n_pts < 0 || n_cand < 0 ||
      (n_pts > 0 && (!pts || !pos || !tet || !eidx || !ew || (n_cand > 0 && !cand))))
    return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  embed_points(n_pts, pts, n_cand, cand, pos, (int)c->m, tet, eidx, ew, c->st);
  return c->check("pd_embed_points");
}

pd_status pd_detect_embedded_spheres(pd_ctx* c, int32_t n_prox, const int32_t* eidx,
                                     const double* ew, int32_t n_sph, const double* spheres,
                                     double k, const double* x2, int32_t* idx, double* w,
                                     double* cc, double* t) {
  if (bad_ctx(c) || n_prox < 0 || n_sph < 0 || !(k >= 0.0) ||
      (n_prox > 0 && (!eidx || !ew || !x2 || !idx || !w || !cc || !t)) || (n_sph > 0 && !spheres))
    return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  PhaseTimer tm(c, PD_PHASE_DETECT);
  detect_embedded_spheres(n_prox, eidx, ew, n_sph, spheres, k, x2, (int)c->m, idx, w, cc, t,
                          c->st);
  return c->check("pd_detect_embedded_spheres");
}

pd_status pd_detect_levelset(pd_ctx* c, int32_t n_prox, const int32_t* eidx, const double* ew,
                             const int32_t* prox_body, int32_t n_cand, const int32_t* cand,
                             const double* cand_phi, const int32_t* cand_body,
                             const double* rest2, double k, const double* x2, int32_t* idx,
                             double* w, double* cc, double* t) {
  if (bad_ctx(c) || n_prox < 0 || n_cand < 0 || !(k >= 0.0) ||
      (n_prox > 0 && (!eidx || !ew || !prox_body || !rest2 || !x2 || !idx || !w || !cc || !t)) ||
      (n_cand > 0 && (!cand || !cand_phi || !cand_body)))
    return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  PhaseTimer tm(c, PD_PHASE_DETECT);
  detect_levelset(n_prox, eidx, ew, prox_body, n_cand, cand, cand_phi, cand_body, rest2, k, x2,
                  (int)c->m, idx, w, cc, t, c->st);
  return c->check("pd_detect_levelset");
}

pd_status pd_collision_update(pd_ctx* c, int32_t n_pen, const int32_t* idx, const double* w,
                              const double* cc, const double* t, const double* x2, double* f_col) {
  if (bad_ctx(c) || n_pen < 0 || !x2 || !f_col || (n_pen > 0 && (!idx || !w || !cc || !t)))
    return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  CK(ensure_pen_cap(c, std::max<int32_t>(n_pen, 1)));
  PhaseTimer tm(c, PD_PHASE_COLLISION);
  if (n_pen > 0) {                    // copies by kernels (capturable like every other step)
    copy_i32(8 * (long)n_pen, idx, c->d_pidx, c->st);
    copy_f64(8 * (long)n_pen, w, c->d_pw, c->st);
    copy_f64((long)n_pen, cc, c->d_pc, c->st);
    copy_f64(3 * (long)n_pen, t, c->d_pt, c->st);
  }
  c->n_pen = n_pen;
  penalty_prepare(n_pen, (int)c->m, c->d_pc, c->d_pidx, c->d_pact, c->d_pnact, c->d_prow,
                  c->d_pcur, c->d_pent, c->st);
  penalty_apply(n_pen, c->d_pact, c->d_prow, c->d_pent, c->d_pidx, c->d_pw, c->d_pc, c->d_pt, 1.0, x2,
                (int)c->m, nullptr, 0, f_col, c->st);
  c->stale = true;
  c->lp_stale = true;
  return c->check("pd_collision_update");
}

pd_status pd_local_step_region(pd_ctx* c, const double* x2, void* R_beta, double* f_beta,
                               int rot_fp32) {
  if (bad_ctx(c) || !x2 || !f_beta) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  if (c->nbeta == 0) {
    zero_f64(3 * c->m, f_beta, c->st);
    return c->check("pd_local_step_region");
  }
  PhaseTimer tm(c, PD_PHASE_LOCAL_REGION);
  local_step(c->nbeta, c->d_tets_beta, c->nbeta, c->d_Bm_beta, c->d_vol_beta, c->nbeta, x2, c->m,
             c->mu, c->mu_p, c->smin, c->smax, c->d_fe_b, R_beta, rot_fp32 ? 1 : 0, c->st);
  node_gather3(c->m, c->d_inc_b_ptr, c->d_inc_b, c->d_fe_b, c->nbeta, nullptr, f_beta, c->m, 0,
               c->st);
  return c->check("pd_local_step_region");
}

pd_status pd_assemble_rhs(pd_ctx* c, const double* ft, const double* f_beta, const double* f_col,
                          double* g) {
  if (bad_ctx(c) || !ft || !g) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  PhaseTimer tm(c, PD_PHASE_ASSEMBLE);
  axpy3_sum((int)c->m, ft, f_beta, f_col, g, c->st);
  return c->check("pd_assemble_rhs");
}

namespace {

// H = S + W^T C W on the lower tiles of d_H (FP64).
void build_H(pd_ctx* c) {
  const int m = (int)c->m;
  PhaseTimer tm(c, PD_PHASE_HBUILD);
  copy_lower_tiles(c->d_S, m, c->d_H, c->ldH, m, c->st);
  if (c->n_pen > 0)
    penalty_apply(c->n_pen, c->d_pact, c->d_prow, c->d_pent, c->d_pidx, c->d_pw, c->d_pc, c->d_pt,
                  0.0, nullptr, m, c->d_H, c->ldH, nullptr, c->st);
}

// res = g - (S + P) u in FP64; returns max over columns of ||res|| / ||g|| (synchronizes).
pd_status residual(pd_ctx* c, const double* g, const double* u, double* rel) {
  const int m = (int)c->m;
  HIPCK(c, hipMemcpyAsync(c->d_res, g, 3 * (size_t)m * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  symv3(c->d_S, m, m, u, m, -1.0, 1.0, c->d_res, m, c->st);
  if (c->n_pen > 0) {
    penalty_apply(c->n_pen, c->d_pact, c->d_prow, c->d_pent, c->d_pidx, c->d_pw, c->d_pc, c->d_pt,
                  0.0, u, m, nullptr, 0, c->d_y, c->st);
    axpy3_sum(m, c->d_res, c->d_y, nullptr, c->d_res, c->st);
  }
  colnorm2_3(m, c->d_res, c->d_norms, c->st);
  colnorm2_3(m, g, c->d_norms + 3, c->st);
  double nrm[6];
  HIPCK(c, hipMemcpyAsync(nrm, c->d_norms, 6 * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCK(c, hipStreamSynchronize(c->st));
  double rr = 0.0;
  for (int v = 0; v < 3; ++v)
    if (nrm[3 + v] > 0) rr = std::max(rr, std::sqrt(nrm[v] / nrm[3 + v]));
  *rel = rr;
  return PD_OK;
}

// nq = -(S + P) p in FP64 (three columns).
void neg_apply_H(pd_ctx* c, const double* p, double* nq) {
  const int m = (int)c->m;
  symv3(c->d_S, m, m, p, m, -1.0, 0.0, nq, m, c->st);
  if (c->n_pen > 0) {
    penalty_apply(c->n_pen, c->d_pact, c->d_prow, c->d_pent, c->d_pidx, c->d_pw, c->d_pc, c->d_pt,
                  0.0, p, m, nullptr, 0, c->d_y, c->st);
    axpy3_sum(m, nq, c->d_y, nullptr, nq, c->st);
  }
}

// z = M^-1 r with M = D^-1 L L^T D^-1 from the low-precision factor.
void lp_precondition(pd_ctx* c, const double* r, double* z) {
  trsv3_lp_solve(c->d_H32, c->ldH32, (int)c->m, c->d_linv32, c->d_dvec, r, c->d_lpb, c->d_lpy, z,
                 0, c->d_lp_ticket, c->d_err, c->st);
}

// max over columns of ||r_v|| / ||g_v|| from squared norms computed on the
// device (synchronizes).
pd_status column_ratio(pd_ctx* c, const double* r, const double* g, double* rel) {
  const int m = (int)c->m;
  colnorm2_3(m, r, c->d_norms, c->st);
  colnorm2_3(m, g, c->d_norms + 3, c->st);
  double nrm[6];
  HIPCK(c, hipMemcpyAsync(nrm, c->d_norms, 6 * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCK(c, hipStreamSynchronize(c->st));
  double rr = 0.0;
  for (int v = 0; v < 3; ++v)
    if (nrm[3 + v] > 0) rr = std::max(rr, std::sqrt(nrm[v] / nrm[3 + v]));
    else if (nrm[v] > 0) rr = std::numeric_limits<double>::infinity();
  *rel = rr;
  return PD_OK;
}

// Preconditioned conjugate gradients on H u = g from the initial u, the
// low-precision factor as preconditioner, H applied in FP64.  The updated
// residual is checked after every step; once it meets the tolerance the true
// residual g - H u is recomputed, and the iteration restarts from it if
// rounding has separated the two.  Returns the true relative residual and
// the number of steps.
pd_status refine_pcg(pd_ctx* c, const double* g, double* u, double* rel, int* steps) {
  const int m = (int)c->m;
  double* r = c->d_res;
  double* p = c->d_cgp;
  double* nq = c->d_cgq;
  double* z = c->d_cgz;
  double* rz[2] = {c->d_cgs, c->d_cgs + 3};
  double* pnq = c->d_cgs + 6;
  double rr = 0.0;
  int it = 0;
  CK(residual(c, g, u, &rr));             // r = g - H u
  while (!(rr <= c->ir_tol) && it < c->max_ir) {
    // (re)start from the true residual in r
    lp_precondition(c, r, z);
    copy_f64(3 * (long)m, z, p, c->st);
    dot3(m, r, z, rz[0], c->st);
    int cur = 0;
    double upd = rr;
    while (it < c->max_ir) {
      neg_apply_H(c, p, nq);
      dot3(m, p, nq, pnq, c->st);
      cg_update(m, rz[cur], pnq, p, nq, u, r, c->st);
      ++it;
      CK(column_ratio(c, r, g, &upd));
      if (upd <= c->ir_tol || !std::isfinite(upd)) break;
      lp_precondition(c, r, z);
      dot3(m, r, z, rz[cur ^ 1], c->st);
      cg_direction(m, rz[cur ^ 1], rz[cur], z, p, c->st);
      cur ^= 1;
    }
    CK(residual(c, g, u, &rr));
    if (!std::isfinite(upd) || !std::isfinite(rr)) break;
  }
  *rel = rr;
  *steps = it;
  return PD_OK;
}

pd_status ensure_lp_buffers(pd_ctx* c) {
  if (c->d_H32) return PD_OK;
  const int64_t m = c->m;
  CK(c->alloc(&c->d_H32, (int64_t)c->ldH32 * m));
  CK(c->alloc(&c->d_linv32, (int64_t)c->ntm * NB * NB));
  CK(c->alloc(&c->d_lpb, 3 * m));
  CK(c->alloc(&c->d_lpy, 3 * m));
  CK(c->alloc(&c->d_dvec, m));
  CK(c->alloc(&c->d_cgp, 3 * m));
  CK(c->alloc(&c->d_cgq, 3 * m));
  CK(c->alloc(&c->d_cgz, 3 * m));
  CK(c->alloc(&c->d_cgs, 16));
  CK(c->alloc(&c->d_lp_ticket, 2));
  HIPCK(c, hipMemsetAsync(c->d_lp_ticket, 0, 2 * sizeof(unsigned long long), c->st));
  sentinel_fill(3 * m, c->d_lpy, c->st);
  return PD_OK;
}

}  // namespace

pd_status pd_global_solve(pd_ctx* c, const double* g, double* u, pd_precision prec,
                          pd_solve_info* info) {
  if (bad_ctx(c) || !g || !u) return PD_ERR_INVALID;
  if (prec != PD_FP64 && prec != PD_FP32_IR && prec != PD_BF16_IR)
    return c->fail(PD_ERR_INVALID, "unknown precision mode %d", (int)prec);
  if (c->broken) return PD_ERR_HIP;
  const int m = (int)c->m;
  if (prec == PD_FP64) {
    bool fused = false;
    if (c->stale) {
      build_H(c);
      zero_int(c->d_info, c->st);
      fused = true;
      if (fused) rhs_pack(m, g, m, c->d_Yt, c->st);
      PhaseTimer tm(c, PD_PHASE_FACTOR);
      cholesky(c, c->d_H, c->ldH, m, fused ? c->d_Yt : nullptr);
      c->stale = false;
      c->lp_stale = true;       // d_H was rebuilt
    }
    {
      PhaseTimer tmsolve(c, PD_PHASE_SOLVE);
      if (fused) {
        // the forward substitution ran inside the factorization
        rhs_unpack(m, c->d_Yt, c->d_ys, m, c->st);
        sentinel_fill(3 * m, u, c->st);     // the backward solve publishes u by value
      } else if (c->overlap) {
        // the factorization may still run on another stream: the forward
        // solve follows its tile flags, the backward one waits for its end
        HIPCK(c, hipStreamWaitEvent(c->st, c->ev_fstart, 0));
        trsv3_forward(c->d_H, c->ldH, m, c->d_linv, g, m, c->d_ys, m, c->d_ticket, c->d_err, u, m,
                      c->st, c->d_tflags, c->d_tticket);
        HIPCK(c, hipStreamWaitEvent(c->st, c->ev_fdone, 0));
        c->overlap = false;
      } else {
        trsv3_forward(c->d_H, c->ldH, m, c->d_linv, g, m, c->d_ys, m, c->d_ticket, c->d_err, u, m,
                      c->st);
      }
      trsv3_backward(c->d_H, c->ldH, m, c->d_linv, c->d_ys, m, u, m, c->d_ticket + 1, c->d_err,
                     c->st);
    }
    CK(c->check("pd_global_solve"));
    if (info) {
      double rr = 0.0;
      CK(residual(c, g, u, &rr));
      int hinfo = 0, herr = 0;
      HIPCK(c, hipMemcpy(&hinfo, c->d_info, sizeof(int), hipMemcpyDeviceToHost));
      HIPCK(c, hipMemcpy(&herr, c->d_err, sizeof(int), hipMemcpyDeviceToHost));
      info->ir_iters = 0;
      info->bad_pivot = hinfo;
      info->fell_back = 0;
      info->reserved = 0;
      info->rel_residual = rr;
      if (herr) return c->fail(PD_ERR_HIP, "dependency wait timed out");
      if (hinfo) return c->fail(PD_ERR_NOT_SPD, "non-positive pivot at %d", hinfo);
    }
    return PD_OK;
  }
  // ---- low-precision factor + iterative refinement with an FP64 residual
  CK(ensure_lp_buffers(c));
  if (c->lp_stale || c->lp_prec != (int)prec) {
    build_H(c);
    c->stale = true;            // d_H no longer holds an FP64 factor
    zero_int(c->d_info, c->st);
    PhaseTimer tm(c, PD_PHASE_FACTOR);
    equilibrate_convert(c->d_H, c->ldH, m, c->d_dvec, c->d_H32, c->ldH32, c->st);
    potrf_dataflow_lp(c->d_H32, c->ldH32, m, c->d_linv32, reinterpret_cast<float*>(c->d_sbuf),
                      c->d_tflags, c->d_tticket, c->d_info, c->d_err, c->n_wg, prec == PD_BF16_IR,
                      c->st, c->d_cumarks);
    c->lp_stale = false;
    c->lp_prec = (int)prec;
    c->lp_info = -1;
  }
  int hinfo = 0, herr = 0;
  double rr = 0.0;
  int it = 0;
  {
    PhaseTimer tmsolve(c, PD_PHASE_SOLVE);
    // a non-positive pivot of the low-precision factor leaves no usable
    // preconditioner: check it before iterating
    if (c->lp_info < 0) {
      HIPCK(c, hipMemcpyAsync(&c->lp_info, c->d_info, sizeof(int), hipMemcpyDeviceToHost, c->st));
      HIPCK(c, hipMemcpyAsync(&herr, c->d_err, sizeof(int), hipMemcpyDeviceToHost, c->st));
      HIPCK(c, hipStreamSynchronize(c->st));
    }
    hinfo = c->lp_info;
    if (!hinfo && !herr) {
      lp_precondition(c, g, u);
      CK(c->check("pd_global_solve"));
      CK(refine_pcg(c, g, u, &rr, &it));
      HIPCK(c, hipMemcpy(&herr, c->d_err, sizeof(int), hipMemcpyDeviceToHost));
    }
  }
  if (herr) return c->fail(PD_ERR_HIP, "dependency wait timed out");
  const bool stalled = hinfo != 0 || !(rr <= c->ir_tol);
  if (stalled && c->ir_fallback) {
    // FP64 factor and solve of the same H
    build_H(c);
    zero_int(c->d_info, c->st);
    {
      PhaseTimer tm(c, PD_PHASE_FACTOR);
      cholesky(c, c->d_H, c->ldH, m, nullptr);
    }
    c->stale = false;
    {
      PhaseTimer tmsolve(c, PD_PHASE_SOLVE);
      trsv3_forward(c->d_H, c->ldH, m, c->d_linv, g, m, c->d_ys, m, c->d_ticket, c->d_err, u, m,
                    c->st);
      trsv3_backward(c->d_H, c->ldH, m, c->d_linv, c->d_ys, m, u, m, c->d_ticket + 1, c->d_err,
                     c->st);
    }
    CK(c->check("pd_global_solve"));
    CK(residual(c, g, u, &rr));
    int finfo = 0;
    HIPCK(c, hipMemcpy(&finfo, c->d_info, sizeof(int), hipMemcpyDeviceToHost));
    HIPCK(c, hipMemcpy(&herr, c->d_err, sizeof(int), hipMemcpyDeviceToHost));
    if (info) {
      info->ir_iters = it;
      info->bad_pivot = finfo;
      info->fell_back = 1;
      info->reserved = 0;
      info->rel_residual = rr;
    }
    if (herr) return c->fail(PD_ERR_HIP, "dependency wait timed out");
    if (finfo) return c->fail(PD_ERR_NOT_SPD, "non-positive pivot at %d", finfo);
    return PD_OK;
  }
  if (info) {
    info->ir_iters = it;
    info->bad_pivot = hinfo;
    info->fell_back = 0;
    info->reserved = 0;
    info->rel_residual = rr;
  }
  if (hinfo) return c->fail(PD_ERR_NOT_SPD, "non-positive pivot at %d", hinfo);
  if (!(rr <= c->ir_tol))
    return c->fail(PD_ERR_IR_STALLED, "refinement reached %.3e after %d steps", rr, it);
  return PD_OK;
}

pd_status pd_set_refinement(pd_ctx* c, int32_t max_steps, double tol, int32_t fallback) {
  if (bad_ctx(c)) return PD_ERR_INVALID;
  if (max_steps < 0 || max_steps > 100000 || !(tol > 0.0) || !std::isfinite(tol) ||
      (fallback != 0 && fallback != 1))
    return c->fail(PD_ERR_INVALID, "bad refinement settings (%d, %g, %d)", max_steps, tol,
                   fallback);
  c->max_ir = max_steps;
  c->ir_tol = tol;
  c->ir_fallback = fallback;
  return PD_OK;
}

pd_status pd_factor(pd_ctx* c, int32_t n_workgroups, int32_t overlap_forward) {
  if (bad_ctx(c)) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  if (overlap_forward != 0 && overlap_forward != 1)
    return c->fail(PD_ERR_INVALID, "overlap_forward must be 0 or 1 (got %d)", (int)overlap_forward);
  if (!c->stale) return PD_OK;
  const bool overlap = overlap_forward == 1;
  if (overlap && !c->ev_fstart) {
    HIPCK(c, hipEventCreateWithFlags(&c->ev_fstart, hipEventDisableTiming));
    HIPCK(c, hipEventCreateWithFlags(&c->ev_fdone, hipEventDisableTiming));
  }
  build_H(c);
  zero_int(c->d_info, c->st);
  {
    PhaseTimer tm(c, PD_PHASE_FACTOR);
    cholesky(c, c->d_H, c->ldH, (int)c->m, nullptr, n_workgroups,
             overlap ? c->ev_fstart : nullptr);
  }
  if (overlap) HIPCK(c, hipEventRecord(c->ev_fdone, c->st));
  c->overlap = overlap;
  c->stale = false;
  c->lp_stale = true;             // d_H was rebuilt
  return c->check("pd_factor");
}

pd_status pd_inner_update(pd_ctx* c, const double* u2, double* x2, double* delta2, double* ft) {
  if (bad_ctx(c) || !u2 || !x2 || !delta2 || !ft) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  const int m = (int)c->m;
  PhaseTimer tm(c, PD_PHASE_INNER_UPDATE);
  inner_update(m, u2, x2, delta2, c->st);
  sweep_symv(c->d_S, m, m, u2, m, c->d_P, c->st);            // lower tiles of S only
  sweep_assemble(m, c->d_P, ft, m, ft, m, c->st);            // ft -= S u2
  if (c->nbeta > 0) csr_spmv3(m, c->d_Abptr, c->d_Abcol, c->d_Abval, u2, m, 1.0, ft, m, ft, m, c->st);
  return c->check("pd_inner_update");
}

pd_status pd_warmstart_input(pd_ctx* c, const double* x2, const double* x2_prev, float scale,
                             int32_t n_prox, const int32_t* prox, const double* cpen, float* out) {
  if (bad_ctx(c) || !x2 || !x2_prev || !out || n_prox < 0 || (n_prox > 0 && (!prox || !cpen)))
    return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  ws_input((int)c->m, x2, x2_prev, scale, n_prox, prox, cpen, out, c->st);
  return c->check("pd_warmstart_input");
}

pd_status pd_warmstart_target(pd_ctx* c, const double* x2, const double* x2_prev1,
                              const double* x2_prev2, float scale, float* out) {
  if (bad_ctx(c) || !x2 || !x2_prev1 || !x2_prev2 || !out) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  ws_target(3 * c->m, x2, x2_prev1, x2_prev2, scale, out, c->st);
  return c->check("pd_warmstart_target");
}

pd_status pd_region_add_f32(pd_ctx* c, const float* d2, double scale, double* x) {
  if (bad_ctx(c) || !d2 || !x) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  region_add_f32(c->m, c->d_region_ids, d2, scale, x, c->n, c->st);
  return c->check("pd_region_add_f32");
}

pd_status pd_displacement_change(pd_ctx* c, const double* x, const double* x_prev, double* out) {
  if (bad_ctx(c) || !x || !x_prev || !out) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  change_norms(c->n_free, c->d_free_ids, x, x_prev, c->d_rest, c->n, c->d_norms, c->st);
  double h[2];
  HIPCK(c, hipMemcpyAsync(h, c->d_norms, 2 * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCK(c, hipStreamSynchronize(c->st));
  out[0] = std::sqrt(h[0]);
  out[1] = std::sqrt(h[1]);
  return PD_OK;
}

pd_status pd_set_stream(pd_ctx* c, void* hip_stream) {
  if (bad_ctx(c)) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  HIPCK(c, hipStreamSynchronize(c->st));
  c->st = (hipStream_t)hip_stream;
  return PD_OK;
}

pd_status pd_use_stream(pd_ctx* c, void* hip_stream) {
  if (bad_ctx(c)) return PD_ERR_INVALID;
  if (c->broken) return PD_ERR_HIP;
  c->st = (hipStream_t)hip_stream;
  return PD_OK;
}

pd_status pd_set_timing(pd_ctx* c, int on) {
  if (bad_ctx(c)) return PD_ERR_INVALID;
  c->timing = on != 0;
  return PD_OK;
}

pd_status pd_get_timings(pd_ctx* c, double* ms, int64_t* counts) {
  if (bad_ctx(c) || !ms) return PD_ERR_INVALID;
  HIPCK(c, hipStreamSynchronize(c->st));
  for (int p = 0; p < PD_N_PHASES; ++p) {
    ms[p] = 0.0;
    if (counts) counts[p] = 0;
  }
  for (auto& pr : c->ev_pairs) {
    float t = 0.f;
    // the pair may have been recorded on another stream (pd_use_stream)
    HIPCK(c, hipEventSynchronize(c->ev_pool[pr.second.second]));
    HIPCK(c, hipEventElapsedTime(&t, c->ev_pool[pr.second.first], c->ev_pool[pr.second.second]));
    ms[pr.first] += t;
    if (counts) counts[pr.first] += 1;
  }
  c->ev_pairs.clear();
  c->ev_used = 0;
  return PD_OK;
}

const char* pd_last_error(const pd_ctx* c) {
  if (!c) return g_build_error.c_str();
  return c->err.c_str();
}

pd_status pd_destroy(pd_ctx* c) {
  if (!c) return PD_ERR_INVALID;
  (void)hipStreamSynchronize(c->st);
  delete c;
  return PD_OK;
}

}  // extern "C"
