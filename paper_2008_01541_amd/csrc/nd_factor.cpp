// Nested-dissection supernodal factor of the interior block A11 (Sec. 4.3:
// the partial factorization that leaves the Schur complement of the region,
// here on the GPU in place of a sparse direct solver).  The interior nodes
// are ordered by geometric nested dissection (recursive coordinate bisection
// with vertex separators taken from the graph of the mesh); every leaf part
// and every separator is a supernode, eliminated children first.  Supernode s
// (n_s nodes, boundary B_s of b_s later nodes) is factored as a dense front
//   [F_ss  .  ]   L_ss = chol(F_ss), Z_s = L_ss^-T L_ss^-1 = F_ss^-1,
//   [F_Bs F_BB]   W_s = F_Bs Z_s, U_s = F_BB - W_s F_Bs^T (into the parent),
// and the roots' updates land in S = K22 - K21 K11^-1 K12.  Z_s and W_s stay
// on the device for the two sweeps of every outer iteration, which run one
// tree height at a time, each height one batch of matrix-vector products
// (no triangular solves): the forward sweep gathers r_s = f_s minus the
// contributions of its descendants and hands W_s r_s to its boundary (the
// region's share gives y2 = f2 - A21 A11^-1 f1); the backward sweep forms
// x_s = Z_s r_s - W_s^T zb_s from the solution zb_s already known on the
// boundary (delta2 on the region), which is A11^-1 (f1 - A12 delta2) on s.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "ctx.h"

using namespace pdk;

namespace {

inline int64_t pad16(int64_t v) { return (v + 15) / 16 * 16; }
// columns of at most this many rows are taken four per wave in the sweeps
// (slab: 0.287 + 0.334 ms with one column per wave, 0.259 + 0.309 ms with
// this bound; 512 and 2,048 are within 2 %)
constexpr int32_t kShortColumn = 1024;

// Recursive coordinate bisection of a set of interior nodes.  A part larger
// than the leaf size is sorted along the longest side of its bounding box of
// rest positions and cut at the change of coordinate nearest to its median;
// the nodes of one side that have a graph neighbour on the other side form
// the separator (the smaller of the two one-sided choices).  Removing it
// leaves two halves with no edge between them, which are bisected in turn;
// a leaf part becomes one supernode per connected component.  Supernodes are created children first, so their creation order is an
// elimination order (every child before its parent).
struct Dissector {
  const double* rest;
  int64_t n;
  const std::vector<int8_t>& cls;
  const std::vector<int64_t>& adj_ptr;
  const std::vector<int32_t>& adj;
  int leaf;
  std::vector<int32_t> stamp, side;
  int32_t tag = 0;
  std::vector<std::vector<int32_t>> nodes;   // per supernode, ascending ids
  std::vector<int32_t> parent;

  Dissector(const double* r, int64_t nn, const std::vector<int8_t>& c,
            const std::vector<int64_t>& ap, const std::vector<int32_t>& a, int lf)
      : rest(r), n(nn), cls(c), adj_ptr(ap), adj(a), leaf(lf), stamp(nn, 0), side(nn, 0) {}

  int32_t make(std::vector<int32_t> v, const std::vector<int32_t>& children) {
    std::sort(v.begin(), v.end());
    nodes.push_back(std::move(v));
    parent.push_back(-1);
    const int32_t id = (int32_t)nodes.size() - 1;
    for (int32_t ch : children) parent[ch] = id;
    return id;
  }

  // One supernode per connected component of a leaf part (a disconnected
  // front would carry zero blocks between its pieces).
  std::vector<int32_t> leaves(std::vector<int32_t> part) {
    const int32_t tg = ++tag;
    for (int32_t v : part) stamp[v] = tg;
    std::vector<int32_t> roots, comp;
    for (int32_t v0 : part) {
      if (stamp[v0] != tg) continue;
      comp.assign(1, v0);
      stamp[v0] = -tg;
      for (size_t q = 0; q < comp.size(); ++q)
        for (int64_t e = adj_ptr[comp[q]]; e < adj_ptr[comp[q] + 1]; ++e)
          if (stamp[adj[e]] == tg) {
            stamp[adj[e]] = -tg;
            comp.push_back(adj[e]);
          }
      roots.push_back(make(comp, {}));
    }
    return roots;
  }

  // Supernodes of the part; returns the roots of its subtrees.
  std::vector<int32_t> run(std::vector<int32_t> part) {
    if (part.empty()) return {};
    if ((int64_t)part.size() <= leaf) return leaves(std::move(part));
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = hi[d] = rest[d * n + part[0]];
      for (int32_t v : part) {
        lo[d] = std::min(lo[d], rest[d * n + v]);
        hi[d] = std::max(hi[d], rest[d * n + v]);
      }
    }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
      if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
    if (!(hi[ax] > lo[ax])) return leaves(std::move(part));   // all at one point
    const double* x = rest + ax * n;
    std::sort(part.begin(), part.end(), [&](int32_t a, int32_t b) {
      return x[a] != x[b] ? x[a] < x[b] : a < b;
    });
    // cut k: [0, k) | [k, size) with x[part[k-1]] < x[part[k]], nearest to the middle
    const int64_t sz = (int64_t)part.size(), mid = sz / 2;
    int64_t cut = -1;
    for (int64_t d = 0; cut < 0 && d < sz; ++d) {
      for (int64_t k : {mid - d, mid + d})
        if (k >= 1 && k < sz && x[part[k - 1]] < x[part[k]]) {
          cut = k;
          break;
        }
    }
    if (cut < 0) return leaves(std::move(part));
    const int32_t tg = ++tag;
    for (int64_t k = 0; k < sz; ++k) {
      stamp[part[k]] = tg;
      side[part[k]] = k < cut ? 0 : 1;
    }
    std::vector<int32_t> sep[2], keep[2];
    for (int64_t k = 0; k < sz; ++k) {
      const int32_t v = part[k];
      const int sd = side[v];
      bool touches = false;
      for (int64_t e = adj_ptr[v]; e < adj_ptr[v + 1] && !touches; ++e) {
        const int32_t w = adj[e];
        touches = stamp[w] == tg && side[w] != sd;
      }
      if (touches) sep[sd].push_back(v);
    }
    const int sd = sep[0].size() <= sep[1].size() ? 0 : 1;
    for (int32_t v : sep[sd]) stamp[v] = -tg;   // separator nodes leave the halves
    for (int64_t k = 0; k < sz; ++k) {
      const int32_t v = part[k];
      if (stamp[v] != -tg) keep[side[v]].push_back(v);
    }
    std::vector<int32_t> s = std::move(sep[sd]);
    part.clear();
    part.shrink_to_fit();
    std::vector<int32_t> roots = run(std::move(keep[0]));
    std::vector<int32_t> rb = run(std::move(keep[1]));
    roots.insert(roots.end(), rb.begin(), rb.end());
    if (s.empty()) return roots;
    return {make(std::move(s), roots)};
  }
};

}  // namespace

pd_status nd_analyse(int64_t n, const double* rest, const std::vector<int8_t>& cls,
                     const std::vector<int32_t>& rloc, const std::vector<int64_t>& adj_ptr,
                     const std::vector<int32_t>& adj, int leaf, NdSymbolic& S, std::string& err) {
  S = NdSymbolic();
  std::vector<int32_t> interior;
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (cls[i] == 1) interior.push_back((int32_t)i);
    if (cls[i] == 2) ++m;
  }
  const int64_t n1 = (int64_t)interior.size();
  S.n1 = (int32_t)n1;
  S.m = (int32_t)m;
  Dissector D(rest, n, cls, adj_ptr, adj, leaf);
  D.run(std::move(interior));
  const int64_t ns = (int64_t)D.nodes.size();
  S.first.assign(ns + 1, 0);
  S.elim.reserve(n1);
  std::vector<int32_t> pos(n, -1), sn_at(std::max<int64_t>(n1, 1), -1);
  for (int64_t s = 0; s < ns; ++s) {
    for (int32_t v : D.nodes[s]) {
      pos[v] = (int32_t)S.elim.size();
      sn_at[S.elim.size()] = (int32_t)s;
      S.elim.push_back(v);
    }
    S.first[s + 1] = (int32_t)S.elim.size();
  }
  // Boundary sets: later neighbours of the supernode's own nodes, and what
  // its children's boundaries hold beyond the supernode itself.  The parent
  // of a supernode is the one that holds the first key of its boundary (the
  // elimination tree; a part of the bisection that does not touch the
  // separator above it hangs below a higher separator), -1 when the boundary
  // is empty or lies in x2.
  S.parent.assign(ns, -1);
  S.bptr.assign(ns + 1, 0);
  S.height.assign(ns, 0);
  std::vector<std::vector<int32_t>> children(ns);
  std::vector<int32_t> mark(n1 + m, -1), keys;
  for (int64_t s = 0; s < ns; ++s) {
    const int32_t f0 = S.first[s], f1 = S.first[s + 1];
    keys.clear();
    auto add = [&](int32_t k) {
      if (mark[k] != (int32_t)s) {
        mark[k] = (int32_t)s;
        keys.push_back(k);
      }
    };
    for (int32_t p = f0; p < f1; ++p) {
      const int32_t u = S.elim[p];
      for (int64_t e = adj_ptr[u]; e < adj_ptr[u + 1]; ++e) {
        const int32_t w = adj[e];
        if (cls[w] == 2) add((int32_t)(n1 + rloc[w]));
        else if (cls[w] == 1 && pos[w] >= f1) add(pos[w]);
      }
    }
    for (int32_t ch : children[s]) {
      S.height[s] = std::max(S.height[s], S.height[ch] + 1);
      for (int64_t e = S.bptr[ch]; e < S.bptr[ch + 1]; ++e) {
        const int32_t k = S.bkey[e];
        if (k >= f0 && k < f1) continue;
        add(k);
      }
    }
    std::sort(keys.begin(), keys.end());
    // every interior key must lie in a separator above s in the bisection
    // (walked up in increasing position)
    int32_t a = D.parent[s];
    for (int32_t k : keys) {
      if (k >= n1) break;
      while (a >= 0 && S.first[a + 1] <= k) a = D.parent[a];
      if (a < 0 || k < S.first[a]) {
        err = "internal: nested-dissection boundary outside the ancestors of a supernode";
        return PD_ERR_INVALID;
      }
    }
    S.bkey.insert(S.bkey.end(), keys.begin(), keys.end());
    S.bptr[s + 1] = (int64_t)S.bkey.size();
    if (S.bkey.size() > (size_t)INT32_MAX) {
      err = "nested-dissection boundary too large";
      return PD_ERR_INVALID;
    }
    if (!keys.empty() && keys[0] < n1) {
      S.parent[s] = sn_at[keys[0]];
      children[S.parent[s]].push_back((int32_t)s);
    }
  }
  return PD_OK;
}

// Device data of the nested-dissection factor.
struct NdFactor {
  NdSymbolic sym;
  int64_t nb = 0;
  // in fac (doubles): [Z_s; W_s] ((n_s + b_s) x n_s, leading dimension
  // ldzw) and W_s^T (n_s x b_s, leading dimension ldwt)
  std::vector<int64_t> zwoff, wtoff;
  std::vector<int32_t> ldzw, ldwt;
  struct Level {                          // one tree height: ranges in tlist / items / elist
    int32_t t_off, t_cnt, fw_off, fw_cnt, bw_off, bw_cnt, e_off, e_cnt;
  };
  std::vector<Level> levels;
  int32_t treg_off = 0;                   // region targets in tlist
  int64_t fac_doubles = 0;
  double* d_fac = nullptr;
  int32_t *d_node_of = nullptr, *d_cpos = nullptr;
  NdTarget* d_trec = nullptr;             // targets of the right-hand-side gathers, tlist order
  NdEntry* d_erec = nullptr;              // entries of the boundary gathers, elist order
  NdItem* d_items = nullptr;
  double *d_r = nullptr, *d_x1 = nullptr, *d_contrib = nullptr, *d_zb = nullptr;
};

void nd_free(NdFactor* f) { delete f; }   // device memory belongs to the context

pd_status nd_prepare(pd_ctx* c, const double* rest, const std::vector<int8_t>& cls,
                     const std::vector<int32_t>& rloc, const std::vector<int64_t>& adj_ptr,
                     const std::vector<int32_t>& adj, int leaf) {
  NdFactor* F = new NdFactor();
  c->nd = F;
  std::string err;
  pd_status s = nd_analyse(c->n, rest, cls, rloc, adj_ptr, adj, leaf, F->sym, err);
  if (s != PD_OK) return c->fail(s, "%s", err.c_str());
  const NdSymbolic& S = F->sym;
  F->nb = (int64_t)S.bkey.size();
  c->n1 = S.n1;
  c->maxw = 0;
  for (size_t k = 0; k + 1 < S.first.size(); ++k)
    c->maxw = std::max<int64_t>(c->maxw, S.first[k + 1] - S.first[k]);
  for (size_t k = 0; k + 1 < S.bptr.size(); ++k)
    if (S.first[k + 1] - S.first[k] + (S.bptr[k + 1] - S.bptr[k]) > 46340)
      return c->fail(PD_ERR_INVALID, "nested-dissection front too large");
  return PD_OK;
}

int nd_height(const pd_ctx* c) {
  return c->nd ? (int)c->nd->levels.size() : 0;
}

pd_status nd_factor(pd_ctx* c, const int32_t* tets, int64_t T, const std::vector<int8_t>& cls,
                    const std::vector<int32_t>& rloc, const double* d_Ke) {
  NdFactor* F = c->nd;
  const NdSymbolic& S = F->sym;
  const int64_t n1 = S.n1, m = S.m, ns = (int64_t)S.parent.size(), nb = F->nb;
  std::vector<int32_t> pos(c->n, -1), sn_of(std::max<int64_t>(n1, 1), -1);
  for (int64_t s = 0; s < ns; ++s)
    for (int32_t p = S.first[s]; p < S.first[s + 1]; ++p) {
      pos[S.elim[p]] = p;
      sn_of[p] = (int32_t)s;
    }
  auto nsz = [&](int64_t s) { return (int64_t)(S.first[s + 1] - S.first[s]); };
  auto bsz = [&](int64_t s) { return S.bptr[s + 1] - S.bptr[s]; };
  auto key_of = [&](int32_t u) -> int32_t { return cls[u] == 2 ? (int32_t)(n1 + rloc[u]) : pos[u]; };
  // index of key k in the front of s: own nodes first, then the boundary
  auto front_index = [&](int64_t s, int32_t k) -> int64_t {
    if (k >= S.first[s] && k < S.first[s + 1]) return k - S.first[s];
    const int32_t* b = S.bkey.data() + S.bptr[s];
    const int32_t* e = S.bkey.data() + S.bptr[s + 1];
    const int32_t* it = std::lower_bound(b, e, k);
    return (it != e && *it == k) ? nsz(s) + (it - b) : -1;
  };

  // layouts: fronts P_s (ld pad16(n_s + b_s), n_s columns), updates U_s
  // (pad16(b_s) x b_s), the kept blocks [Z_s; W_s] (ld pad16(n_s + b_s), n_s
  // columns) and W_s^T (pad16(n_s) x b_s), and the work blocks of the inverse
  // (pad16(n_s) x n_s); all offsets multiples of 16 doubles
  std::vector<int64_t> poff(ns), ldp(ns), uoff(ns), ldu(ns);
  F->zwoff.assign(ns, 0);
  F->wtoff.assign(ns, 0);
  F->ldzw.assign(ns, 0);
  F->ldwt.assign(ns, 0);
  int64_t ptot = 0, utot = 0, mmax = 0;
  F->fac_doubles = 0;
  for (int64_t s = 0; s < ns; ++s) {
    const int64_t a = nsz(s), b = bsz(s);
    ldp[s] = pad16(a + b);
    poff[s] = ptot;
    ptot += ldp[s] * a;
    ldu[s] = pad16(b);
    uoff[s] = utot;
    utot += ldu[s] * b;
    F->ldzw[s] = (int32_t)pad16(a + b);
    F->ldwt[s] = (int32_t)pad16(a);
    F->zwoff[s] = F->fac_doubles;
    F->fac_doubles += (int64_t)F->ldzw[s] * a;
    F->wtoff[s] = F->fac_doubles;
    F->fac_doubles += (int64_t)F->ldwt[s] * b;
    mmax = std::max(mmax, pad16(a) * a);
  }
  double *d_P = nullptr, *d_U = nullptr, *d_M = nullptr, *d_X = nullptr;
  int32_t* d_fmap = nullptr;
  CK(c->alloc(&F->d_fac, F->fac_doubles));
  CK(c->alloc(&d_P, ptot));
  CK(c->alloc(&d_U, utot));
  CK(c->alloc(&d_M, mmax));
  CK(c->alloc(&d_X, mmax));
  HIPCK(c, hipMemsetAsync(d_P, 0, std::max<int64_t>(ptot, 1) * sizeof(double), c->st));
  HIPCK(c, hipMemsetAsync(d_U, 0, std::max<int64_t>(utot, 1) * sizeof(double), c->st));
  HIPCK(c, hipMemsetAsync(F->d_fac, 0, std::max<int64_t>(F->fac_doubles, 1) * sizeof(double),
                          c->st));

  // assembly of the original entries: K(u, v) with v interior goes to the
  // front of v's supernode when u is v's supernode or later (row u of the
  // front, column v); region-region entries go to S.  Each destination sums
  // its element contributions in increasing element-matrix order.
  {
    std::vector<std::pair<int64_t, int64_t>> ep, es;   // (destination, source)
    ep.reserve((size_t)T * 10);
    for (int64_t e = 0; e < T; ++e)
      for (int a = 0; a < 4; ++a) {
        const int32_t u = tets[a * T + e];
        if (cls[u] == 0) continue;
        for (int b = 0; b < 4; ++b) {
          const int32_t v = tets[b * T + e];
          if (cls[v] == 0) continue;
          const int64_t src = (int64_t)(a * 4 + b) * T + e;
          if (cls[v] == 2) {
            if (cls[u] == 2) es.emplace_back((int64_t)rloc[u] + (int64_t)rloc[v] * m, src);
            continue;
          }
          const int64_t s = sn_of[pos[v]];
          if (cls[u] == 1 && pos[u] < S.first[s]) continue;
          const int64_t i = front_index(s, key_of(u));
          if (i < 0) return c->fail(PD_ERR_INVALID, "internal: entry outside its front");
          ep.emplace_back(poff[s] + i + (pos[v] - S.first[s]) * ldp[s], src);
        }
      }
    for (auto* V : {&ep, &es}) {
      std::sort(V->begin(), V->end());
      Plan pl;
      for (size_t i = 0; i < V->size();) {
        size_t j = i;
        std::vector<int64_t> srcs;
        while (j < V->size() && (*V)[j].first == (*V)[i].first) srcs.push_back((*V)[j++].second);
        pl.add_group(srcs.data(), (int64_t)srcs.size(), (*V)[i].first);
        i = j;
      }
      CK(run_plan(c, pl, d_Ke, V == &ep ? d_P : c->d_S));
    }
  }
  if (c->dt > 0.0) {
    // inertia diagonal on the diagonals of the fronts and of S
    std::vector<int64_t> op, os;
    std::vector<double> vp, vs;
    for (int64_t u = 0; u < c->n; ++u) {
      if (cls[u] == 2) {
        os.push_back((int64_t)rloc[u] * (m + 1));
        vs.push_back(c->h_D[u]);
      } else if (cls[u] == 1) {
        const int64_t s = sn_of[pos[u]], j = pos[u] - S.first[s];
        op.push_back(poff[s] + j * (ldp[s] + 1));
        vp.push_back(c->h_D[u]);
      }
    }
    int64_t *d_op = nullptr, *d_os = nullptr;
    double *d_vp = nullptr, *d_vs = nullptr;
    CK(c->upload(&d_op, op));
    CK(c->upload(&d_vp, vp));
    CK(c->upload(&d_os, os));
    CK(c->upload(&d_vs, vs));
    add_at((int64_t)op.size(), d_op, d_vp, d_P, c->st);
    add_at((int64_t)os.size(), d_os, d_vs, c->d_S, c->st);
    CK(c->check("inertia diagonal"));
    HIPCK(c, hipStreamSynchronize(c->st));
    for (void* p : {(void*)d_op, (void*)d_vp, (void*)d_os, (void*)d_vs}) free_now(c, p);
  }

  // where each boundary entry lands in the parent's front (roots: in S)
  {
    std::vector<int32_t> fmap(std::max<int64_t>(nb, 1), 0);
    for (int64_t s = 0; s < ns; ++s) {
      const int32_t p = S.parent[s];
      for (int64_t e = S.bptr[s]; e < S.bptr[s + 1]; ++e) {
        const int32_t k = S.bkey[e];
        int64_t idx;
        if (p < 0) idx = k >= n1 ? k - n1 : -1;
        else idx = front_index(p, k);
        if (idx < 0) return c->fail(PD_ERR_INVALID, "internal: boundary outside the parent front");
        fmap[e] = (int32_t)idx;
      }
    }
    CK(c->upload(&d_fmap, fmap));
  }

  // numeric factorization, children first
  std::vector<std::vector<int32_t>> children(ns);
  for (int64_t s = 0; s < ns; ++s)
    if (S.parent[s] >= 0) children[S.parent[s]].push_back((int32_t)s);
  // per supernode: L_ss = chol(F_ss), X = L_ss^-1, Z = X^T X = A_ss^-1,
  // W = F_Bs Z, U -= W F_Bs^T (= L_Bs L_Bs^T), W^T for the forward sweep
  for (int64_t s = 0; s < ns; ++s) {
    const int a = (int)nsz(s), b = (int)bsz(s);
    const int ldx = (int)pad16(a), lzw = F->ldzw[s];
    double* P = d_P + poff[s];
    double* U = d_U + uoff[s];
    double* ZW = F->d_fac + F->zwoff[s];
    for (int32_t ch : children[s])
      nd_extend_add(d_U + uoff[ch], ldu[ch], (int)bsz(ch), d_fmap + S.bptr[ch], a, P, ldp[s], U,
                    ldu[s], 0, c->st);
    potrf_dataflow(P, (int)ldp[s], a, c->d_linv, c->d_sbuf, c->d_tflags, c->d_tticket, c->d_info,
                   c->d_err, c->n_wg, nullptr, c->st, c->d_cumarks, nullptr);
    trtri_from_factor(P, (int)ldp[s], a, c->d_linv, d_M, d_X, ldx, c->st);
    lauum_full(d_X, ldx, a, ZW, lzw, c->st);
    if (b > 0) {
      gemm_nt(P + a, ldp[s], ZW, lzw, ZW + a, lzw, b, a, a, 1.0, 0.0, 0, 0, c->st);
      gemm_nt(ZW + a, lzw, P + a, ldp[s], U, ldu[s], b, b, a, -1.0, 1.0, 1, 0, c->st);
      nd_transpose(ZW + a, lzw, b, a, F->d_fac + F->wtoff[s], F->ldwt[s], c->st);
      if (S.parent[s] < 0)
        nd_extend_add(U, ldu[s], b, d_fmap + S.bptr[s], 0, nullptr, 0, c->d_S, m, 1, c->st);
    }
    CK(c->check("nested-dissection factorization"));
  }
  HIPCK(c, hipStreamSynchronize(c->st));
  free_now(c, d_P);
  free_now(c, d_U);
  free_now(c, d_M);
  free_now(c, d_X);
  free_now(c, d_fmap);
  {
    int info = 0;
    HIPCK(c, hipMemcpy(&info, c->d_info, sizeof(int), hipMemcpyDeviceToHost));
    if (info != 0)
      return c->fail(PD_ERR_NOT_SPD, "interior supernode not positive definite (pivot %d)", info);
  }

  // sweep structures: node of every target, the contributions of every
  // target (boundary entries in increasing order, stored target-major by the
  // forward products: cpos[e] is entry e's position), the per-height lists
  {
    std::vector<int32_t> node_of(S.elim);
    node_of.insert(node_of.end(), c->region_ids.begin(), c->region_ids.end());
    std::vector<int32_t> cptr(n1 + m + 1, 0), cslot(std::max<int64_t>(nb, 1), 0);
    for (int64_t e = 0; e < nb; ++e) cptr[S.bkey[e] + 1]++;
    for (int64_t t = 0; t < n1 + m; ++t) cptr[t + 1] += cptr[t];
    {
      std::vector<int32_t> cur(cptr.begin(), cptr.end() - 1);
      for (int64_t e = 0; e < nb; ++e) cslot[cur[S.bkey[e]]++] = (int32_t)e;
    }
    int H = 0;
    for (int64_t s = 0; s < ns; ++s) H = std::max(H, S.height[s] + 1);
    std::vector<std::vector<int32_t>> at(H);
    for (int64_t s = 0; s < ns; ++s) at[S.height[s]].push_back((int32_t)s);
    std::vector<int32_t> tlist, elist;
    std::vector<NdItem> items;
    F->levels.assign(H, NdFactor::Level{});
    for (int h = 0; h < H; ++h) {
      NdFactor::Level& L = F->levels[h];
      L.t_off = (int32_t)tlist.size();
      L.e_off = (int32_t)elist.size();
      for (int32_t s : at[h]) {
        for (int32_t p = S.first[s]; p < S.first[s + 1]; ++p) tlist.push_back(p);
        for (int64_t e = S.bptr[s]; e < S.bptr[s + 1]; ++e) elist.push_back((int32_t)e);
      }
      L.t_cnt = (int32_t)tlist.size() - L.t_off;
      L.e_cnt = (int32_t)elist.size() - L.e_off;
      // four columns per item: the forward sweep's W_s r_s (columns of
      // W_s^T), the backward sweep's Z_s r_s - W_s^T zb_s (columns of [Z_s; W_s])
      // (four per wave when the columns are short: their vector loads are
      // then shared and the waves fewer)
      L.fw_off = (int32_t)items.size();
      for (int32_t s : at[h]) {
        const int32_t a = (int32_t)nsz(s), b = (int32_t)bsz(s);
        const int32_t f0 = S.first[s], b0 = (int32_t)S.bptr[s];
        const int32_t cpw = a <= kShortColumn ? 4 : 1;
        for (int32_t q = 0; q < b; q += 4 * cpw)
          items.push_back({F->wtoff[s], F->ldwt[s], a, b, q, f0, b0, a, 0, cpw});
      }
      L.fw_cnt = (int32_t)items.size() - L.fw_off;
      L.bw_off = (int32_t)items.size();
      for (int32_t s : at[h]) {
        const int32_t a = (int32_t)nsz(s), b = (int32_t)bsz(s);
        const int32_t f0 = S.first[s], b0 = (int32_t)S.bptr[s];
        const int32_t cpw = a + b <= kShortColumn ? 4 : 1;
        for (int32_t q = 0; q < a; q += 4 * cpw)
          items.push_back({F->zwoff[s], F->ldzw[s], a + b, a, q, f0, f0, a, b0, cpw});
      }
      L.bw_cnt = (int32_t)items.size() - L.bw_off;
    }
    F->treg_off = (int32_t)tlist.size();
    for (int64_t r = 0; r < m; ++r) tlist.push_back((int32_t)(n1 + r));
    std::vector<int32_t> cpos(std::max<int64_t>(nb, 1), 0);
    for (int64_t q = 0; q < nb; ++q) cpos[cslot[q]] = (int32_t)q;
    std::vector<NdTarget> trec(std::max<size_t>(tlist.size(), 1), NdTarget{0, 0, 0, 0});
    for (size_t g = 0; g < tlist.size(); ++g) {
      const int32_t t = tlist[g];
      trec[g] = NdTarget{node_of[t], t < n1 ? t : (int32_t)(t - n1), cptr[t], cptr[t + 1]};
    }
    std::vector<NdEntry> erec(std::max<size_t>(elist.size(), 1), NdEntry{0, 0});
    for (size_t i = 0; i < elist.size(); ++i) erec[i] = NdEntry{elist[i], S.bkey[elist[i]]};
    CK(c->upload(&F->d_node_of, node_of));
    CK(c->upload(&F->d_cpos, cpos));
    CK(c->upload(&F->d_trec, trec));
    CK(c->upload(&F->d_erec, erec));
    CK(c->upload(&F->d_items, items));
    const int64_t v1 = 3 * std::max<int64_t>(n1, 1), vb = 3 * std::max<int64_t>(nb, 1);
    CK(c->alloc(&F->d_r, v1));
    CK(c->alloc(&F->d_x1, v1));
    CK(c->alloc(&F->d_contrib, vb));
    CK(c->alloc(&F->d_zb, vb));
  }
  HIPCK(c, hipStreamSynchronize(c->st));
  return PD_OK;
}

void nd_condense(pd_ctx* c, const double* f, double* y2) {
  NdFactor* F = c->nd;
  const int n1 = F->sym.n1, m = F->sym.m;
  const long nb = (long)F->nb;
  for (const NdFactor::Level& L : F->levels) {
    // r = f1 - (contributions of the descendants), then the contributions
    // W r of this height to its boundary
    nd_gather_rhs(L.t_cnt, F->d_trec + L.t_off, f, c->n, F->d_contrib, nb, F->d_r, n1, c->st);
    nd_gemv(L.fw_cnt, F->d_items + L.fw_off, F->d_fac, F->d_r, n1, nullptr, 0, F->d_contrib, nb,
            F->d_cpos, c->st);
  }
  nd_gather_rhs(m, F->d_trec + F->treg_off, f, c->n, F->d_contrib, nb, y2, m, c->st);
}

void nd_backsub(pd_ctx* c, const double* delta2, double* x, bool zero_w) {
  NdFactor* F = c->nd;
  const int n1 = F->sym.n1, m = F->sym.m;
  const long nb = (long)F->nb;
  if (n1 == 0) return;
  if (zero_w) zero_f64(3L * n1, F->d_r, c->st);
  for (size_t h = F->levels.size(); h-- > 0;) {
    const NdFactor::Level& L = F->levels[h];
    // zb = solution at the boundary (ancestors, or delta2 on the region),
    // x1 = Z r - W^T zb
    nd_gather_zb(L.e_cnt, F->d_erec + L.e_off, n1, F->d_x1, n1, delta2, m, F->d_zb, nb, c->st);
    nd_gemv(L.bw_cnt, F->d_items + L.bw_off, F->d_fac, F->d_r, n1, F->d_zb, nb, F->d_x1, n1,
            nullptr, c->st);
  }
  scatter_add_rows3(n1, F->d_node_of, F->d_x1, n1, x, c->n, c->st);
}

// Free-node adjacency (both directions, no self loops, ascending per node).
void free_adjacency(int64_t n, int64_t T, const int32_t* tets, const std::vector<int8_t>& cls,
                    std::vector<int64_t>& adj_ptr, std::vector<int32_t>& adj) {
  std::vector<std::pair<int32_t, int32_t>> pairs;
  pairs.reserve((size_t)T * 12);
  for (int64_t e = 0; e < T; ++e)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        if (a == b) continue;
        const int32_t u = tets[a * T + e], v = tets[b * T + e];
        if (cls[u] != 0 && cls[v] != 0) pairs.emplace_back(u, v);
      }
  std::sort(pairs.begin(), pairs.end());
  pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
  adj_ptr.assign(n + 1, 0);
  adj.resize(pairs.size());
  for (size_t i = 0; i < pairs.size(); ++i) {
    adj_ptr[pairs[i].first + 1]++;
    adj[i] = pairs[i].second;
  }
  for (int64_t i = 0; i < n; ++i) adj_ptr[i + 1] += adj_ptr[i];
}

extern "C" pd_status pd_nd_analyse(const pd_mesh* M, int32_t leaf, int64_t* sizes, int32_t* elim,
                                   int32_t* first, int32_t* parent, int64_t* bptr,
                                   int32_t* bkey) {
  if (!M || !M->rest || !M->tets || !M->region || !M->dirichlet || !sizes || M->n_nodes <= 0 ||
      M->n_tets <= 0 || M->n_nodes > INT32_MAX || M->n_tets > INT32_MAX / 4 || leaf < 1)
    return PD_ERR_INVALID;
  const int64_t n = M->n_nodes, T = M->n_tets;
  for (int64_t i = 0; i < 4 * T; ++i)
    if (M->tets[i] < 0 || M->tets[i] >= n) return PD_ERR_INVALID;
  std::vector<int8_t> cls(n);
  std::vector<int32_t> rloc(n, -1);
  int32_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    cls[i] = M->dirichlet[i] ? 0 : (M->region[i] ? 2 : 1);
    if (cls[i] == 2) rloc[i] = m++;
  }
  std::vector<int64_t> adj_ptr;
  std::vector<int32_t> adj;
  free_adjacency(n, T, M->tets, cls, adj_ptr, adj);
  NdSymbolic S;
  std::string err;
  pd_status s = nd_analyse(n, M->rest, cls, rloc, adj_ptr, adj, leaf, S, err);
  if (s != PD_OK) return s;
  const int64_t ns = (int64_t)S.parent.size();
  sizes[0] = S.n1;
  sizes[1] = ns;
  sizes[2] = (int64_t)S.bkey.size();
  if (elim) std::copy(S.elim.begin(), S.elim.end(), elim);
  if (first) std::copy(S.first.begin(), S.first.end(), first);
  if (parent) std::copy(S.parent.begin(), S.parent.end(), parent);
  if (bptr) std::copy(S.bptr.begin(), S.bptr.end(), bptr);
  if (bkey) std::copy(S.bkey.begin(), S.bkey.end(), bkey);
  return PD_OK;
}
