// Internal host-side context of the C ABI library (shared by api.cpp and the
// nested-dissection interior factor in nd_factor.cpp): device allocations owned by
// a context, the context itself, error macros and the gather plans that
// assemble matrix entries from element-stiffness contributions.
#pragma once
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/pdschur.h"
#include "common.h"

// Device allocations of a context, freed with it.
struct PdDevAlloc {
  std::vector<void*> ptrs;
  ~PdDevAlloc() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

struct NdFactor;
void nd_free(NdFactor* f);

struct pd_ctx {
  hipStream_t st = nullptr;
  std::string err;
  bool broken = false;

  int64_t n = 0, T = 0, m = 0, n1 = 0, nbeta = 0, nalpha = 0;
  int K = 0;
  double mu = 0.0;

  std::vector<int32_t> region_ids;   // global ids of x2, ascending
  std::vector<int64_t> lev_off;      // [K+1] offsets into the interior ordering
  std::vector<int64_t> lev_mat_off;  // [K] offsets (doubles) of Z_k in levmat
  std::vector<int64_t> B_ptr_off, B_nnz_off, Bt_ptr_off, Bt_nnz_off, Brows_off, Brows_cnt;
  int64_t maxw = 0;
  int64_t maxldw = 0;
  int ntm = 0;                        // tiles of the m x m system
  int ldH = 0, ldH32 = 0;             // padded leading dimensions of the work matrices
  std::vector<int> ldw;               // padded leading dimension of each level block

  PdDevAlloc mem;
  // mesh subsets
  int32_t* d_tets_alpha = nullptr;   // [4][nalpha] global ids
  double* d_Bm_alpha = nullptr;      // [9][nalpha]
  double* d_vol_alpha = nullptr;
  int32_t* d_tets_beta = nullptr;    // [4][nbeta] region-local ids
  double* d_Bm_beta = nullptr;
  double* d_vol_beta = nullptr;
  double* d_fe = nullptr;            // [12][nalpha]: element forces of the full local step
  double* d_fe_b = nullptr;          // [12][nbeta]: element forces of the region local step
  int32_t *d_inc_a_ptr = nullptr, *d_inc_a = nullptr;
  int32_t *d_inc_b_ptr = nullptr, *d_inc_b = nullptr;
  int32_t* d_region_ids = nullptr;
  int32_t* d_free_ids = nullptr;      // every free node (x1 and x2)
  double* d_rest = nullptr;           // rest positions [3][n]
  int64_t n_free = 0;
  int32_t* d_lev_nodes = nullptr;    // [n1] global ids in level order
  double* d_levmat = nullptr;        // Z_k = S_k^-1, full symmetric, per level
  int32_t *d_Bptr = nullptr, *d_Bcol = nullptr, *d_Btptr = nullptr, *d_Btcol = nullptr;
  double *d_Bval = nullptr, *d_Btval = nullptr;
  int32_t* d_Brows = nullptr;
  int32_t *d_Abptr = nullptr, *d_Abcol = nullptr;
  double* d_Abval = nullptr;
  // dense system
  double* d_S = nullptr;
  double* d_H = nullptr;
  double* d_linv = nullptr;
  double* d_sbuf = nullptr;           // partial sums of the first sub-diagonal tiles (factor)
  double* d_y = nullptr;               // scratch of the residual products
  double* d_ys = nullptr;              // forward-solve result (holds the sentinel between solves)
  double* d_Yt = nullptr;             // 64 x m right-hand-side tile row of the fused solve
  double* d_res = nullptr;
  double* d_norms = nullptr;
  int* d_info = nullptr;
  int* d_err = nullptr;
  unsigned long long* d_ticket = nullptr;
  int* d_tflags = nullptr;            // tile-ready flags of the dataflow Cholesky
  int* d_cumarks = nullptr;           // per-compute-unit marks of the dataflow Cholesky
  unsigned* d_tticket = nullptr;
  int chol_epoch = 0;
  int n_wg = 512;
  // low-precision factor for the refined solves
  float* d_H32 = nullptr;
  float* d_linv32 = nullptr;
  double* d_lpb = nullptr;            // workspaces of the float-factor solves (3 m each)
  double* d_lpy = nullptr;
  double* d_dvec = nullptr;
  unsigned long long* d_lp_ticket = nullptr;
  int lp_prec = -1;                   // precision of the current low-precision factor
  bool lp_stale = true;
  int lp_info = -1;                   // its first non-positive pivot (0: none; -1: not read yet)
  int max_ir = 100;
  double ir_tol = 1e-8;
  int ir_fallback = 1;                // refactor in FP64 when the refinement stalls
  double* d_cgp = nullptr;            // conjugate-gradient vectors (3 m each) and scalars
  double* d_cgq = nullptr;
  double* d_cgz = nullptr;
  double* d_cgs = nullptr;
  // sweeps
  double *d_fhat = nullptr, *d_v = nullptr, *d_xs = nullptr, *d_tmp = nullptr;
  double* d_ext = nullptr;     // warm start: predicted region increment in FP64
  double dt = 0.0;             // backward-Euler time step (0: quasistatic)
  double mu_p = 0.0, smin = 0.0, smax = 0.0;   // biphasic material (mu_p = 0: corotated)
  std::vector<double> h_D;     // inertia diagonal M / dt^2 per node (0 on prescribed nodes)
  double* d_D = nullptr;
  const double* d_target = nullptr;  // caller's inertial target x_n + dt v_n
  bool have_condense = false;
  double* d_P = nullptr;              // tile parts of a level's (or S's) dense product
  bool overlap = false;               // the forward solve may overlap the running factorization
  hipEvent_t ev_fstart = nullptr;     // factorization epoch advanced (its flags may be polled)
  hipEvent_t ev_fdone = nullptr;      // factorization finished
  // penalties
  int32_t n_pen = 0, pen_cap = 0;
  int32_t* d_pidx = nullptr;
  double *d_pw = nullptr, *d_pc = nullptr, *d_pt = nullptr;
  int32_t* d_pact = nullptr;          // active penalties (c != 0), increasing
  int32_t* d_pnact = nullptr;         // their count (device)
  int32_t* d_prow = nullptr;          // incidence of the active slots on region rows: row pointers
  int32_t* d_pcur = nullptr;          // (m + 1), cursors (m), keys (8 per penalty)
  int32_t* d_pent = nullptr;
  bool stale = true;

  // optional per-phase timing with HIP events recorded on the stream
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, std::pair<size_t, size_t>>> ev_pairs;   // (phase, (start, end))
  hipEvent_t next_event() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }
  NdFactor* nd = nullptr;             // nested-dissection interior factor (interior_order = 1)
  ~pd_ctx() {
    nd_free(nd);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (ev_fstart) (void)hipEventDestroy(ev_fstart);
    if (ev_fdone) (void)hipEventDestroy(ev_fdone);
  }

  pd_status fail(pd_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    if (s == PD_ERR_HIP) broken = true;
    return s;
  }
  template <typename TT>
  pd_status alloc(TT** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc((void**)p, count * sizeof(TT)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(PD_ERR_OOM, "device allocation of %zu bytes failed", count * sizeof(TT));
    }
    mem.ptrs.push_back((void*)*p);
    return PD_OK;
  }
  template <typename TT>
  pd_status upload(TT** p, const std::vector<TT>& h) {
    pd_status s = alloc(p, h.size());
    if (s != PD_OK) return s;
    if (!h.empty() && hipMemcpy(*p, h.data(), h.size() * sizeof(TT), hipMemcpyHostToDevice) != hipSuccess)
      return fail(PD_ERR_HIP, "host-to-device copy failed");
    return PD_OK;
  }
  pd_status check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return PD_OK;
  }
};

#define CK(expr)                             \
  do {                                       \
    pd_status _s = (expr);                   \
    if (_s != PD_OK) return _s;              \
  } while (0)

#define HIPCK(ctx, expr)                                                                 \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) return (ctx)->fail(PD_ERR_HIP, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

// Gather plan: dst[dst_off[i]] = sum of vals[src[e]] for e in [ptr[i], ptr[i+1]).
struct Plan {
  std::vector<int64_t> ptr{0}, src, dst;
  void add_group(const int64_t* s, int64_t cnt, int64_t d) {
    for (int64_t i = 0; i < cnt; ++i) src.push_back(s[i]);
    ptr.push_back((int64_t)src.size());
    dst.push_back(d);
  }
};

// Runs a plan on the context's stream (synchronizes; the plan's device copy
// is freed right away) / frees one of the context's allocations now.
pd_status run_plan(pd_ctx* c, const Plan& P, const double* vals, double* dst);
void free_now(pd_ctx* c, void* p);

// Nested-dissection interior factor (nd_factor.cpp).  Symbolic part: the
// elimination order of the interior nodes (cls 1) grouped into supernodes
// (children before parents), the parent of each supernode (the one holding
// the first key of its boundary; -1: the boundary is empty or in the region,
// whose Schur complement takes the update), its height in the tree (leaves 0)
// and its boundary keys (ascending; a key below n1 is an elimination
// position, n1 + r the region node r).
struct NdSymbolic {
  int32_t n1 = 0, m = 0;
  std::vector<int32_t> elim;     // [n1] node at each elimination position
  std::vector<int32_t> first;    // [ns + 1] positions of each supernode
  std::vector<int32_t> parent;   // [ns]
  std::vector<int32_t> height;   // [ns]
  std::vector<int64_t> bptr;     // [ns + 1] ranges in bkey
  std::vector<int32_t> bkey;
};
pd_status nd_analyse(int64_t n, const double* rest, const std::vector<int8_t>& cls,
                     const std::vector<int32_t>& rloc, const std::vector<int64_t>& adj_ptr,
                     const std::vector<int32_t>& adj, int leaf, NdSymbolic& S, std::string& err);
// Free-node adjacency (cls != 0 on both ends), ascending per node.
void free_adjacency(int64_t n, int64_t T, const int32_t* tets, const std::vector<int8_t>& cls,
                    std::vector<int64_t>& adj_ptr, std::vector<int32_t>& adj);
// nd_prepare: ordering and symbolic factorization (sets c->nd, c->n1 and
// c->maxw, the largest supernode).  nd_factor: with c->d_S holding K22 (no
// inertia yet) and the dense-factor workspaces allocated for c->maxw,
// assembles the fronts, factors them on the GPU and adds the Schur update
// into c->d_S (with the inertia diagonal when dt > 0).
pd_status nd_prepare(pd_ctx* c, const double* rest, const std::vector<int8_t>& cls,
                     const std::vector<int32_t>& rloc, const std::vector<int64_t>& adj_ptr,
                     const std::vector<int32_t>& adj, int leaf);
pd_status nd_factor(pd_ctx* c, const int32_t* tets, int64_t T, const std::vector<int8_t>& cls,
                    const std::vector<int32_t>& rloc, const double* d_Ke);
int nd_height(const pd_ctx* c);
// nd_condense: y2 = f2 - A21 A11^-1 f1 (keeps the gathered right-hand sides
// r_s of the supernodes for nd_backsub);
// nd_backsub: x1 += A11^-1 (f1 - A12 delta2) on the interior nodes of x
// (zero_w: with f1 = 0); the region part is left to the caller.
void nd_condense(pd_ctx* c, const double* f, double* y2);
void nd_backsub(pd_ctx* c, const double* delta2, double* x, bool zero_w);
