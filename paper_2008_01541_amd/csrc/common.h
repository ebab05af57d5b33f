// Internal definitions shared by the HIP kernels and the host library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdk {

// Dense tiles are NB x NB doubles, column-major; matrices are lower triangular
// where it matters (Cholesky factors), or full symmetric.
constexpr int NB = 64;

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// ---- launchers (all asynchronous on `st`) --------------------------------

// dense FP64
void copy_lower_tiles(const double* S, int lds, double* H, int ldh, int n, hipStream_t st);
// Single-launch dataflow Cholesky; flags: (nt + 2) * nt ints and ticket[2]
// (task counter, launch epoch), all zero-initialised once; each call advances
// the epoch on the device (safe under graph replay).  sbuf: nt * NB * NB
// doubles of workspace (partial sums of the first sub-diagonal tiles).
// With Yt (64 x n, rows 0..2 = g^T) the forward substitution L^-1 g is fused
// in (result in the same rows).  A task never waits for work enqueued on
// another stream: streams may share a hardware queue, which runs in order.
// cu_marks (optional): potrf_cu_slots() zero-initialised ints, the per-unit
// marks by which tasks off the critical path yield to a diagonal task.
// after_reset (optional): recorded once the launch epoch is advanced, before
// the factorization kernel (work on other streams may wait for it and then
// poll the tile flags of the running factorization).
void potrf_dataflow(double* A, int lda, int n, double* linv_ws, double* sbuf, int* flags,
                    unsigned* ticket, int* info, int* err, int n_wg, double* Yt, hipStream_t st,
                    int* cu_marks = nullptr,
                    hipEvent_t after_reset = nullptr);
int potrf_cu_slots();
void rhs_pack(int n, const double* g, int ldg, double* Yt, hipStream_t st);
void rhs_unpack(int n, const double* Yt, double* y, int ldy, hipStream_t st);
// Fill kernels (used instead of memset so the calls can be graph-captured).
void zero_int(int* p, hipStream_t st);
void zero_f64(long n, double* p, hipStream_t st);
void copy_f64(long n, const double* src, double* dst, hipStream_t st);
void copy_i32(long n, const int32_t* src, int32_t* dst, hipStream_t st);
void trtri_from_factor(const double* L, int ldl, int n, const double* linv_ws, double* M,
                       double* X, int ldx, hipStream_t st);
void lauum_full(const double* X, int ldx, int n, double* Z, int ldz, hipStream_t st);
// Triangular solves with the tiled factor, three right-hand sides.  The
// output vector publishes each value as it is stored: before the forward
// solve y must hold the sentinel everywhere (sentinel_fill once; the backward
// solve refills y as it reads it), and the forward solve writes the sentinel
// into xfill (the backward solve's output; may alias g) as it reads g.
// fflags/fticket: the tile flags and ticket of a dataflow Cholesky of L still
// running on another stream (forward solve overlapped with it), or null.
void sentinel_fill(long n, double* p, hipStream_t st);
void trsv3_forward(const double* L, int ld, int n, const double* linv_ws, const double* g,
                   int ldg, double* y, int ldy, unsigned long long* ticket, int* err,
                   double* xfill, int ldxf, hipStream_t st, const int* fflags = nullptr,
                   const unsigned* fticket = nullptr);
void trsv3_backward(const double* L, int ld, int n, const double* linv_ws, double* y, int ldy,
                    double* x, int ldx, unsigned long long* ticket, int* err, hipStream_t st);
// the same solves with a float factor (FP64 vectors and arithmetic)
void trsv3_forward(const float* L, int ld, int n, const float* linv_ws, const double* g, int ldg,
                   double* y, int ldy, unsigned long long* ticket, int* err, double* xfill,
                   int ldxf, hipStream_t st);
void trsv3_backward(const float* L, int ld, int n, const float* linv_ws, double* y, int ldy,
                    double* x, int ldx, unsigned long long* ticket, int* err, hipStream_t st);
// y = alpha * A v + beta * y for symmetric A (full storage), 3 right-hand sides.
void symv3(const double* A, int lda, int n, const double* v, int ldv, double alpha,
           double beta, double* y, int ldy, hipStream_t st);

// low precision (FP32 / BF16-operand) factor of the equilibrated system, on
// the schedule of potrf_dataflow (same flags layout; sbuf: nt * NB * NB floats)
void potrf_dataflow_lp(float* A, int lda, int n, float* linv_ws, float* sbuf, int* flags,
                       unsigned* ticket, int* info, int* err, int n_wg, bool bf16, hipStream_t st,
                       int* cu_marks = nullptr);
void equilibrate_convert(const double* H, int ld, int n, double* d, float* H32, int ld32,
                         hipStream_t st);
// x (+)= D L^-T L^-1 D r with L the FP32 factor of D H D (three right-hand
// sides); b, y: 3 n doubles of workspace, y holding the sentinel
// (sentinel_fill once; each call leaves it so); tickets[2].
void trsv3_lp_solve(const float* L, int ld, int n, const float* linv_ws, const double* d,
                    const double* r, double* b, double* y, double* x, int accumulate,
                    unsigned long long* tickets, int* err, hipStream_t st);

// conjugate-gradient steps on three independent columns [3][n] (scalars in
// device memory): out[v] = a_v . b_v; with nq = -H p and pnq = p . nq,
// u += alpha p, r += alpha nq for alpha = rz / (p^T H p); p = z + (rz_new / rz_old) p.
void dot3(int n, const double* a, const double* b, double* out, hipStream_t st);
void cg_update(int n, const double* rz, const double* pnq, const double* p, const double* nq,
               double* u, double* r, hipStream_t st);
void cg_direction(int n, const double* rz_new, const double* rz_old, const double* z, double* p,
                  hipStream_t st);

// condensation sweeps, one interior level at a time: sweep_symv writes the
// tile parts of Z x for a level of width w (Z symmetric, only its lower tiles
// read) into P (sweep_workspace(maxw) doubles); sweep_assemble forms
// out = Z x, or out = base - Z x when base is non-null (all [3][*] with
// leading dimensions ldx, ldb, ldo).
int64_t sweep_workspace(int64_t maxw);
void sweep_symv(const double* Z, long ldz, int w, const double* x, long ldx, double* P,
                hipStream_t st);
void sweep_assemble(int w, const double* P, const double* base, long ldb, double* out, long ldo,
                    hipStream_t st);

// FEM / sparse
void tet_geometry(const double* rest, int64_t n, const int32_t* tets, int64_t T,
                  double* Bm, double* vol, hipStream_t st);
void element_stiffness(const double* Bm, const double* vol, int64_t T, double mu,
                       double* Ke, hipStream_t st);
void gather_assign(int64_t count, const int64_t* ptr, const int64_t* src, const double* vals,
                   const int64_t* dst_off, double* dst, hipStream_t st);
// biphasic material when mu_p > 0 (strain limits smin, smax)
void local_step(int64_t T, const int32_t* tets, int64_t ldt, const double* Bm,
                const double* vol, int64_t ldb, const double* x, int64_t ldx, double mu,
                double mu_p, double smin, double smax, double* fe, void* R, int rot_fp32,
                hipStream_t st);
void node_gather3(int64_t count, const int32_t* ptr, const int32_t* ent, const double* fe,
                  int64_t ldfe, const int32_t* node_of_row, double* f, int64_t ldf,
                  int accumulate, hipStream_t st);
void gather_rows3(int64_t count, const int32_t* ids, const double* src, int64_t lds,
                  double* dst, int64_t ldd, hipStream_t st);
void scatter_add_rows3(int64_t count, const int32_t* ids, const double* src, int64_t lds,
                       double* dst, int64_t ldd, hipStream_t st);
void csr_spmv3(int64_t rows, const int32_t* ptr, const int32_t* col, const double* val,
               const double* v, int64_t ldv, double alpha, double* y, int64_t ldy,
               const double* base, int64_t ldbase, hipStream_t st);
void dense_times_sparse_t(const double* Z, int ldz, int w, int nr, const int32_t* rows,
                          const int32_t* ptr, const int32_t* col, const double* val,
                          double* U, hipStream_t st);
void sub_sparse_times_dense(double* Next, int ldn, int nr, const int32_t* rows,
                            const int32_t* ptr, const int32_t* col, const double* val,
                            const double* U, int ldu, hipStream_t st);
void detect_spheres(int n_prox, const int32_t* prox, int n_sph, const double* sph, double k,
                    const double* x2, int m, int32_t* idx, double* w, double* c, double* t,
                    hipStream_t st);
void detect_pairs(int n_pairs, const int32_t* pairs, double k, const double* x2, int m,
                  int32_t* idx, double* w, double* c, double* t, hipStream_t st);
// embedded proxies and rest-pose level sets (embed.hip)
void embed_points(int n, const double* pts, int nc, const int32_t* cand, const double* pos, int m,
                  int32_t* tet, int32_t* eidx, double* ew, hipStream_t st);
void detect_embedded_spheres(int n_prox, const int32_t* eidx, const double* ew, int n_sph,
                             const double* sph, double k, const double* x2, int m, int32_t* idx,
                             double* w, double* c, double* t, hipStream_t st);
void detect_levelset(int n_prox, const int32_t* eidx, const double* ew, const int32_t* prox_body,
                     int nc, const int32_t* cand, const double* cand_phi,
                     const int32_t* cand_body, const double* rest2, double k, const double* x2,
                     int m, int32_t* idx, double* w, double* c, double* t, hipStream_t st);
// act[0..*cnt) <- indices j < n_pen with c[j] != 0, increasing (device count);
// rowptr (m + 1) and ent (8 n_pen) <- for every region row a, the keys 8 q + s
// of the active slots naming it (act[q], slot s), increasing; cursor: m ints
// of scratch.
void penalty_prepare(int n_pen, int m, const double* c, const int32_t* idx, int32_t* act,
                     int32_t* cnt, int32_t* rowptr, int32_t* cursor, int32_t* ent, hipStream_t st);
// Over the active penalties, through the incidence built by penalty_prepare:
// row a of H (lower part) += (W^T C W)[a, :]  when H != NULL;
// fcol[:, a] = -(W^T C (W x2 - tscale * t))[a]  when fcol != NULL.
void penalty_apply(int n_pen, const int32_t* act, const int32_t* rowptr, const int32_t* ent,
                   const int32_t* idx, const double* w, const double* c, const double* t,
                   double tscale, const double* x2, int m, double* H, int ldh, double* fcol,
                   hipStream_t st);
// out = (sum ||x - xp||^2, sum ||x - X||^2) over the listed nodes (device, 2 doubles).
void change_norms(int64_t cnt, const int32_t* ids, const double* x, const double* xp,
                  const double* X, int64_t n, double* out, hipStream_t st);
// out[v] = sum_i a[v][i]^2 for the three columns (out: 3 doubles, device).
void colnorm2_3(int m, const double* a, double* out, hipStream_t st);
void ws_input(int m, const double* x2, const double* x2p, float scale, int n_prox,
              const int32_t* prox, const double* c, float* out, hipStream_t st);
void add_at(int64_t count, const int64_t* dst, const double* val, double* base, hipStream_t st);
void inertia_force(int64_t n, const double* D, const double* x, const double* y, double* f,
                   hipStream_t st);
void time_step_advance(int64_t len, double dt, const double* x, double* xp, double* v, double* y,
                       hipStream_t st);
void scale_f32_to_f64(int64_t n, const float* d, double scale, const double* a, const double* b,
                      double* out, hipStream_t st);
void ws_target(int64_t n, const double* x, const double* xp, const double* xpp, float scale,
               float* out, hipStream_t st);
void region_add_f32(int64_t count, const int32_t* ids, const float* d, double scale, double* x,
                    int64_t ldx, hipStream_t st);
void axpy3_sum(int m, const double* a, const double* b, const double* c, double* out,
               hipStream_t st);
void inner_update(int m, const double* u, double* x2, double* d2, hipStream_t st);

// C(r, c) = beta C(r, c) + alpha sum_{k < K} A(r, k) B(c, k) for r < m, c < nc
// (column-major; beta = 0: C is not read).  lower: C is square and only its
// tiles on or below the diagonal are formed.  blower: B is lower triangular
// and only its tiles on or below the diagonal are read (X = L^-1 from
// trtri_from_factor, whose tiles above the diagonal are never written).
void gemm_nt(const double* A, long lda, const double* B, long ldb, double* C, long ldc, int m,
             int nc, int K, double alpha, double beta, int lower, int blower, hipStream_t st);

// ---- nested-dissection interior factor (nd.hip) ----------------------------

// One work item of the supernodal sweeps: 4 cpw columns (cpw = 1 or 4 per
// wave), from col0, of the matrix block at moff (leading dimension ldm,
// rows x cols); rows below split are dotted with one vector (from xoff), the
// rest with another (from x2off, subtracted); the results go to yoff + column.
struct NdItem {
  int64_t moff;
  int32_t ldm, rows, cols, col0, xoff, yoff, split, x2off, cpw;
};
// A target of the right-hand-side gather: the node whose force it starts
// from, its output index, and the range [c0, c1) of its contributions in the
// target-major contribution vector.
struct alignas(16) NdTarget {
  int32_t node, out, c0, c1;
};
// An entry of the boundary gather: boundary entry e and its key.
struct alignas(8) NdEntry {
  int32_t e, key;
};
// Adds the lower entries (r >= c) of the b x b update matrix U of a child
// into its parent's front: i = map[r], j = map[c]; j < ns: into the front's
// first ns columns P (F_ss entries mirrored to the upper triangle), else into
// the trailing update block Uo at (i - ns, j - ns) (mirrored when mirror).
void nd_extend_add(const double* U, long ldu, int b, const int32_t* map, int ns, double* P,
                   long ldp, double* Uo, long lduo, int mirror, hipStream_t st);
// dst[v][out] = f[v][node] - sum_{c0 <= e < c1} contrib[v][e] for the cnt targets of trec.
void nd_gather_rhs(int cnt, const NdTarget* trec, const double* f, long ldf,
                   const double* contrib, long ldc, double* dst, long ldd, hipStream_t st);
// y = M^T [xa; -xb] per item (see NdItem), three right-hand sides; the result
// of column index q = yoff + column goes to y[ymap[q]] (ymap may be null: y[q]).
void nd_gemv(int nitems, const NdItem* items, const double* M, const double* xa, long ldxa,
             const double* xb, long ldxb, double* y, long ldy, const int32_t* ymap,
             hipStream_t st);
// dst (cols x rows) = src^T (src rows x cols), column-major.
void nd_transpose(const double* src, long lds, int rows, int cols, double* dst, long ldd,
                  hipStream_t st);
// zb[v][e] = key < n1 ? z[v][key] : d2[v][key - n1] for the cnt entries (e, key) of erec.
void nd_gather_zb(int cnt, const NdEntry* erec, int n1, const double* z, long ldz,
                  const double* d2, long ldd2, double* zb, long ldzb, hipStream_t st);

}  // namespace pdk
