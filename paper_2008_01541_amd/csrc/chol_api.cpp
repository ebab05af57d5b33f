// Host side of the standalone dense Cholesky entry points (pd_chol_*): the
// single-launch dataflow factorization used for H = S + P, with its own
// workspace, for callers that need the factorization alone.
#include <algorithm>
#include <mutex>

#include "../../include/pdschur.h"
#include "common.h"
#include "df_schedule.h"

using namespace pdk;

struct pd_chol {
  hipStream_t st = nullptr;
  int64_t n_max = 0;
  int n_wg = 512;
  double* linv = nullptr;      // tile inverses, nt x 64 x 64
  double* sbuf = nullptr;      // partial sums of the first sub-diagonal tiles, nt x 64 x 64
  int* flags = nullptr;        // (nt + 2) x nt ready flags (launch epochs)
  unsigned* ticket = nullptr;  // task ticket and launch epoch
  int* info = nullptr;
  int* err = nullptr;
  int* marks = nullptr;        // per-compute-unit marks
  ~pd_chol() {
    for (void* p : {(void*)linv, (void*)sbuf, (void*)flags, (void*)ticket, (void*)info, (void*)err,
                    (void*)marks})
      if (p) (void)hipFree(p);
  }
};

// ---- workspace without allocation (pd_chol_factor_noalloc) ------------------
// The same workspace as a pd_chol handle for n <= PD_CHOL_NOALLOC_MAX_N, in one
// static device array: tile inverses, partial sums, ready flags, ticket, info,
// error word and the per-unit marks.  Every GPU the library runs on holds its
// own copy until the process ends.
constexpr int64_t NA_NT = (PD_CHOL_NOALLOC_MAX_N + NB - 1) / NB;
constexpr int64_t NA_LINV = 0;                               // doubles
constexpr int64_t NA_SBUF = NA_LINV + NA_NT * NB * NB;       // doubles
constexpr int64_t NA_INTS = NA_SBUF + NA_NT * NB * NB;       // doubles: start of the int area
constexpr int64_t NA_FLAGS_N = (NA_NT + 2) * NA_NT;
constexpr int64_t NA_MARKS_N = 2048;
constexpr int64_t NA_INT_N = NA_FLAGS_N + 4 + 1 + 1 + NA_MARKS_N;
constexpr int64_t NA_DOUBLES = NA_INTS + (NA_INT_N + 1) / 2;
static __device__ __align__(256) double scratch[NA_DOUBLES];

namespace {
constexpr int NA_MAX_DEV = 64;
struct NoallocDev {
  double* ptr = nullptr;   // device address of scratch on this device
  int n_wg = 512;
  bool cleared = false;
};
std::mutex na_mu;
NoallocDev na_dev[NA_MAX_DEV];

// Device address of this device's copy of the scratch array (looked up once
// per device, with the device current; never the host-side symbol itself).
pd_status noalloc_setup(int dev, NoallocDev** out) {
  if (dev < 0 || dev >= NA_MAX_DEV) return PD_ERR_INVALID;
  std::lock_guard<std::mutex> lk(na_mu);
  NoallocDev& d = na_dev[dev];
  if (!d.ptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PD_ERR_HIP;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        ncu > 0)
      d.n_wg = 2 * ncu;
    d.ptr = static_cast<double*>(p);
  }
  *out = &d;
  return PD_OK;
}
}  // namespace

extern "C" {

pd_status pd_chol_create(int64_t n_max, void* stream, pd_chol** out) {
  if (!out) return PD_ERR_INVALID;
  *out = nullptr;
  if (n_max <= 0 || n_max > (int64_t)INT32_MAX / 2) return PD_ERR_INVALID;
  pd_chol* h = new pd_chol();
  h->st = (hipStream_t)stream;
  h->n_max = n_max;
  const int64_t nt = (n_max + NB - 1) / NB;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
    h->n_wg = 2 * ncu;
  const int nmarks = potrf_cu_slots();
  bool ok = hipMalloc(&h->linv, nt * NB * NB * sizeof(double)) == hipSuccess &&
            hipMalloc(&h->sbuf, nt * NB * NB * sizeof(double)) == hipSuccess &&
            hipMalloc(&h->flags, (nt + 2) * nt * sizeof(int)) == hipSuccess &&
            hipMalloc(&h->ticket, 4 * sizeof(unsigned)) == hipSuccess &&
            hipMalloc(&h->info, sizeof(int)) == hipSuccess &&
            hipMalloc(&h->err, sizeof(int)) == hipSuccess &&
            hipMalloc(&h->marks, nmarks * sizeof(int)) == hipSuccess;
  if (!ok) {
    delete h;
    return PD_ERR_OOM;
  }
  ok = hipMemsetAsync(h->flags, 0, (nt + 2) * nt * sizeof(int), h->st) == hipSuccess &&
       hipMemsetAsync(h->ticket, 0, 4 * sizeof(unsigned), h->st) == hipSuccess &&
       hipMemsetAsync(h->marks, 0, nmarks * sizeof(int), h->st) == hipSuccess &&
       hipStreamSynchronize(h->st) == hipSuccess;
  if (!ok) {
    delete h;
    return PD_ERR_HIP;
  }
  *out = h;
  return PD_OK;
}

pd_status pd_chol_factor(pd_chol* h, double* A, int64_t lda, int64_t n, int32_t n_workgroups,
                         int32_t* info_host) {
  // Tiles are published across workgroups with write-through stores and read
  // back with ordinary cached loads; that is only safe when no two tiles share
  // a 128-byte line, i.e. every column (and so every tile) starts on one.
  if (!h || !A || n <= 0 || n > h->n_max || lda < n || lda % 16 != 0 || lda > INT32_MAX ||
      reinterpret_cast<uintptr_t>(A) % 128 != 0)
    return PD_ERR_INVALID;
  zero_int(h->info, h->st);
  zero_int(h->err, h->st);
  const int nwg = n_workgroups > 0 ? std::min<int>(n_workgroups, h->n_wg) : h->n_wg;
  potrf_dataflow(A, (int)lda, (int)n, h->linv, h->sbuf, h->flags, h->ticket, h->info, h->err, nwg,
                 nullptr, h->st, h->marks, nullptr);
  if (hipGetLastError() != hipSuccess) return PD_ERR_HIP;
  if (!info_host) return PD_OK;
  int hinfo = 0, herr = 0;
  if (hipStreamSynchronize(h->st) != hipSuccess ||
      hipMemcpy(&hinfo, h->info, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&herr, h->err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return PD_ERR_HIP;
  *info_host = hinfo;
  if (herr) return PD_ERR_HIP;
  return hinfo ? PD_ERR_NOT_SPD : PD_OK;
}

pd_status pd_chol_factor_noalloc(double* A, int64_t lda, int64_t n, int32_t n_workgroups,
                                 void* hip_stream, int32_t* info_host) {
  if (!A || n <= 0 || n > PD_CHOL_NOALLOC_MAX_N || lda < n || lda % 16 != 0 || lda > INT32_MAX ||
      reinterpret_cast<uintptr_t>(A) % 128 != 0)
    return PD_ERR_INVALID;
  if (potrf_cu_slots() > NA_MARKS_N) return PD_ERR_INVALID;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PD_ERR_HIP;
  NoallocDev* d = nullptr;
  pd_status s = noalloc_setup(dev, &d);
  if (s != PD_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  double* base = d->ptr;
  double* linv = base + NA_LINV;
  double* sbuf = base + NA_SBUF;
  int* ints = reinterpret_cast<int*>(base + NA_INTS);
  int* flags = ints;
  unsigned* ticket = reinterpret_cast<unsigned*>(ints + NA_FLAGS_N);
  int* info = ints + NA_FLAGS_N + 4;
  int* err = info + 1;
  int* marks = err + 1;
  {
    // first call on this device: flags, ticket and marks start at zero (a fill
    // kernel on the caller's stream, ahead of the factorization)
    std::lock_guard<std::mutex> lk(na_mu);
    if (!d->cleared) {
      zero_f64(NA_DOUBLES - NA_INTS, base + NA_INTS, st);
      d->cleared = true;
    }
  }
  zero_int(info, st);
  zero_int(err, st);
  const int nwg = n_workgroups > 0 ? std::min<int>(n_workgroups, d->n_wg) : d->n_wg;
  potrf_dataflow(A, (int)lda, (int)n, linv, sbuf, flags, ticket, info, err, nwg, nullptr, st,
                 marks, nullptr);
  if (hipGetLastError() != hipSuccess) return PD_ERR_HIP;
  if (!info_host) return PD_OK;
  int hinfo = 0, herr = 0;
  if (hipStreamSynchronize(st) != hipSuccess ||
      hipMemcpy(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&herr, err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return PD_ERR_HIP;
  *info_host = hinfo;
  if (herr) return PD_ERR_HIP;
  return hinfo ? PD_ERR_NOT_SPD : PD_OK;
}

pd_status pd_chol_destroy(pd_chol* h) {
  if (!h) return PD_ERR_INVALID;
  (void)hipStreamSynchronize(h->st);
  delete h;
  return PD_OK;
}

pd_status pd_dataflow_task(int64_t n, int32_t rhs, int64_t q, int32_t* i, int32_t* j,
                           int32_t* kend, int64_t* ntask) {
  if (n < 1 || n > 46340 || (rhs != 0 && rhs != 1) || !ntask) return PD_ERR_INVALID;
  const int nt = (int)((n + NB - 1) / NB);
  *ntask = df_task_count(nt, rhs);
  if (q < 0) return PD_OK;
  if (q >= *ntask || !i || !j || !kend) return PD_ERR_INVALID;
  int ti, tj;
  df_task_of_ticket((int)q, nt, rhs, ti, tj);
  *i = ti;
  *j = tj;
  *kend = df_task_kend(ti, tj);
  return PD_OK;
}

}  // extern "C"
