// Host side of the standalone dense Cholesky entry points (pd_chol_*): the
// single-launch dataflow factorization used for H = S + P, with its own
// workspace, for callers that need the factorization alone.
#include <algorithm>

#include "../../include/pdschur.h"
#include "common.h"

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
                 nullptr, h->st, nullptr, 0, h->marks, nullptr);
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

pd_status pd_chol_destroy(pd_chol* h) {
  if (!h) return PD_ERR_INVALID;
  (void)hipStreamSynchronize(h->st);
  delete h;
  return PD_OK;
}

}  // extern "C"
