// Host side of the warm-start MLP entry points (pd_mlp_*): parameter buffers,
// forward pass, backward pass and Adam, all enqueued on one stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pdschur.h"
#include "common.h"

namespace pdk {
void mlp_gemm(int M, int N, int K, const void* A, bool a_bf16, bool a_kcontig, long lda,
              const void* B, bool b_bf16, bool b_kcontig, long ldb, float* part, int nsplit,
              hipStream_t st);
int mlp_gemm_nsplit(int M, int N, int K, int nsplit);
void mlp_split_reduce(int M, int N, int nsplit, const float* part, const float* bias, int relu,
                      float* out, hipStream_t st);
void mlp_loss_grad(long total, int n_out_times_b, const float* Y, const float* T, float* dY,
                   double* part, double* loss, hipStream_t st);
void mlp_relu_back(long n, const float* H, float* dA, hipStream_t st);
void mlp_colsum(int M, int N, const float* dZ, float* gb, hipStream_t st);
void mlp_adam(long n, float* w, const float* g, float* m, float* v, __bf16* wb, float lr, int step,
              hipStream_t st);
void mlp_to_bf16(long n, const float* w, __bf16* wb, hipStream_t st);
void mlp_gather_rows_scaled(int B, int n_cols, const float* src, const int32_t* rows, int n_scaled,
                            float scale, float* dst, hipStream_t st);
void mlp_abs_mean(long n, const float* a, double* out, hipStream_t st);
}  // namespace pdk

using namespace pdk;

struct pd_mlp {
  hipStream_t st = nullptr;
  std::string err;
  int nin = 0, nh1 = 0, nh2 = 0, nout = 0, maxb = 0, step = 0;
  long off[7] = {0};                 // W1 b1 W2 b2 W3 b3 end (floats)
  long boff[4] = {0};                // W1 W2 W3 end (bf16)
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  __bf16* wb = nullptr;
  float *H1 = nullptr, *H2 = nullptr, *Y = nullptr, *dY = nullptr, *dA2 = nullptr, *dA1 = nullptr;
  float* part = nullptr;
  long part_size = 0;
  double *lpart = nullptr, *loss = nullptr;
  std::vector<void*> mem;
  ~pd_mlp() {
    for (void* q : mem) (void)hipFree(q);
  }
  template <typename T>
  bool alloc(T** q, long n) {
    if (hipMalloc((void**)q, std::max<long>(n, 1) * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      err = "device allocation failed";
      return false;
    }
    mem.push_back(*q);
    return true;
  }
};

namespace {

int pick_split(int M, int N, int K) {
  const long tiles = (long)((M + 63) / 64) * ((N + 63) / 64);
  int s = (int)std::max<long>(1, 512 / std::max<long>(tiles, 1));
  s = std::min(s, std::max(1, K / 256));
  return s;
}

// out = opA opB^T (+ bias) (relu) through the split-K workspace
void gemm_to(pd_mlp* h, int M, int N, int K, const void* A, bool abf, bool akc, long lda,
             const void* B, bool bbf, bool bkc, long ldb, const float* bias, int relu, float* out) {
  const int s = pick_split(M, N, K);
  const int nz = mlp_gemm_nsplit(M, N, K, s);
  if (nz == 1 && !bias && !relu) {
    mlp_gemm(M, N, K, A, abf, akc, lda, B, bbf, bkc, ldb, out, s, h->st);
    return;
  }
  mlp_gemm(M, N, K, A, abf, akc, lda, B, bbf, bkc, ldb, h->part, s, h->st);
  mlp_split_reduce(M, N, nz, h->part, bias, relu, out, h->st);
}

void forward(pd_mlp* h, const float* x, int B, float* y) {
  const float* P = h->p;
  gemm_to(h, B, h->nh1, h->nin, x, false, true, h->nin, h->wb + h->boff[0], true, true, h->nin,
          P + h->off[1], 1, h->H1);
  gemm_to(h, B, h->nh2, h->nh1, h->H1, false, true, h->nh1, h->wb + h->boff[1], true, true, h->nh1,
          P + h->off[3], 1, h->H2);
  gemm_to(h, B, h->nout, h->nh2, h->H2, false, true, h->nh2, h->wb + h->boff[2], true, true, h->nh2,
          P + h->off[5], 0, y);
}

bool bad_batch(const pd_mlp* h, int B) { return B <= 0 || B > h->maxb; }

}  // namespace

extern "C" {

pd_status pd_mlp_create(int32_t n_in, int32_t n_h1, int32_t n_h2, int32_t n_out, int32_t max_batch,
                        const float* params_host, void* stream, pd_mlp** out) {
  if (!out) return PD_ERR_INVALID;
  *out = nullptr;
  if (n_in <= 0 || n_h1 <= 0 || n_h2 <= 0 || n_out <= 0 || max_batch <= 0 || !params_host)
    return PD_ERR_INVALID;
  pd_mlp* h = new pd_mlp();
  h->st = (hipStream_t)stream;
  h->nin = n_in; h->nh1 = n_h1; h->nh2 = n_h2; h->nout = n_out; h->maxb = max_batch;
  const long sizes[6] = {(long)n_h1 * n_in, n_h1, (long)n_h2 * n_h1, n_h2, (long)n_out * n_h2, n_out};
  for (int i = 0; i < 6; ++i) h->off[i + 1] = h->off[i] + sizes[i];
  h->boff[1] = sizes[0];
  h->boff[2] = sizes[0] + sizes[2];
  h->boff[3] = sizes[0] + sizes[2] + sizes[4];
  const long np = h->off[6];
  long part = (long)std::max({n_h1, n_h2, n_out}) * std::max<long>(n_in, n_h2);   // gradient of W
  part = std::max<long>(part, 64L * max_batch * std::max({n_h1, n_h2, n_out}));
  h->part_size = part;
  bool ok = h->alloc(&h->p, np) && h->alloc(&h->g, np) && h->alloc(&h->m, np) && h->alloc(&h->v, np) &&
            h->alloc(&h->wb, h->boff[3]) && h->alloc(&h->H1, (long)max_batch * n_h1) &&
            h->alloc(&h->H2, (long)max_batch * n_h2) && h->alloc(&h->Y, (long)max_batch * n_out) &&
            h->alloc(&h->dY, (long)max_batch * n_out) && h->alloc(&h->dA2, (long)max_batch * n_h2) &&
            h->alloc(&h->dA1, (long)max_batch * n_h1) && h->alloc(&h->part, part) &&
            h->alloc(&h->lpart, 256) && h->alloc(&h->loss, 1);
  if (!ok) {
    delete h;
    return PD_ERR_OOM;
  }
  if (hipMemcpy(h->p, params_host, np * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemsetAsync(h->m, 0, np * sizeof(float), h->st) != hipSuccess ||
      hipMemsetAsync(h->v, 0, np * sizeof(float), h->st) != hipSuccess) {
    delete h;
    return PD_ERR_HIP;
  }
  mlp_to_bf16(h->off[1], h->p + h->off[0], h->wb + h->boff[0], h->st);
  mlp_to_bf16(h->off[3] - h->off[2], h->p + h->off[2], h->wb + h->boff[1], h->st);
  mlp_to_bf16(h->off[5] - h->off[4], h->p + h->off[4], h->wb + h->boff[2], h->st);
  if (hipStreamSynchronize(h->st) != hipSuccess) {
    delete h;
    return PD_ERR_HIP;
  }
  *out = h;
  return PD_OK;
}

pd_status pd_mlp_get_params(pd_mlp* h, float* params_host) {
  if (!h || !params_host) return PD_ERR_INVALID;
  if (hipStreamSynchronize(h->st) != hipSuccess ||
      hipMemcpy(params_host, h->p, h->off[6] * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return PD_ERR_HIP;
  return PD_OK;
}

pd_status pd_mlp_forward(pd_mlp* h, const float* x, float* y, int32_t batch) {
  if (!h || !x || !y || bad_batch(h, batch)) return PD_ERR_INVALID;
  forward(h, x, batch, y);
  return hipGetLastError() == hipSuccess ? PD_OK : PD_ERR_HIP;
}

pd_status pd_mlp_train_step(pd_mlp* h, const float* x, const float* target, int32_t B, float lr,
                            double* loss_host, float* grads_host) {
  if (!h || !x || !target || bad_batch(h, B) || !(lr >= 0.f)) return PD_ERR_INVALID;
  float* P = h->p;
  float* G = h->g;
  forward(h, x, B, h->Y);
  mlp_loss_grad((long)B * h->nout, B * h->nout, h->Y, target, h->dY, h->lpart, h->loss, h->st);
  // layer 3
  gemm_to(h, h->nout, h->nh2, B, h->dY, false, false, h->nout, h->H2, false, false, h->nh2, nullptr,
          0, G + h->off[4]);
  mlp_colsum(B, h->nout, h->dY, G + h->off[5], h->st);
  gemm_to(h, B, h->nh2, h->nout, h->dY, false, true, h->nout, h->wb + h->boff[2], true, false,
          h->nh2, nullptr, 0, h->dA2);
  mlp_relu_back((long)B * h->nh2, h->H2, h->dA2, h->st);
  // layer 2
  gemm_to(h, h->nh2, h->nh1, B, h->dA2, false, false, h->nh2, h->H1, false, false, h->nh1, nullptr,
          0, G + h->off[2]);
  mlp_colsum(B, h->nh2, h->dA2, G + h->off[3], h->st);
  gemm_to(h, B, h->nh1, h->nh2, h->dA2, false, true, h->nh2, h->wb + h->boff[1], true, false,
          h->nh1, nullptr, 0, h->dA1);
  mlp_relu_back((long)B * h->nh1, h->H1, h->dA1, h->st);
  // layer 1
  gemm_to(h, h->nh1, h->nin, B, h->dA1, false, false, h->nh1, x, false, false, h->nin, nullptr, 0,
          G + h->off[0]);
  mlp_colsum(B, h->nh1, h->dA1, G + h->off[1], h->st);
  if (grads_host) {
    if (hipMemcpyAsync(grads_host, G, h->off[6] * sizeof(float), hipMemcpyDeviceToHost, h->st) !=
        hipSuccess)
      return PD_ERR_HIP;
  } else {
    h->step += 1;
    for (int sgm = 0; sgm < 6; ++sgm) {
      __bf16* wbp = nullptr;
      if (sgm == 0) wbp = h->wb + h->boff[0];
      if (sgm == 2) wbp = h->wb + h->boff[1];
      if (sgm == 4) wbp = h->wb + h->boff[2];
      mlp_adam(h->off[sgm + 1] - h->off[sgm], P + h->off[sgm], G + h->off[sgm], h->m + h->off[sgm],
               h->v + h->off[sgm], wbp, lr, h->step, h->st);
    }
  }
  if (loss_host) {
    if (hipMemcpyAsync(loss_host, h->loss, sizeof(double), hipMemcpyDeviceToHost, h->st) != hipSuccess ||
        hipStreamSynchronize(h->st) != hipSuccess)
      return PD_ERR_HIP;
  } else if (grads_host) {
    if (hipStreamSynchronize(h->st) != hipSuccess) return PD_ERR_HIP;
  }
  return hipGetLastError() == hipSuccess ? PD_OK : PD_ERR_HIP;
}

pd_status pd_mlp_gather_rows(pd_mlp* h, const float* src, int32_t n_rows, int32_t n_cols,
                             const int32_t* rows, int32_t B, int32_t n_scaled, float scale,
                             float* dst) {
  if (!h || !src || !rows || !dst || n_rows <= 0 || n_cols <= 0 || B <= 0 || B > 65535 ||
      n_scaled < 0 || n_scaled > n_cols || !std::isfinite(scale))
    return PD_ERR_INVALID;
  mlp_gather_rows_scaled(B, n_cols, src, rows, n_scaled, scale, dst, h->st);
  return hipGetLastError() == hipSuccess ? PD_OK : PD_ERR_HIP;
}

pd_status pd_mlp_abs_mean(pd_mlp* h, const float* a, int64_t n, double* out_host) {
  if (!h || !a || n <= 0 || !out_host) return PD_ERR_INVALID;
  mlp_abs_mean(n, a, h->loss, h->st);
  if (hipMemcpyAsync(out_host, h->loss, sizeof(double), hipMemcpyDeviceToHost, h->st) != hipSuccess ||
      hipStreamSynchronize(h->st) != hipSuccess)
    return PD_ERR_HIP;
  return PD_OK;
}

pd_status pd_mlp_destroy(pd_mlp* h) {
  if (!h) return PD_ERR_INVALID;
  (void)hipStreamSynchronize(h->st);
  delete h;
  return PD_OK;
}

}  // extern "C"
