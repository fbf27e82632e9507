// muca_mlp_host.hip -- C ABI of the learned-initial-weights network
// (include/muca.h, section "Learned initial weights").
#include <hip/hip_runtime.h>

#include <cmath>

#include "muca_context.h"
#include "muca_mlp.h"

using muca_detail::fail;

#define MLP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(e_ == hipErrorOutOfMemory ? MUCA_ENOMEM : MUCA_EHIP, "%s: %s", #expr,     \
                  hipGetErrorString(e_));                                                   \
  } while (0)

#define MLP_LAUNCHED()                                                                      \
  do {                                                                                      \
    hipError_t e_ = hipGetLastError();                                                      \
    if (e_ != hipSuccess) return fail(MUCA_EHIP, "kernel launch: %s", hipGetErrorString(e_)); \
  } while (0)

struct muca_mlp {
  int max_rows = 0;
  int step = 0;
  float* P = nullptr;        // FP32 master parameters
  uint16_t* Pb = nullptr;    // BF16 copy
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* Z = nullptr;        // 3 x rows x 128 pre-activations
  uint16_t* A = nullptr;     // 3 x rows x 128 activations
  float* dZ = nullptr;       // 3 x rows x 128
  float* Y = nullptr;        // rows
  float* dY = nullptr;       // rows
  float* X = nullptr;        // rows x 4 (features built by mucaMlpPredictWeights)
  ~muca_mlp() {
    (void)hipFree(P);
    (void)hipFree(Pb);
    (void)hipFree(grad);
    (void)hipFree(m);
    (void)hipFree(v);
    (void)hipFree(Z);
    (void)hipFree(A);
    (void)hipFree(dZ);
    (void)hipFree(Y);
    (void)hipFree(dY);
    (void)hipFree(X);
  }
};

namespace {

template <typename T>
int alloc(T** p, size_t n) {
  *p = nullptr;
  MLP_TRY(hipMalloc((void**)p, (n ? n : 1) * sizeof(T)));
  return MUCA_OK;
}

int check(muca_mlp_t net, int rows) {
  if (!net) return fail(MUCA_EINVAL, "null network");
  if (rows < 1 || rows > net->max_rows)
    return fail(MUCA_EINVAL, "rows must be in [1, %d] (got %d)", net->max_rows, rows);
  return MUCA_OK;
}

unsigned tiles(int rows) { return (unsigned)((rows + 15) / 16); }

int forward(muca_mlp_t net, const float* X, int rows, hipStream_t s) {
  hipLaunchKernelGGL(muca::k_mlp_fwd, dim3(tiles(rows)), dim3(muca::kMlpHidden), 0, s, net->P,
                     net->Pb, X, rows, net->Z, net->A, net->Y);
  MLP_LAUNCHED();
  return MUCA_OK;
}

int gradient(muca_mlp_t net, const float* X, const float* T, int rows, float* loss,
             hipStream_t s) {
  if (int r = forward(net, X, rows, s)) return r;
  hipLaunchKernelGGL(muca::k_mlp_loss, dim3(1), dim3(256), 0, s, net->Y, T, rows, net->dY, loss);
  hipLaunchKernelGGL(muca::k_mlp_bwd, dim3(tiles(rows)), dim3(muca::kMlpHidden), 0, s, net->P,
                     net->Pb, net->Z, net->dY, rows, net->dZ);
  hipLaunchKernelGGL(muca::k_mlp_wgrad, dim3((muca::kMlpParams + 255) / 256), dim3(256), 0, s, X,
                     net->A, net->dZ, net->dY, rows, net->grad);
  MLP_LAUNCHED();
  return MUCA_OK;
}

}  // namespace

extern "C" {

int mucaMlpParamCount(void) { return muca::kMlpParams; }

int mucaMlpCreate(muca_mlp_t* out, int max_rows) {
  if (!out) return fail(MUCA_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_rows < 1 || max_rows > (1 << 22)) return fail(MUCA_EINVAL, "max_rows out of range");
  auto* n = new (std::nothrow) muca_mlp();
  if (!n) return fail(MUCA_ENOMEM, "host allocation failed");
  n->max_rows = max_rows;
  const size_t P = muca::kMlpParams, H = (size_t)3 * max_rows * muca::kMlpHidden;
  int r;
  if ((r = alloc(&n->P, P)) || (r = alloc(&n->Pb, P)) || (r = alloc(&n->grad, P)) ||
      (r = alloc(&n->m, P)) || (r = alloc(&n->v, P)) || (r = alloc(&n->Z, H)) ||
      (r = alloc(&n->A, H)) || (r = alloc(&n->dZ, H)) || (r = alloc(&n->Y, (size_t)max_rows)) ||
      (r = alloc(&n->dY, (size_t)max_rows)) ||
      (r = alloc(&n->X, (size_t)max_rows * muca::kMlpIn))) {
    delete n;
    return r;
  }
  *out = n;
  return MUCA_OK;
}

int mucaMlpDestroy(muca_mlp_t net) {
  if (!net) return MUCA_OK;
  (void)hipDeviceSynchronize();
  delete net;
  return MUCA_OK;
}

int mucaMlpSetParams(muca_mlp_t net, const float* params, int n) {
  if (!net || !params) return fail(MUCA_EINVAL, "null argument");
  if (n != muca::kMlpParams) return fail(MUCA_EINVAL, "expected %d parameters", muca::kMlpParams);
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return fail(MUCA_ENONFINITE, "parameter %d is not finite", i);
  MLP_TRY(hipMemcpy(net->P, params, sizeof(float) * n, hipMemcpyHostToDevice));
  MLP_TRY(hipMemset(net->m, 0, sizeof(float) * n));
  MLP_TRY(hipMemset(net->v, 0, sizeof(float) * n));
  net->step = 0;
  hipLaunchKernelGGL(muca::k_to_bf16, dim3((n + 255) / 256), dim3(256), 0, nullptr, net->P,
                     net->Pb, n);
  MLP_LAUNCHED();
  MLP_TRY(hipDeviceSynchronize());
  return MUCA_OK;
}

int mucaMlpGetParams(muca_mlp_t net, float* params, int n) {
  if (!net || !params) return fail(MUCA_EINVAL, "null argument");
  if (n != muca::kMlpParams) return fail(MUCA_EINVAL, "expected %d parameters", muca::kMlpParams);
  MLP_TRY(hipDeviceSynchronize());
  MLP_TRY(hipMemcpy(params, net->P, sizeof(float) * n, hipMemcpyDeviceToHost));
  return MUCA_OK;
}

int mucaMlpForward(muca_mlp_t net, const float* X, int rows, float* Y, void* stream) {
  if (int r = check(net, rows)) return r;
  if (!X || !Y) return fail(MUCA_EINVAL, "X and Y must not be NULL");
  hipStream_t s = (hipStream_t)stream;
  if (int r = forward(net, X, rows, s)) return r;
  MLP_TRY(hipMemcpyAsync(Y, net->Y, sizeof(float) * rows, hipMemcpyDeviceToDevice, s));
  return MUCA_OK;
}

int mucaMlpGradient(muca_mlp_t net, const float* X, const float* T, int rows, float* grad,
                    float* loss, void* stream) {
  if (int r = check(net, rows)) return r;
  if (!X || !T || !grad) return fail(MUCA_EINVAL, "X, T and grad must not be NULL");
  hipStream_t s = (hipStream_t)stream;
  if (int r = gradient(net, X, T, rows, loss, s)) return r;
  MLP_TRY(hipMemcpyAsync(grad, net->grad, sizeof(float) * muca::kMlpParams,
                         hipMemcpyDeviceToDevice, s));
  return MUCA_OK;
}

int mucaMlpTrainStep(muca_mlp_t net, const float* X, const float* T, int rows, float lr,
                     float* loss, void* stream) {
  if (int r = check(net, rows)) return r;
  if (!X || !T) return fail(MUCA_EINVAL, "X and T must not be NULL");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(MUCA_EINVAL, "lr must be positive");
  hipStream_t s = (hipStream_t)stream;
  if (int r = gradient(net, X, T, rows, loss, s)) return r;
  net->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - std::pow(b1, (float)net->step);
  const float c2 = 1.0f - std::pow(b2, (float)net->step);
  hipLaunchKernelGGL(muca::k_mlp_adam, dim3((muca::kMlpParams + 255) / 256), dim3(256), 0, s,
                     net->P, net->Pb, net->grad, net->m, net->v, lr, b1, b2, eps, c1, c2);
  MLP_LAUNCHED();
  return MUCA_OK;
}

int mucaMlpTableRows(muca_ctx ctx, int group, const double* lnW, float* X, float* T,
                     void* stream) {
  if (!ctx) return fail(MUCA_EINVAL, "null context");
  if (group < 0 || group >= ctx->ngroups) return fail(MUCA_EINVAL, "group out of range");
  if (!X || (T && !lnW)) return fail(MUCA_EINVAL, "X (and lnW with T) must not be NULL");
  const int nb = ctx->g[group].nbins;
  hipLaunchKernelGGL(muca::k_mlp_rows, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, ctx->d_groups, group, lnW, X, T);
  MLP_LAUNCHED();
  return MUCA_OK;
}

int mucaMlpPredictWeights(muca_mlp_t net, muca_ctx ctx, int group, double* lnW, void* stream) {
  if (!net || !ctx || !lnW) return fail(MUCA_EINVAL, "null argument");
  if (group < 0 || group >= ctx->ngroups) return fail(MUCA_EINVAL, "group out of range");
  const int nb = ctx->g[group].nbins;
  if (int r = check(net, nb)) return r;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(muca::k_mlp_rows, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s,
                     ctx->d_groups, group, nullptr, net->X, nullptr);
  MLP_LAUNCHED();
  if (int r = forward(net, net->X, nb, s)) return r;
  hipLaunchKernelGGL(muca::k_mlp_weights, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s,
                     ctx->d_groups, group, net->Y, lnW);
  MLP_LAUNCHED();
  return MUCA_OK;
}

}  // extern "C"
