// muca_mlp.h -- sizes, parameter layout and kernels of the learned initial
// weights network (see muca_mlp.hip).
#pragma once

#include "muca_device.h"

namespace muca {

constexpr int kMlpIn = 4;
constexpr int kMlpHidden = 128;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHidden * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpHidden * kMlpHidden;
constexpr int kOffW4 = kOffB3 + kMlpHidden;
constexpr int kOffB4 = kOffW4 + kMlpHidden;
constexpr int kMlpParams = kOffB4 + 1;

__global__ void k_to_bf16(const float* src, uint16_t* dst, int n);
__global__ void k_mlp_fwd(const float* P, const uint16_t* Pb, const float* X, int rows, float* Z,
                          uint16_t* A, float* Y);
__global__ void k_mlp_loss(const float* Y, const float* T, int rows, float* dY, float* loss);
__global__ void k_mlp_bwd(const float* P, const uint16_t* Pb, const float* Z, const float* dY,
                          int rows, float* dZ);
__global__ void k_mlp_wgrad(const float* X, const uint16_t* A, const float* dZ, const float* dY,
                            int rows, float* grad);
__global__ void k_mlp_adam(float* P, uint16_t* Pb, const float* grad, float* m, float* v, float lr,
                           float b1, float b2, float eps, float c1, float c2);
__global__ void k_mlp_rows(const GroupDesc* groups, int gi, const double* lnW, float* X,
                           float* T);
__global__ void k_mlp_weights(const GroupDesc* groups, int gi, const float* Y, double* lnW);

}  // namespace muca
