// muca_mlp.hip -- kernels of the learned initial weights: a small MLP
// (d, L, rho, E/E_lo) -> (lnW(E) - lnW(E_lo)) / N, trained on converged weight
// tables of the MUCA iteration and used to propose initial weights for a new
// lattice (not part of the paper; the plain recursion from flat weights is
// its fallback).
//
// Network: 4 -> 128 -> 128 -> 128 -> 1, SiLU hidden activations.  Hidden
// layers use BF16 weights (round-to-nearest-even copies of FP32 master
// weights) and BF16 activations with FP32 accumulation; the first layer
// reads the FP32 inputs, the output layer has FP32 weights.  Training: mean
// squared error, full batch, Adam on the FP32 master weights.  Gradients pass
// straight through the BF16 rounding of activations.
//
// Parameter layout (FP32, flat): W1[128][4] b1[128] W2[128][128] b2[128]
// W3[128][128] b3[128] W4[128] b4[1].
#include "muca_mlp.h"

namespace muca {

namespace {

constexpr int kTile = 16;  // rows per block in the row-parallel kernels

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }

__device__ __forceinline__ float silu_grad(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

}  // namespace

// FP32 -> BF16, round to nearest, ties to even (NaN kept quiet).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__global__ void k_to_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    dst[i] = to_bf16(src[i]);
}

// Forward pass of rows [tile * kTile, ...): thread j = hidden unit j.
// Saves pre-activations Z (FP32) and activations A (BF16) of the three hidden
// layers for the backward pass, and the outputs Y.
__global__ void __launch_bounds__(kMlpHidden) k_mlp_fwd(const float* __restrict__ P,
                                                        const uint16_t* __restrict__ Pb,
                                                        const float* __restrict__ X, int rows,
                                                        float* __restrict__ Z,
                                                        uint16_t* __restrict__ A,
                                                        float* __restrict__ Y) {
  __shared__ float act[kTile][kMlpHidden];
  __shared__ float red[kTile][kMlpHidden];
  const int j = threadIdx.x;
  const int r0 = blockIdx.x * kTile;
  const int nr = min(kTile, rows - r0);
  // layer 1: FP32 inputs, BF16 weights
  for (int r = 0; r < nr; ++r) {
    const float* x = X + (size_t)(r0 + r) * kMlpIn;
    float z = P[kOffB1 + j];
    for (int i = 0; i < kMlpIn; ++i) z += from_bf16(Pb[kOffW1 + j * kMlpIn + i]) * x[i];
    Z[((size_t)0 * rows + r0 + r) * kMlpHidden + j] = z;
    const uint16_t a = to_bf16(silu(z));
    A[((size_t)0 * rows + r0 + r) * kMlpHidden + j] = a;
    act[r][j] = from_bf16(a);
  }
  __syncthreads();
  // layers 2, 3: BF16 weights and activations, FP32 accumulation
  for (int l = 1; l < 3; ++l) {
    const int offW = l == 1 ? kOffW2 : kOffW3;
    const int offB = l == 1 ? kOffB2 : kOffB3;
    float acc[kTile];
    for (int r = 0; r < kTile; ++r) acc[r] = P[offB + j];
    for (int i = 0; i < kMlpHidden; ++i) {
      const float w = from_bf16(Pb[offW + j * kMlpHidden + i]);
      for (int r = 0; r < kTile; ++r) acc[r] += w * act[r][i];
    }
    __syncthreads();
    for (int r = 0; r < nr; ++r) {
      Z[((size_t)l * rows + r0 + r) * kMlpHidden + j] = acc[r];
      const uint16_t a = to_bf16(silu(acc[r]));
      A[((size_t)l * rows + r0 + r) * kMlpHidden + j] = a;
      act[r][j] = from_bf16(a);
    }
    __syncthreads();
  }
  // output head: FP32 weights, FP32 accumulation (tree over the 128 units)
  for (int r = 0; r < kTile; ++r) red[r][j] = (r < nr) ? P[kOffW4 + j] * act[r][j] : 0.f;
  __syncthreads();
  for (int s = kMlpHidden / 2; s > 0; s >>= 1) {
    if (j < s)
      for (int r = 0; r < kTile; ++r) red[r][j] += red[r][j + s];
    __syncthreads();
  }
  if (j < nr) Y[r0 + j] = red[j][0] + P[kOffB4];
}

// dL/dy for the mean squared error and the loss itself (one block, fixed
// summation order).
__global__ void __launch_bounds__(256) k_mlp_loss(const float* __restrict__ Y,
                                                  const float* __restrict__ T, int rows,
                                                  float* __restrict__ dY,
                                                  float* __restrict__ loss) {
  __shared__ float part[256];
  float s = 0.f;
  for (int r = threadIdx.x; r < rows; r += blockDim.x) {
    const float e = Y[r] - T[r];
    dY[r] = 2.0f * e / (float)rows;
    s += e * e;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) part[threadIdx.x] += part[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = part[0] / (float)rows;
}

// Backward through the activations: dZ of the three hidden layers per row.
__global__ void __launch_bounds__(kMlpHidden) k_mlp_bwd(const float* __restrict__ P,
                                                        const uint16_t* __restrict__ Pb,
                                                        const float* __restrict__ Z,
                                                        const float* __restrict__ dY, int rows,
                                                        float* __restrict__ dZ) {
  __shared__ float dz[kTile][kMlpHidden];
  const int j = threadIdx.x;
  const int r0 = blockIdx.x * kTile;
  const int nr = min(kTile, rows - r0);
  for (int r = 0; r < nr; ++r) {
    const float z = Z[((size_t)2 * rows + r0 + r) * kMlpHidden + j];
    const float g = dY[r0 + r] * P[kOffW4 + j] * silu_grad(z);
    dZ[((size_t)2 * rows + r0 + r) * kMlpHidden + j] = g;
    dz[r][j] = g;
  }
  __syncthreads();
  for (int l = 2; l >= 1; --l) {  // dA_{l-1} = W_l^T dZ_l
    const int offW = l == 2 ? kOffW3 : kOffW2;
    float acc[kTile];
    for (int r = 0; r < kTile; ++r) acc[r] = 0.f;
    for (int o = 0; o < kMlpHidden; ++o) {
      const float w = from_bf16(Pb[offW + o * kMlpHidden + j]);
      for (int r = 0; r < kTile; ++r) acc[r] += w * dz[r][o];
    }
    __syncthreads();
    for (int r = 0; r < nr; ++r) {
      const float z = Z[((size_t)(l - 1) * rows + r0 + r) * kMlpHidden + j];
      const float g = acc[r] * silu_grad(z);
      dZ[((size_t)(l - 1) * rows + r0 + r) * kMlpHidden + j] = g;
      dz[r][j] = g;
    }
    __syncthreads();
  }
}

// Parameter gradients: one thread per parameter, rows summed in order
// (deterministic).
__global__ void __launch_bounds__(256) k_mlp_wgrad(const float* __restrict__ X,
                                                   const uint16_t* __restrict__ A,
                                                   const float* __restrict__ dZ,
                                                   const float* __restrict__ dY, int rows,
                                                   float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  float s = 0.f;
  if (p < kOffB1) {  // W1[j][i]
    const int j = p / kMlpIn, i = p % kMlpIn;
    for (int r = 0; r < rows; ++r) s += dZ[(size_t)r * kMlpHidden + j] * X[(size_t)r * kMlpIn + i];
  } else if (p < kOffW2) {
    const int j = p - kOffB1;
    for (int r = 0; r < rows; ++r) s += dZ[(size_t)r * kMlpHidden + j];
  } else if (p < kOffB2 || (p >= kOffW3 && p < kOffB3)) {  // W2 or W3
    const int l = p < kOffB2 ? 1 : 2;
    const int q = p - (l == 1 ? kOffW2 : kOffW3);
    const int j = q / kMlpHidden, i = q % kMlpHidden;
    const float* dz = dZ + (size_t)l * rows * kMlpHidden;
    const uint16_t* a = A + (size_t)(l - 1) * rows * kMlpHidden;
    for (int r = 0; r < rows; ++r)
      s += dz[(size_t)r * kMlpHidden + j] * from_bf16(a[(size_t)r * kMlpHidden + i]);
  } else if (p < kOffW3 || (p >= kOffB3 && p < kOffW4)) {  // b2 or b3
    const int l = p < kOffW3 ? 1 : 2;
    const int j = p - (l == 1 ? kOffB2 : kOffB3);
    const float* dz = dZ + (size_t)l * rows * kMlpHidden;
    for (int r = 0; r < rows; ++r) s += dz[(size_t)r * kMlpHidden + j];
  } else if (p < kOffB4) {  // W4[j]
    const int j = p - kOffW4;
    const uint16_t* a = A + (size_t)2 * rows * kMlpHidden;
    for (int r = 0; r < rows; ++r) s += dY[r] * from_bf16(a[(size_t)r * kMlpHidden + j]);
  } else {
    for (int r = 0; r < rows; ++r) s += dY[r];
  }
  grad[p] = s;
}

// Adam on the FP32 master weights, then the BF16 working copy.
__global__ void __launch_bounds__(256) k_mlp_adam(float* __restrict__ P, uint16_t* __restrict__ Pb,
                                                  const float* __restrict__ grad,
                                                  float* __restrict__ m, float* __restrict__ v,
                                                  float lr, float b1, float b2, float eps,
                                                  float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.0f - b1) * g;
  const float vv = b2 * v[p] + (1.0f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float th = P[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  P[p] = th;
  Pb[p] = to_bf16(th);
}

// Features of the bins of one group: x = ((d - 2.5) 2, L / 64, 10 rho, E / E_lo).
__device__ __forceinline__ void features(const GroupDesc& g, int b, float* x) {
  const int E = g.e_lo + b;
  x[0] = ((float)g.d - 2.5f) * 2.0f;
  x[1] = (float)g.L / 64.0f;
  x[2] = 10.0f * (float)g.N / (float)g.V;
  x[3] = g.e_lo != 0 ? (float)E / (float)g.e_lo : 0.0f;
}

__global__ void k_mlp_rows(const GroupDesc* __restrict__ groups, int gi,
                           const double* __restrict__ lnW, float* __restrict__ X,
                           float* __restrict__ T) {
  const GroupDesc g = groups[gi];
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= g.nbins) return;
  features(g, b, X + (size_t)b * kMlpIn);
  if (T) {
    const double* lw = lnW + g.bin_off;
    T[b] = (float)((lw[b] - lw[0]) / (double)g.N);
  }
}

// lnW of a group from the network outputs: N y(E), shifted to lnW(e_hi) = 0.
__global__ void k_mlp_weights(const GroupDesc* __restrict__ groups, int gi,
                              const float* __restrict__ Y, double* __restrict__ lnW) {
  const GroupDesc g = groups[gi];
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= g.nbins) return;
  const double top = (double)g.N * (double)Y[g.nbins - 1];
  lnW[g.bin_off + b] = (double)g.N * (double)Y[b] - top;
}

}  // namespace muca
