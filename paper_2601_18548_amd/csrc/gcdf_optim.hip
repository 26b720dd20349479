// Adam update of a flat FP32 parameter vector (the training form's optimiser).
//
//   m = b1 m + (1 - b1) g,   v = b2 v + (1 - b2) g^2,
//   p -= (lr / (1 - b1^t)) * m / (sqrt(v) / sqrt(1 - b2^t) + eps)
//
// in the operation order of torch.optim.Adam (no weight decay, no amsgrad), one
// thread per element, grid over the whole vector (a single large tensor would
// otherwise run on a handful of workgroups).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "gcdf_internal.h"

namespace gcdf {
namespace {

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr_corr, float b1, float b2, float inv_sqrt_bc2,
                            float eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float denom = sqrtf(vi) * inv_sqrt_bc2 + eps;
  p[i] = p[i] - lr_corr * (mi / denom);
}

}  // namespace

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int64_t step, hipStream_t s) {
  const double bc1 = 1.0 - std::pow((double)b1, (double)step);
  const double bc2 = 1.0 - std::pow((double)b2, (double)step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n,
                     (float)(lr / bc1), b1, b2, (float)(1.0 / std::sqrt(bc2)), eps);
  return hipGetLastError();
}

}  // namespace gcdf
