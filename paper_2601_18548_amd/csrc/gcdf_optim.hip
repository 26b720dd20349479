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
                            float* __restrict__ v, int64_t n, AdamConsts a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  adam_update(p, g, m, v, i, a);
}

}  // namespace

AdamConsts AdamConsts::make(float lr, float b1, float b2, float eps, int64_t step) {
  const double bc1 = 1.0 - std::pow((double)b1, (double)step);
  const double bc2 = 1.0 - std::pow((double)b2, (double)step);
  return AdamConsts{(float)(lr / bc1), b1, b2, (float)(1.0 / std::sqrt(bc2)), eps};
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int64_t step, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n,
                     AdamConsts::make(lr, b1, b2, eps, step));
  return hipGetLastError();
}

}  // namespace gcdf
