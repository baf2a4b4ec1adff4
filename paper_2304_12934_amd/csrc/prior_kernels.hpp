// Launch interface of the prior and MBIR-update kernels (prior_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace nrk {

struct PriorArgs {
  float p, sigma, c, lambda;
  float w_face, w_edge, w_corner;
};

// grad += scale * dH/df over a [nz][n][n] volume; value (if not null) = H(f)
hipError_t launch_qggmrf(const float* f, float* grad, double* value, int nz, int n, const PriorArgs& pr,
                         float scale, hipStream_t st);
// s -= b
hipError_t launch_residual(float* s, const float* b, size_t count, hipStream_t st);
// s -= b and value = 1/2 sum (s - b)^2
hipError_t launch_residual_norm(float* s, const float* b, size_t count, double* value, hipStream_t st);
// restart test, momentum and the x/y update; state = {t, dot, nonfinite, restarts, beta, ...}
hipError_t launch_mbir_update(float* x, float* x_prev, float* y, const float* g, size_t count, float inv_L,
                              int nonneg, double* state, hipStream_t st);

}  // namespace nrk
