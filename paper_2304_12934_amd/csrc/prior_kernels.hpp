// Launch interface of the prior and MBIR-update kernels (prior_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nrk {

struct PriorArgs {
  float p, sigma, c, lambda;
  float w_face, w_edge, w_corner;
};

// grad += scale * dH/df over a [nz][n][n] volume (grad = scale * dH/df when
// accumulate is false and value is null); value (if not null) = H(f)
hipError_t launch_qggmrf(const float* f, float* grad, double* value, int nz, int n, const PriorArgs& pr,
                         float scale, hipStream_t st, bool accumulate = true);
// s -= b
hipError_t launch_residual(float* s, const float* b, size_t count, hipStream_t st);
// s -= b and value = 1/2 sum (s - b)^2
hipError_t launch_residual_norm(float* s, const float* b, size_t count, double* value, hipStream_t st);
// Slots of the float64 MBIR state array (kStCount doubles on the device).
enum {
  kStT = 0,          // momentum parameter t_k
  kStDot,            // <g, x' - x> of the last step
  kStNonfinite,      // 1 once a NaN/Inf appeared
  kStRestarts,       // momentum restarts so far (gradient test and rejected steps)
  kStBeta,           // momentum coefficient of the last step
  kStPhiX,           // objective at x (monotone steps)
  kStPhiKnown,       // 1 once kStPhiX holds a value
  kStPhiData,        // data term at the last candidate
  kStPhiPrior,       // prior at the last candidate
  kStAccepted,       // 1 if the last candidate was accepted
  kStRejects,        // candidates rejected by the monotone test
  kStCount = 16
};

// restart test (restart != 0), momentum and the x/y update; with add_x_prev
// the gradient is g + x_prev (a part computed into x_prev, whose contents the
// update overwrites), stored back into g first
hipError_t launch_mbir_update(float* x, float* x_prev, float* y, float* g, size_t count, float inv_L,
                              int nonneg, int restart, double* state, hipStream_t st, bool add_x_prev = false);
// monotone step, first half: the restart dot product and the candidate
// x' = y - g/L (clamped when nonneg) into x_prev
hipError_t launch_mbir_candidate(const float* x, float* x_prev, const float* y, const float* g, size_t count,
                                 float inv_L, int nonneg, double* state, hipStream_t st);
// monotone step, second half (the candidate's objective already in the
// state): accept or reject, momentum, x/x_prev/y update
hipError_t launch_mbir_finish_monotone(float* x, float* x_prev, float* y, size_t count, int restart, double* state,
                                       hipStream_t st);
// t = 1, every other slot 0
hipError_t launch_mbir_state_init(double* state, hipStream_t st);
// y = x + beta (x - x_prev), beta from the state (the last finalised step)
hipError_t launch_mbir_extrapolate(float* y, const float* x, const float* x_prev, size_t count, const double* state,
                                   hipStream_t st);
// state's <g, x' - x> += that of these elements, with g <- g + gp when gp
// is given and x' = y - g/L (clamped when nonneg) stored into cand
hipError_t launch_mbir_dot_accumulate(const float* x, const float* y, float* g, const float* gp, size_t count,
                                      float inv_L, int nonneg, double* state, float* cand, hipStream_t st);
// restart test on the accumulated dot product, then t and beta
hipError_t launch_mbir_finalize(double* state, int restart, hipStream_t st);
// v[i] = uniform in [-1, 1) from (seed, first + i); v[i] = value
hipError_t launch_fill_random(float* v, size_t count, uint64_t seed, uint64_t first, hipStream_t st);
hipError_t launch_fill_value(float* v, size_t count, float value, hipStream_t st);
// *out = 1/2 sum v^2 (float64); *p = v
hipError_t launch_half_sum_squares(const float* v, size_t count, double* out, hipStream_t st);
hipError_t launch_set_double(double* p, double v, hipStream_t st);
// *ss = sum w^2 (float64), then v = w / sqrt(*ss)
hipError_t launch_normalize(float* v, const float* w, size_t count, double* ss, hipStream_t st);

}  // namespace nrk
