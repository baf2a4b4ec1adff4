// qGGMRF prior gradient and the accelerated-gradient update for gfx950.
//
// Prior (Sec. 3, eqs. "reg2" and "reg3"): for voxel m and each of its 26
// neighbours n (voxels outside the volume dropped),
//   rho(u)  = u^2 / (c + |u|^(2-p)),           u = (f_m - f_n)/sigma
//   rho'(u) = u (2c + p|u|^(2-p)) / (c + |u|^(2-p))^2
//   dH/df_m = (2 lambda/sigma) sum_n w_mn rho'((f_m - f_n)/sigma)
// (H sums rho over ordered pairs; each unordered pair appears twice.)
//
// The stencil kernel stages a (TZ+2) x (TY+2) x (TX+2) block of the volume in
// LDS (the "shared memory caching" of the paper's Sec. 4.1, reorganised for
// 64-wide wavefronts) and accumulates into the gradient in place (Sec. 4,
// gradients updated in place).
#include <hip/hip_runtime.h>

#include "prior_kernels.hpp"

namespace nrk {

namespace {

constexpr int TX = 64, TY = 4, TZ = 4;   // 1024 voxels per block, 256 threads x 4 z-planes

__device__ __forceinline__ float pow_2mp(float a, float e) {   // a^e for a > 0
  return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(a));   // v_exp_f32, v_log_f32 (base 2)
}

// rho'(u) and (optionally) rho(u)
__device__ __forceinline__ float rho_prime(float u, const PriorArgs& pr, float& rho) {
  const float a = fabsf(u);
  if (a == 0.f) {
    rho = 0.f;
    return 0.f;
  }
  const float s = pow_2mp(a, 2.f - pr.p);
  const float den = pr.c + s;
  const float inv = 1.f / den;
  rho = a * a * inv;
  return u * (2.f * pr.c + pr.p * s) * inv * inv;
}

}  // namespace

__global__ __launch_bounds__(256) void k_qggmrf(const float* __restrict__ f, float* __restrict__ grad,
                                                double* __restrict__ value, int nz, int n, PriorArgs pr,
                                                float scale) {
  __shared__ float blk[TZ + 2][TY + 2][TX + 2];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
  const size_t plane = size_t(n) * n;
  // stage the block with a one-voxel halo; outside the volume -> NaN marker
  constexpr int BX = TX + 2, BY = TY + 2, BZ = TZ + 2;
  for (int i = tid; i < BX * BY * BZ; i += 256) {
    const int bx = i % BX, by = (i / BX) % BY, bz = i / (BX * BY);
    const int x = x0 + bx - 1, y = y0 + by - 1, z = z0 + bz - 1;
    float v = __int_as_float(0x7fc00000);
    if (x >= 0 && x < n && y >= 0 && y < n && z >= 0 && z < nz) v = f[size_t(z) * plane + size_t(y) * n + x];
    blk[bz][by][bx] = v;
  }
  __syncthreads();
  const float inv_sigma = 1.f / pr.sigma;
  const float gscale = scale * 2.f * pr.lambda * inv_sigma;
  double hsum = 0.0;
  const int lx = tid % TX, ly = tid / TX;   // 64 x 4 threads, loop over TZ planes
  for (int lz = 0; lz < TZ; ++lz) {
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    if (x >= n || y >= n || z >= nz) continue;
    const float fm = blk[lz + 1][ly + 1][lx + 1];
    float g = 0.f, h = 0.f;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (dx == 0 && dy == 0 && dz == 0) continue;
          const float fn = blk[lz + 1 + dz][ly + 1 + dy][lx + 1 + dx];
          if (fn != fn) continue;   // neighbour outside the volume
          const int d2 = dx * dx + dy * dy + dz * dz;
          const float w = d2 == 1 ? pr.w_face : (d2 == 2 ? pr.w_edge : pr.w_corner);
          float r;
          const float rp = rho_prime((fm - fn) * inv_sigma, pr, r);
          g = fmaf(w, rp, g);
          h = fmaf(w, r, h);
        }
    grad[size_t(z) * plane + size_t(y) * n + x] += gscale * g;
    hsum += double(h);
  }
  if (value) {
    red[tid] = hsum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) atomicAdd(value, double(pr.lambda) * red[0]);
  }
}

__global__ void k_set_double(double* p, double v) { *p = v; }

// r = s - b (the residual of the data term), in place in s
__global__ void k_residual(float* __restrict__ s, const float* __restrict__ b, size_t count) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += size_t(gridDim.x) * blockDim.x)
    s[i] -= b[i];
}

// r = s - b in place and value += 1/2 sum r^2 (float64 block sums)
__global__ __launch_bounds__(256) void k_residual_norm(float* __restrict__ s, const float* __restrict__ b,
                                                       size_t count, double* value) {
  __shared__ double red[256];
  double acc = 0.0;
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256) {
    const float r = s[i] - b[i];
    s[i] = r;
    acc += double(r) * double(r);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(value, 0.5 * red[0]);
}

// <g, x' - x> with x' = y - g/L (clamped at 0 when nonneg); non-finite flag
__global__ __launch_bounds__(256) void k_mbir_dot(const float* __restrict__ x, const float* __restrict__ y,
                                                  const float* __restrict__ g, size_t count, float inv_L,
                                                  int nonneg, double* state) {
  __shared__ double red[256];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double acc = 0.0;
  int nf = 0;
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256) {
    const float gi = g[i];
    float xn = y[i] - inv_L * gi;
    if (nonneg) xn = fmaxf(xn, 0.f);
    acc += double(gi) * double(xn - x[i]);
    if (!isfinite(gi) || !isfinite(xn)) nf = 1;
  }
  if (nf) bad = 1;
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&state[1], red[0]);
    if (bad) state[2] = 1.0;
  }
}

// restart test and momentum: t <- 1 if <g, x'-x> > 0; t' = (1+sqrt(1+4t^2))/2; beta = (t-1)/t'
__global__ void k_mbir_finalize(double* state) {
  double t = state[0];
  if (state[1] > 0.0) {
    t = 1.0;
    state[3] += 1.0;
  }
  const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
  state[4] = (t - 1.0) / tn;
  state[0] = tn;
}

// x' = y - g/L; y <- x' + beta (x' - x); x_prev <- x; x <- x'
__global__ __launch_bounds__(256) void k_mbir_update(float* __restrict__ x, float* __restrict__ x_prev,
                                                     float* __restrict__ y, const float* __restrict__ g,
                                                     size_t count, float inv_L, int nonneg,
                                                     const double* __restrict__ state) {
  const float beta = float(state[4]);
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256) {
    float xn = y[i] - inv_L * g[i];
    if (nonneg) xn = fmaxf(xn, 0.f);
    const float xo = x[i];
    y[i] = xn + beta * (xn - xo);
    x_prev[i] = xo;
    x[i] = xn;
  }
}

hipError_t launch_qggmrf(const float* f, float* grad, double* value, int nz, int n, const PriorArgs& pr,
                         float scale, hipStream_t st) {
  if (value) hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, value, 0.0);
  const dim3 grid((n + TX - 1) / TX, (n + TY - 1) / TY, (nz + TZ - 1) / TZ);
  hipLaunchKernelGGL(k_qggmrf, grid, dim3(256), 0, st, f, grad, value, nz, n, pr, scale);
  return hipGetLastError();
}

hipError_t launch_residual(float* s, const float* b, size_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_residual, dim3(2048), dim3(256), 0, st, s, b, count);
  return hipGetLastError();
}

hipError_t launch_residual_norm(float* s, const float* b, size_t count, double* value, hipStream_t st) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, value, 0.0);
  hipLaunchKernelGGL(k_residual_norm, dim3(2048), dim3(256), 0, st, s, b, count, value);
  return hipGetLastError();
}

hipError_t launch_mbir_update(float* x, float* x_prev, float* y, const float* g, size_t count, float inv_L,
                              int nonneg, double* state, hipStream_t st) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, state + 1, 0.0);
  hipLaunchKernelGGL(k_mbir_dot, dim3(2048), dim3(256), 0, st, x, y, g, count, inv_L, nonneg, state);
  hipLaunchKernelGGL(k_mbir_finalize, dim3(1), dim3(1), 0, st, state);
  hipLaunchKernelGGL(k_mbir_update, dim3(4096), dim3(256), 0, st, x, x_prev, y, g, count, inv_L, nonneg, state);
  return hipGetLastError();
}

}  // namespace nrk
