// qGGMRF prior gradient and the accelerated-gradient update for gfx950.
//
// Prior (Sec. 3, eqs. "reg2" and "reg3"): for voxel m and each of its 26
// neighbours n (voxels outside the volume dropped),
//   rho(u)  = u^2 / (c + |u|^(2-p)),           u = (f_m - f_n)/sigma
//   rho'(u) = u (2c + p|u|^(2-p)) / (c + |u|^(2-p))^2
//   dH/df_m = (2 lambda/sigma) sum_n w_mn rho'((f_m - f_n)/sigma)
// (H sums rho over ordered pairs; each unordered pair appears twice.)
//
// The stencil kernel stages a block of the volume with a one-voxel halo in
// LDS (the "shared memory caching" of the paper's Sec. 4.1, reorganised for
// 64-wide wavefronts), evaluates every unordered neighbour pair once and
// accumulates into the gradient in place (Sec. 4, gradients updated in place).
#include <hip/hip_runtime.h>

#include "prior_kernels.hpp"

namespace nrk {

namespace {

// Block of 64 x 8 x 8 voxels (x, y, z), 512 threads: thread (lx, ly) owns the
// z-column of 8 voxels.  The block stages its voxels with a one-voxel halo.
constexpr int TX = 64, TY = 8, TZ = 8;
constexpr int NT = TX * TY;
constexpr int FX = TX + 2, FY = TY + 2, FZ = TZ + 2;   // staged block (halo on every side)
constexpr int RX = TX + 2, RY = TY + 2, RZ = TZ + 1;   // pair terms: x, y in [-1, T], z in [-1, T)

__device__ __forceinline__ float pow_2mp(float a, float e) {   // a^e for a > 0
  return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(a));   // v_exp_f32, v_log_f32 (base 2)
}

// rho'(u) and, with VALUE, rho(u)
template <bool VALUE>
__device__ __forceinline__ float rho_prime(float u, const PriorArgs& pr, float& rho) {
  const float a = fabsf(u);
  if (a == 0.f) {
    rho = 0.f;
    return 0.f;
  }
  const float s = pow_2mp(a, 2.f - pr.p);
  const float inv = 1.f / (pr.c + s);
  if (VALUE) rho = a * a * inv;
  return u * (2.f * pr.c + pr.p * s) * inv * inv;
}

// The 13 neighbour offsets (dz, dy, dx) that are lexicographically positive;
// the other 13 are their negations.
__constant__ int8_t kDirs[13][3] = {{0, 0, 1},  {0, 1, -1},  {0, 1, 0},  {0, 1, 1},  {1, -1, -1},
                                    {1, -1, 0}, {1, -1, 1}, {1, 0, -1}, {1, 0, 0},  {1, 0, 1},
                                    {1, 1, -1}, {1, 1, 0},  {1, 1, 1}};

}  // namespace

// Each unordered neighbour pair (m, m + d) is evaluated once: r_d(m) =
// w_d rho'((f_m - f_{m+d})/sigma) enters voxel m with + and voxel m + d with -
// (rho' is odd).  Per direction the block evaluates r_d on its voxels and on
// their one-voxel shift by -d, in LDS, then every voxel adds r_d(m) - r_d(m-d).
template <bool VALUE, bool INTERIOR>
__device__ __forceinline__ void qggmrf_block(const float* __restrict__ f, float* __restrict__ grad,
                                             double* __restrict__ value, int nz, int n, const PriorArgs& pr,
                                             float scale, float* F, float* R, double* red) {
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
  const size_t plane = size_t(n) * n;
  for (int i = tid; i < FX * FY * FZ; i += NT) {
    const int bx = i % FX, by = (i / FX) % FY, bz = i / (FX * FY);
    const int x = x0 + bx - 1, y = y0 + by - 1, z = z0 + bz - 1;
    float v = 0.f;
    if (INTERIOR || (x >= 0 && x < n && y >= 0 && y < n && z >= 0 && z < nz))
      v = f[size_t(z) * plane + size_t(y) * n + x];
    F[i] = v;
  }
  __syncthreads();
  const float inv_sigma = 1.f / pr.sigma;
  const int lx = tid % TX, ly = tid / TX;
  float acc[TZ];
#pragma unroll
  for (int z = 0; z < TZ; ++z) acc[z] = 0.f;
  float hsum = 0.f;
  auto inside = [&](int bz, int by, int bx) {   // block-local coordinates, -1..T
    const int x = x0 + bx, y = y0 + by, z = z0 + bz;
    return x >= 0 && x < n && y >= 0 && y < n && z >= 0 && z < nz;
  };
#pragma unroll 1
  for (int k = 0; k < 13; ++k) {
    const int dz = kDirs[k][0], dy = kDirs[k][1], dx = kDirs[k][2];
    const int d2 = dz * dz + dy * dy + dx * dx;
    const float w = d2 == 1 ? pr.w_face : (d2 == 2 ? pr.w_edge : pr.w_corner);
    // region: the block and its shift by -d
    const int xa = dx > 0 ? -1 : 0, xb = dx < 0 ? TX + 1 : TX;
    const int ya = dy > 0 ? -1 : 0, yb = dy < 0 ? TY + 1 : TY;
    const int za = dz > 0 ? -1 : 0;
    const int ex = xb - xa, ey = yb - ya, ez = TZ - za;
    for (int i = tid; i < ex * ey * ez; i += NT) {
      const int bx = xa + i % ex, by = ya + (i / ex) % ey, bz = za + i / (ex * ey);
      float r = 0.f, rh = 0.f;
      if (INTERIOR || (inside(bz, by, bx) && inside(bz + dz, by + dy, bx + dx))) {
        const float fm = F[(bz + 1) * FY * FX + (by + 1) * FX + (bx + 1)];
        const float fn = F[(bz + 1 + dz) * FY * FX + (by + 1 + dy) * FX + (bx + 1 + dx)];
        r = w * rho_prime<VALUE>((fm - fn) * inv_sigma, pr, rh);
        // the value counts each ordered pair: 2 w rho per unordered pair, once (at its owned m)
        if (VALUE && bx >= 0 && bx < TX && by >= 0 && by < TY && bz >= 0) hsum += 2.f * w * rh;
      }
      R[(bz + 1) * RY * RX + (by + 1) * RX + (bx + 1)] = r;
    }
    __syncthreads();
#pragma unroll
    for (int z = 0; z < TZ; ++z)
      acc[z] += R[(z + 1) * RY * RX + (ly + 1) * RX + (lx + 1)] -
                R[(z + 1 - dz) * RY * RX + (ly + 1 - dy) * RX + (lx + 1 - dx)];
    __syncthreads();
  }
  const float gscale = scale * 2.f * pr.lambda * inv_sigma;
  const int x = x0 + lx, y = y0 + ly;
  if (x < n && y < n) {
#pragma unroll
    for (int z = 0; z < TZ; ++z)
      if (z0 + z < nz) grad[size_t(z0 + z) * plane + size_t(y) * n + x] += gscale * acc[z];
  }
  if (VALUE) {
    red[tid] = double(hsum);
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) atomicAdd(value, double(pr.lambda) * red[0]);
  }
}

template <bool VALUE>
__global__ __launch_bounds__(NT) void k_qggmrf(const float* __restrict__ f, float* __restrict__ grad,
                                               double* __restrict__ value, int nz, int n, PriorArgs pr,
                                               float scale) {
  __shared__ float F[FZ * FY * FX];
  __shared__ float R[RZ * RY * RX];
  __shared__ double red[NT];
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
  // interior block: the block and its halo lie inside the volume
  const bool interior = x0 >= 1 && x0 + TX + 1 <= n && y0 >= 1 && y0 + TY + 1 <= n && z0 >= 1 && z0 + TZ + 1 <= nz;
  if (interior) qggmrf_block<VALUE, true>(f, grad, value, nz, n, pr, scale, F, R, red);
  else qggmrf_block<VALUE, false>(f, grad, value, nz, n, pr, scale, F, R, red);
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
  if (value) hipLaunchKernelGGL(k_qggmrf<true>, grid, dim3(NT), 0, st, f, grad, value, nz, n, pr, scale);
  else hipLaunchKernelGGL(k_qggmrf<false>, grid, dim3(NT), 0, st, f, grad, value, nz, n, pr, scale);
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
