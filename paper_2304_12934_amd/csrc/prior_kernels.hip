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

#include <algorithm>

#include "prior_kernels.hpp"

namespace nrk {

namespace {

// Block of 64 x 8 x 8 voxels (x, y, z), 512 threads: thread (lx, ly) owns the
// z-column of 8 voxels (one wavefront per x-row).  The block stages its voxels
// with a one-voxel halo in F; staged index of block-local (x, y, z), each in
// [-1, T], is (z+1)*FP + (y+1)*FX + (x+1).  The pair terms of one direction go
// to R (same indexing, z in [-1, TZ)), double-buffered across directions.
constexpr int TX = 64, TY = 8, TZ = 8;
constexpr int NT = TX * TY;
constexpr int FX = TX + 2, FY = TY + 2, FZ = TZ + 2;
constexpr int FP = FX * FY;
constexpr int RSZ = (TZ + 1) * FP;

__device__ __forceinline__ float pow_2mp(float a, float e) {   // a^e for a > 0
  return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(a));   // v_exp_f32, v_log_f32 (base 2)
}

// w rho'(u) and, with VALUE, w rho(u).  s = |u|^(2-p) is taken as 0 at u = 0
// (a select, no branch); both results are 0 there whatever s is.
template <bool VALUE>
__device__ __forceinline__ float rho_prime(float u, const PriorArgs& pr, float w, float& rho) {
  const float a = fabsf(u);
  const float s = a > 0.f ? pow_2mp(a, 2.f - pr.p) : 0.f;
  const float inv = __builtin_amdgcn_rcpf(pr.c + s);
  if (VALUE) rho = w * a * a * inv;
  return w * u * fmaf(pr.p, s, 2.f * pr.c) * inv * inv;
}

struct BlockCtx {
  int x0, y0, z0, n, nz, lx, ly, tid;
  float inv_sigma;
  __device__ __forceinline__ bool inside(int bx, int by, int bz) const {   // block-local coordinates
    const int x = x0 + bx, y = y0 + by, z = z0 + bz;
    return x >= 0 && x < n && y >= 0 && y < n && z >= 0 && z < nz;
  }
};

__device__ __forceinline__ constexpr int fidx(int bx, int by, int bz) { return (bz + 1) * FP + (by + 1) * FX + (bx + 1); }

// r_d at block-local m = (bx, by, bz): w rho'((f_m - f_{m+d})/sigma), 0 when m
// or m + d lies outside the volume.
template <bool VALUE, bool INTERIOR, int DZ, int DY, int DX>
__device__ __forceinline__ float pair_term(const BlockCtx& b, const float* F, float fm, float fn, int bx, int by,
                                           int bz, const PriorArgs& pr, float w, float& rho) {
  if (!INTERIOR && !(b.inside(bx, by, bz) && b.inside(bx + DX, by + DY, bz + DZ))) {
    rho = 0.f;
    return 0.f;
  }
  return rho_prime<VALUE>((fm - fn) * b.inv_sigma, pr, w, rho);
}

// One of the 13 lexicographically positive offsets d = (DZ, DY, DX).  Each
// unordered pair (m, m + d) is evaluated once: r_d(m) enters voxel m with +
// and voxel m + d with - (rho' is odd), so voxel m gathers r_d(m) - r_d(m - d).
// The terms r_d(m - d) of the block's own voxels come from the thread that owns
// column m - d or, off the block, from the halo rows evaluated here.
template <bool VALUE, bool INTERIOR, int DZ, int DY, int DX>
__device__ __forceinline__ void direction(const BlockCtx& b, const float* F, float* R, const float (&fc)[FZ],
                                          float (&acc)[TZ], float& hsum, const PriorArgs& pr) {
  constexpr int d2 = DZ * DZ + DY * DY + DX * DX;
  const float w = d2 == 1 ? pr.w_face : (d2 == 2 ? pr.w_edge : pr.w_corner);
  constexpr int ZLO = -DZ;
  float r[TZ + 1];   // r[z + 1] for z in [ZLO, TZ)
#pragma unroll
  for (int z = ZLO; z < TZ; ++z) {
    const float fn = (DX == 0 && DY == 0) ? fc[z + 1 + DZ] : F[fidx(b.lx + DX, b.ly + DY, z + DZ)];
    float rho;
    r[z + 1] = pair_term<VALUE, INTERIOR, DZ, DY, DX>(b, F, fc[z + 1], fn, b.lx, b.ly, z, pr, w, rho);
    if (VALUE && z >= 0) hsum += 2.f * rho;
  }
  if constexpr (DX == 0 && DY == 0) {   // d = (1, 0, 0): the partner term is in this thread
#pragma unroll
    for (int z = 0; z < TZ; ++z) acc[z] += r[z + 1] - r[z];
    return;
  } else {
#pragma unroll
    for (int z = ZLO; z < TZ; ++z) R[fidx(b.lx, b.ly, z)] = r[z + 1];
    float rho;
    if constexpr (DY != 0) {   // the row y = -1 (DY > 0) or y = TY (DY < 0) of m - d: one term per thread
      constexpr int yh = DY > 0 ? -1 : TY;
      const int xh = (b.tid & (TX - 1)) - DX, zh = (b.tid / TX) - DZ;
      R[fidx(xh, yh, zh)] = pair_term<false, INTERIOR, DZ, DY, DX>(
          b, F, F[fidx(xh, yh, zh)], F[fidx(xh + DX, yh + DY, zh + DZ)], xh, yh, zh, pr, w, rho);
    }
    if constexpr (DX != 0) {   // the column x = -1 (DX > 0) or x = TX (DX < 0): 64 terms, first wavefront
      constexpr int xh = DX > 0 ? -1 : TX;
      if (b.tid < TY * TZ) {
        const int yh = (b.tid % TY) - DY, zh = (b.tid / TY) - DZ;
        R[fidx(xh, yh, zh)] = pair_term<false, INTERIOR, DZ, DY, DX>(
            b, F, F[fidx(xh, yh, zh)], F[fidx(xh + DX, yh + DY, zh + DZ)], xh, yh, zh, pr, w, rho);
      }
    }
    __syncthreads();
#pragma unroll
    for (int z = 0; z < TZ; ++z) acc[z] += R[fidx(b.lx, b.ly, z)] - R[fidx(b.lx - DX, b.ly - DY, z - DZ)];
  }
  // Materialise the sums here: otherwise the compiler sinks every direction's
  // adds into the guarded store at the end and keeps all loaded terms live.
#pragma unroll
  for (int z = 0; z < TZ; ++z) asm volatile("" : "+v"(acc[z]));
  if (VALUE) asm volatile("" : "+v"(hsum));
}

}  // namespace

template <bool VALUE, bool INTERIOR>
__device__ __forceinline__ void qggmrf_block(const float* __restrict__ f, float* __restrict__ grad,
                                             double* __restrict__ value, const BlockCtx& b, const PriorArgs& pr,
                                             float scale, float* F, float* R0, float* R1, double* red) {
  const size_t plane = size_t(b.n) * b.n;
  for (int i = b.tid; i < FZ * FP; i += NT) {
    const int bx = i % FX - 1, by = (i / FX) % FY - 1, bz = i / FP - 1;
    float v = 0.f;
    if (INTERIOR || b.inside(bx, by, bz)) v = f[size_t(b.z0 + bz) * plane + size_t(b.y0 + by) * b.n + (b.x0 + bx)];
    F[i] = v;
  }
  __syncthreads();
  float fc[FZ];
#pragma unroll
  for (int k = 0; k < FZ; ++k) fc[k] = F[fidx(b.lx, b.ly, k - 1)];
  float acc[TZ];
#pragma unroll
  for (int z = 0; z < TZ; ++z) acc[z] = 0.f;
  float hsum = 0.f;
  // R buffers alternate between the directions that exchange terms through LDS,
  // so one barrier per direction suffices.
  direction<VALUE, INTERIOR, 1, 0, 0>(b, F, nullptr, fc, acc, hsum, pr);
  direction<VALUE, INTERIOR, 0, 0, 1>(b, F, R0, fc, acc, hsum, pr);
  direction<VALUE, INTERIOR, 0, 1, -1>(b, F, R1, fc, acc, hsum, pr);
  direction<VALUE, INTERIOR, 0, 1, 0>(b, F, R0, fc, acc, hsum, pr);
  direction<VALUE, INTERIOR, 0, 1, 1>(b, F, R1, fc, acc, hsum, pr);
  direction<VALUE, INTERIOR, 1, -1, -1>(b, F, R0, fc, acc, hsum, pr);
  direction<VALUE, INTERIOR, 1, -1, 0>(b, F, R1, fc, acc, hsum, pr);
  direction<VALUE, INTERIOR, 1, -1, 1>(b, F, R0, fc, acc, hsum, pr);
  direction<VALUE, INTERIOR, 1, 0, -1>(b, F, R1, fc, acc, hsum, pr);
  direction<VALUE, INTERIOR, 1, 0, 1>(b, F, R0, fc, acc, hsum, pr);
  direction<VALUE, INTERIOR, 1, 1, -1>(b, F, R1, fc, acc, hsum, pr);
  direction<VALUE, INTERIOR, 1, 1, 0>(b, F, R0, fc, acc, hsum, pr);
  direction<VALUE, INTERIOR, 1, 1, 1>(b, F, R1, fc, acc, hsum, pr);
  const float gscale = scale * 2.f * pr.lambda * b.inv_sigma;
  const int x = b.x0 + b.lx, y = b.y0 + b.ly;
  if (grad && x < b.n && y < b.n) {   // no gradient output: the value alone
#pragma unroll
    for (int z = 0; z < TZ; ++z)
      if (b.z0 + z < b.nz) grad[size_t(b.z0 + z) * plane + size_t(y) * b.n + x] += gscale * acc[z];
  }
  if (VALUE) {
    red[b.tid] = double(hsum);
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
      if (b.tid < w) red[b.tid] += red[b.tid + w];
      __syncthreads();
    }
    if (b.tid == 0) atomicAdd(value, double(pr.lambda) * red[0]);
  }
}

template <bool VALUE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_qggmrf(const float* __restrict__ f, float* __restrict__ grad,
                                               double* __restrict__ value, int nz, int n, PriorArgs pr,
                                               float scale) {
  __shared__ float F[FZ * FP];
  __shared__ float R0[RSZ], R1[RSZ];
  __shared__ double red[VALUE ? NT : 1];
  BlockCtx b;
  b.x0 = blockIdx.x * TX, b.y0 = blockIdx.y * TY, b.z0 = blockIdx.z * TZ;
  b.n = n, b.nz = nz, b.tid = threadIdx.x, b.lx = threadIdx.x % TX, b.ly = threadIdx.x / TX;
  b.inv_sigma = 1.f / pr.sigma;
  // interior block: the block and its halo lie inside the volume
  const bool interior =
      b.x0 >= 1 && b.x0 + TX + 1 <= n && b.y0 >= 1 && b.y0 + TY + 1 <= n && b.z0 >= 1 && b.z0 + TZ + 1 <= nz;
  if (interior) qggmrf_block<VALUE, true>(f, grad, value, b, pr, scale, F, R0, R1, red);
  else qggmrf_block<VALUE, false>(f, grad, value, b, pr, scale, F, R0, R1, red);
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

// <g, x' - x> with x' = y - g/L (clamped at 0 when nonneg); non-finite flag.
// With cand, x' is also stored there (the monotone step evaluates it).
__global__ __launch_bounds__(256) void k_mbir_dot(const float* __restrict__ x, const float* __restrict__ y,
                                                  const float* __restrict__ g, size_t count, float inv_L,
                                                  int nonneg, double* state, float* __restrict__ cand) {
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
    if (cand) cand[i] = xn;
  }
  if (nf) bad = 1;
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&state[kStDot], red[0]);
    if (bad) state[kStNonfinite] = 1.0;
  }
}

// Restart test and momentum: t <- 1 if <g, x'-x> > 0 (when restart is on);
// with monotone, the candidate x' is rejected (x kept, t <- 1, no momentum)
// when its objective exceeds that of x (the first step, with no objective
// recorded yet, is accepted); t' = (1 + sqrt(1 + 4t^2))/2, beta = (t - 1)/t'.
__global__ void k_mbir_finalize(double* state, int restart, int monotone) {
  double t = state[kStT];
  if (restart && state[kStDot] > 0.0) {
    t = 1.0;
    state[kStRestarts] += 1.0;
  }
  double accept = 1.0;
  if (monotone) {
    const double phi = state[kStPhiData] + state[kStPhiPrior];
    if (state[kStPhiKnown] != 0.0 && !(phi <= state[kStPhiX])) {
      accept = 0.0;
      t = 1.0;
      state[kStRejects] += 1.0;
    } else {
      state[kStPhiX] = phi;
      state[kStPhiKnown] = 1.0;
    }
  }
  const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
  state[kStBeta] = accept != 0.0 ? (t - 1.0) / tn : 0.0;
  state[kStT] = tn;
  state[kStAccepted] = accept;
}

// x' = y - g/L; y <- x' + beta (x' - x); x_prev <- x; x <- x'
__global__ __launch_bounds__(256) void k_mbir_update(float* __restrict__ x, float* __restrict__ x_prev,
                                                     float* __restrict__ y, const float* __restrict__ g,
                                                     size_t count, float inv_L, int nonneg,
                                                     const double* __restrict__ state) {
  const float beta = float(state[kStBeta]);
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256) {
    float xn = y[i] - inv_L * g[i];
    if (nonneg) xn = fmaxf(xn, 0.f);
    const float xo = x[i];
    y[i] = xn + beta * (xn - xo);
    x_prev[i] = xo;
    x[i] = xn;
  }
}

// Monotone update, the candidate x' held in x_prev: accepted, x <- x',
// x_prev <- x, y <- x' + beta (x' - x); rejected, x stays and y = x_prev = x.
__global__ __launch_bounds__(256) void k_mbir_update_mono(float* __restrict__ x, float* __restrict__ x_prev,
                                                          float* __restrict__ y, size_t count,
                                                          const double* __restrict__ state) {
  const float beta = float(state[kStBeta]);
  const bool accept = state[kStAccepted] != 0.0;
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256) {
    const float xo = x[i], xn = x_prev[i];
    if (accept) {
      y[i] = xn + beta * (xn - xo);
      x[i] = xn;
    } else {
      y[i] = xo;
    }
    x_prev[i] = xo;
  }
}

// ---------------------------------------------------------------------------
// power iteration for the largest eigenvalue of R^T R
// ---------------------------------------------------------------------------

// uniform in [-1, 1) from a counter-based generator: splitmix64 of
// (seed, index), the published finaliser of Steele, Lea and Flood (2014)
__device__ __forceinline__ float uniform_pm1(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return float(int64_t(z >> 40) - (int64_t(1) << 23)) * (1.0f / float(1 << 23));
}

__global__ __launch_bounds__(256) void k_fill_random(float* __restrict__ v, size_t count, uint64_t seed,
                                                     uint64_t first) {
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256)
    v[i] = uniform_pm1(seed, first + i);
}

__global__ __launch_bounds__(256) void k_fill_value(float* __restrict__ v, size_t count, float value) {
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256) v[i] = value;
}

// *out += scale * sum v^2 (float64)
__global__ __launch_bounds__(256) void k_sum_squares(const float* __restrict__ v, size_t count, double* out,
                                                     double scale) {
  __shared__ double red[256];
  double acc = 0.0;
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256)
    acc += double(v[i]) * double(v[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, scale * red[0]);
}

// v = w / sqrt(*ss) (a zero norm leaves v = 0)
__global__ __launch_bounds__(256) void k_scale_inv_norm(float* __restrict__ v, const float* __restrict__ w,
                                                        size_t count, const double* __restrict__ ss) {
  const double n2 = *ss;
  const float inv = n2 > 0.0 ? float(1.0 / sqrt(n2)) : 0.f;
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256)
    v[i] = w[i] * inv;
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
  const size_t blocks = std::min<size_t>(2048, std::max<size_t>(1, (count + 255) / 256));
  hipLaunchKernelGGL(k_residual, dim3(unsigned(blocks)), dim3(256), 0, st, s, b, count);
  return hipGetLastError();
}

hipError_t launch_residual_norm(float* s, const float* b, size_t count, double* value, hipStream_t st) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, value, 0.0);
  hipLaunchKernelGGL(k_residual_norm, dim3(2048), dim3(256), 0, st, s, b, count, value);
  return hipGetLastError();
}

hipError_t launch_mbir_update(float* x, float* x_prev, float* y, const float* g, size_t count, float inv_L,
                              int nonneg, int restart, double* state, hipStream_t st) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, state + kStDot, 0.0);
  hipLaunchKernelGGL(k_mbir_dot, dim3(2048), dim3(256), 0, st, x, y, g, count, inv_L, nonneg, state,
                     static_cast<float*>(nullptr));
  hipLaunchKernelGGL(k_mbir_finalize, dim3(1), dim3(1), 0, st, state, restart, 0);
  hipLaunchKernelGGL(k_mbir_update, dim3(4096), dim3(256), 0, st, x, x_prev, y, g, count, inv_L, nonneg, state);
  return hipGetLastError();
}

hipError_t launch_mbir_candidate(const float* x, float* x_prev, const float* y, const float* g, size_t count,
                                 float inv_L, int nonneg, double* state, hipStream_t st) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, state + kStDot, 0.0);
  hipLaunchKernelGGL(k_mbir_dot, dim3(2048), dim3(256), 0, st, x, y, g, count, inv_L, nonneg, state, x_prev);
  return hipGetLastError();
}

hipError_t launch_mbir_finish_monotone(float* x, float* x_prev, float* y, size_t count, int restart, double* state,
                                       hipStream_t st) {
  hipLaunchKernelGGL(k_mbir_finalize, dim3(1), dim3(1), 0, st, state, restart, 1);
  hipLaunchKernelGGL(k_mbir_update_mono, dim3(4096), dim3(256), 0, st, x, x_prev, y, count,
                     static_cast<const double*>(state));
  return hipGetLastError();
}

__global__ void k_mbir_state_init(double* state) {
  if (threadIdx.x < kStCount) state[threadIdx.x] = threadIdx.x == kStT ? 1.0 : 0.0;
}

hipError_t launch_mbir_state_init(double* state, hipStream_t st) {
  hipLaunchKernelGGL(k_mbir_state_init, dim3(1), dim3(64), 0, st, state);
  return hipGetLastError();
}

hipError_t launch_fill_random(float* v, size_t count, uint64_t seed, uint64_t first, hipStream_t st) {
  const size_t blocks = std::min<size_t>(4096, std::max<size_t>(1, (count + 255) / 256));
  hipLaunchKernelGGL(k_fill_random, dim3(unsigned(blocks)), dim3(256), 0, st, v, count, seed, first);
  return hipGetLastError();
}

hipError_t launch_fill_value(float* v, size_t count, float value, hipStream_t st) {
  const size_t blocks = std::min<size_t>(4096, std::max<size_t>(1, (count + 255) / 256));
  hipLaunchKernelGGL(k_fill_value, dim3(unsigned(blocks)), dim3(256), 0, st, v, count, value);
  return hipGetLastError();
}

hipError_t launch_half_sum_squares(const float* v, size_t count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, out, 0.0);
  hipLaunchKernelGGL(k_sum_squares, dim3(2048), dim3(256), 0, st, v, count, out, 0.5);
  return hipGetLastError();
}

hipError_t launch_set_double(double* p, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
}

hipError_t launch_normalize(float* v, const float* w, size_t count, double* ss, hipStream_t st) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, ss, 0.0);
  hipLaunchKernelGGL(k_sum_squares, dim3(2048), dim3(256), 0, st, w, count, ss, 1.0);
  hipLaunchKernelGGL(k_scale_inv_norm, dim3(4096), dim3(256), 0, st, v, w, count, static_cast<const double*>(ss));
  return hipGetLastError();
}

}  // namespace nrk
