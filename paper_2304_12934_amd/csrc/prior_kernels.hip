// qGGMRF prior gradient and the accelerated-gradient update for gfx950.
//
// Prior (Sec. 3, eqs. "reg2" and "reg3"): for voxel m and each of its 26
// neighbours n (voxels outside the volume dropped),
//   rho(u)  = u^2 / (c + |u|^(2-p)),           u = (f_m - f_n)/sigma
//   rho'(u) = u (2c + p|u|^(2-p)) / (c + |u|^(2-p))^2
//   dH/df_m = (2 lambda/sigma) sum_n w_mn rho'((f_m - f_n)/sigma)
// (H sums rho over ordered pairs; each unordered pair appears twice.)
//
// The stencil kernel gives each wavefront a strip of the volume, 64 columns
// wide (62 owned, one halo column on each side) and TY rows high, and marches
// it along z: a lane holds its column of the strip for two consecutive planes
// in registers, exchanges x-neighbours with its adjacent lanes by DPP wave
// shifts, evaluates every unordered neighbour pair once and accumulates into
// the gradient in place (Sec. 4, gradients updated in place).  Nothing is
// staged in LDS and no barrier is taken: the neighbourhood caching of the
// paper's Sec. 4.1 lives in registers here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "prior_kernels.hpp"

namespace nrk {

namespace {

// Wavefront tiling: lane l covers column x0 - 1 + l; lanes 1..OWN own their
// column, lanes 0 and 63 only supply the neighbours of the owned ones.  Rows
// are held as index i = 0..TY+1 for y = y0 - 1 + i; rows 1..TY are owned.
constexpr int OWN = 62;
constexpr int TY = 8;
constexpr int QG_WAVES = 4;     // wavefronts per workgroup (independent strips)

// lane l receives lane l - 1 (lane 0 receives 0) / lane l + 1 (lane 63 receives 0)
__device__ __forceinline__ float from_left(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ int from_left_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int from_right_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false); }

// Per neighbour class (face, edge, corner) the gradient term of a pair with
// difference d = f_m - f_n is
//   scale (2 lambda / sigma) w rho'(d / sigma) = d (Ap s + A2c) / (c + s)^2,
//   s = |d / sigma|^(2-p) = 2^((2-p) log2|d| + (2-p) log2(1/sigma)),
// with A = scale 2 lambda w / sigma^2, Ap = A p, A2c = A 2c; and the value
// term w rho(d / sigma) = w d^2 / (sigma^2 (c + s)).  At d = 0, log2 gives
// -inf and s = 0 (p < 2); with p = 2, s = 1.
struct QgConst {
  float e, elog, c;       // 2 - p, (2 - p) log2(1/sigma), c
  float ap[3], a2c[3];    // face, edge, corner
  float w[3];
};

template <bool P2>
__device__ __forceinline__ float qg_s(float d, const QgConst& k) {
  if (P2) return 1.f;
  return __builtin_amdgcn_exp2f(fmaf(k.e, __builtin_amdgcn_logf(fabsf(d)), k.elog));
}

// gradient term of one pair; with VALUE, h += w d^2/(c + s) (the value term
// up to the factor 1/sigma^2 applied once at the end)
template <bool VALUE, bool P2, int CLS>
__device__ __forceinline__ float qg_term(float d, const QgConst& k, float& h) {
  const float s = qg_s<P2>(d, k);
  const float inv = __builtin_amdgcn_rcpf(k.c + s);
  if (VALUE) h = fmaf(k.w[CLS] * d * d, inv, h);
  return d * fmaf(k.ap[CLS], s, k.a2c[CLS]) * inv * inv;
}

// One wavefront's strip: columns x0-1 .. x0+62, rows y0-1 .. y0+TY, owned
// planes [z0, z1).  EDGE: some column or row of the strip lies outside the
// volume (pairs with a partner outside are dropped).
template <bool VALUE, bool P2, bool EDGE, bool ACC>
__device__ __forceinline__ void qg_strip(const float* __restrict__ f, float* __restrict__ grad, int n, int nz,
                                         int x0, int y0, int z0, int z1, const QgConst& k, int lane,
                                         double& hsum) {
  const size_t plane = size_t(n) * n;
  const int x = x0 - 1 + lane;
  const bool lv = !EDGE || (x >= 0 && x < n);
  // pairs with the right (x + 1) / left (x - 1) neighbour lie inside the volume
  const bool okR = !EDGE || (lv && from_right_i(int(lv)) != 0);
  const bool okL = !EDGE || (lv && from_left_i(int(lv)) != 0);
  const bool own = lane >= 1 && lane <= OWN && x < n;
  const int xc = EDGE ? min(max(x, 0), n - 1) : x;
  // rows inside the volume (wave-uniform)
  bool rv[TY + 2];
#pragma unroll
  for (int i = 0; i < TY + 2; ++i) rv[i] = !EDGE || (y0 - 1 + i >= 0 && y0 - 1 + i < n);
  int roff[TY + 2];
#pragma unroll
  for (int i = 0; i < TY + 2; ++i) {
    const int y = EDGE ? min(max(y0 - 1 + i, 0), n - 1) : y0 - 1 + i;
    roff[i] = y * n + xc;
  }

  float p[TY + 2], q[TY + 2];
  float accP[TY + 2], accQ[TY + 2], toR[TY + 2], toL[TY + 2];
  float hP = 0.f, hQ = 0.f;   // value terms whose + side is in plane P / Q

  const int zs = z0 > 0 ? z0 - 1 : 0;
  const int zl = min(z1, nz - 1);

  auto load_plane = [&](int z, float (&v)[TY + 2]) {
    const float* fp = f + size_t(z) * plane;
#pragma unroll
    for (int i = 0; i < TY + 2; ++i) v[i] = fp[roff[i]];
  };
  // Materialise the accumulators between groups of pairs: otherwise the
  // scheduler interleaves the transcendental chains of every pair of the
  // z-step and runs out of registers.
  auto fence = [&]() {
#pragma unroll
    for (int i = 1; i <= TY; ++i) asm volatile("" : "+v"(accQ[i]), "+v"(accP[i]), "+v"(toR[i]), "+v"(toL[i]));
  };
  // a pair with a partner outside the volume contributes nothing
  auto mask = [&](bool ok, float& r, float& h) {
    if (EDGE) {
      r = ok ? r : 0.f;
      h = ok ? h : 0.f;
    }
  };
  // in-plane pairs of Q: (0,0,1), (0,1,0), (0,1,1), (0,1,-1)
  auto in_plane = [&]() {
#pragma unroll
    for (int i = 1; i <= TY; ++i) {
      if (!rv[i]) continue;
      float h = 0.f;
      float r = qg_term<VALUE, P2, 0>(q[i] - from_right(q[i]), k, h);
      mask(okR, r, h);
      accQ[i] += r;
      if (VALUE) hQ += h;
      toR[i] -= r;
    }
    fence();
#pragma unroll
    for (int i = 0; i <= TY; ++i) {
      if (!(rv[i] && rv[i + 1])) continue;
      float h = 0.f;
      const float r = qg_term<VALUE, P2, 0>(q[i] - q[i + 1], k, h);
      if (i >= 1) {
        accQ[i] += r;
        if (VALUE) hQ += h;
      }
      if (i + 1 <= TY) accQ[i + 1] -= r;
    }
    fence();
#pragma unroll
    for (int i = 0; i <= TY; ++i) {
      if (!(rv[i] && rv[i + 1])) continue;
      float h = 0.f;
      float r = qg_term<VALUE, P2, 1>(q[i] - from_right(q[i + 1]), k, h);
      mask(okR, r, h);
      if (i >= 1) {
        accQ[i] += r;
        if (VALUE) hQ += h;
      }
      if (i + 1 <= TY) toR[i + 1] -= r;
    }
    fence();
#pragma unroll
    for (int i = 0; i <= TY; ++i) {
      if (!(rv[i] && rv[i + 1])) continue;
      float h = 0.f;
      float r = qg_term<VALUE, P2, 1>(q[i] - from_left(q[i + 1]), k, h);
      mask(okL, r, h);
      if (i >= 1) {
        accQ[i] += r;
        if (VALUE) hQ += h;
      }
      if (i + 1 <= TY) toL[i + 1] -= r;
    }
  };
  // pairs between P (plane z-1) and Q (plane z): d = (1, dy, dx)
  auto cross = [&]() {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
      for (int i = 0; i <= TY + 1; ++i) {
        const int j = i + dy;                            // row of the partner in Q
        if (j < 0 || j > TY + 1) continue;
        if ((i < 1 || i > TY) && (j < 1 || j > TY)) continue;   // neither side owned
        if (!(rv[i] && rv[j])) continue;
        // dx = 0
        {
          float h = 0.f;
          const float r = dy == 0 ? qg_term<VALUE, P2, 0>(p[i] - q[j], k, h) : qg_term<VALUE, P2, 1>(p[i] - q[j], k, h);
          if (i >= 1 && i <= TY) {
            accP[i] += r;
            if (VALUE) hP += h;
          }
          if (j >= 1 && j <= TY) accQ[j] -= r;
        }
        // dx = +1
        {
          float h = 0.f;
          float r = dy == 0 ? qg_term<VALUE, P2, 1>(p[i] - from_right(q[j]), k, h) : qg_term<VALUE, P2, 2>(p[i] - from_right(q[j]), k, h);
          mask(okR, r, h);
          if (i >= 1 && i <= TY) {
            accP[i] += r;
            if (VALUE) hP += h;
          }
          if (j >= 1 && j <= TY) toR[j] -= r;
        }
        // dx = -1
        {
          float h = 0.f;
          float r = dy == 0 ? qg_term<VALUE, P2, 1>(p[i] - from_left(q[j]), k, h) : qg_term<VALUE, P2, 2>(p[i] - from_left(q[j]), k, h);
          mask(okL, r, h);
          if (i >= 1 && i <= TY) {
            accP[i] += r;
            if (VALUE) hP += h;
          }
          if (j >= 1 && j <= TY) toL[j] -= r;
        }
        fence();
      }
    }
  };
  auto clear_q = [&]() {
#pragma unroll
    for (int i = 0; i < TY + 2; ++i) accQ[i] = 0.f, toR[i] = 0.f, toL[i] = 0.f;
    hQ = 0.f;
  };
  // the terms this lane computed for its neighbours' columns
  auto receive = [&]() {
#pragma unroll
    for (int i = 1; i <= TY; ++i) accQ[i] += from_left(toR[i]) + from_right(toL[i]);
  };
  auto write = [&](int z, const float (&acc)[TY + 2], float h) {
    if (grad && own) {
      float* gp = grad + size_t(z) * plane;
#pragma unroll
      for (int i = 1; i <= TY; ++i)
        if (!EDGE || y0 - 1 + i < n) gp[roff[i]] = ACC ? gp[roff[i]] + acc[i] : acc[i];
    }
    if (VALUE && own) hsum += double(h);
  };

  // first plane: the owned plane z0 = 0, or the halo plane z0 - 1
  load_plane(zs, q);
  clear_q();
  if (zs == z0) in_plane();
  receive();
  float qn[TY + 2];
  for (int z = zs + 1; z <= zl; ++z) {
#pragma unroll
    for (int i = 0; i < TY + 2; ++i) p[i] = q[i], accP[i] = accQ[i];
    hP = hQ;
    load_plane(z, qn);
#pragma unroll
    for (int i = 0; i < TY + 2; ++i) q[i] = qn[i];
      clear_q();
    cross();
    if (z < z1) in_plane();
    receive();
    if (z - 1 >= z0) write(z - 1, accP, hP);
  }
  if (zl < z1) write(zl, accQ, hQ);   // the volume's last plane is owned
}

}  // namespace

// One workgroup = QG_WAVES independent wavefronts; wavefront g covers x-tile
// g % xt, row strip (g / xt) % yt, z-chunk g / (xt yt).
template <bool VALUE, bool P2, bool ACC>
__device__ __forceinline__ void qggmrf_body(const float* __restrict__ f, float* __restrict__ grad,
                                            double* __restrict__ value, int nz, int n, const QgConst& k, int xt,
                                            int yt, int zchunk, int nwaves, double value_scale) {
  __shared__ double red[QG_WAVES];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // wave-uniform: keeps the strip's geometry and row tests in scalar registers
  const int g = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * QG_WAVES + wv);
  double hsum = 0.0;
  if (g < nwaves) {
    const int tx = g % xt, ty = (g / xt) % yt, tz = g / (xt * yt);
    const int x0 = tx * OWN, y0 = ty * TY, z0 = tz * zchunk, z1 = min(nz, z0 + zchunk);
    const bool interior = x0 >= 1 && x0 + OWN <= n - 1 && y0 >= 1 && y0 + TY <= n - 1;
    if (interior) qg_strip<VALUE, P2, false, ACC>(f, grad, n, nz, x0, y0, z0, z1, k, lane, hsum);
    else qg_strip<VALUE, P2, true, ACC>(f, grad, n, nz, x0, y0, z0, z1, k, lane, hsum);
  }
  if (VALUE) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) hsum += __shfl_xor(hsum, off);
    if (lane == 0) red[wv] = hsum;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < QG_WAVES; ++w) t += red[w];
      atomicAdd(value, value_scale * t);
    }
  }
}

// gradient only (ACC: added into grad, else stored): 4 wavefronts per SIMD
// (the strip's registers fit in 128)
template <bool P2, bool ACC>
__global__ __launch_bounds__(64 * QG_WAVES) __attribute__((amdgpu_waves_per_eu(4))) void k_qggmrf(
    const float* __restrict__ f, float* __restrict__ grad, int nz, int n, QgConst k, int xt, int yt, int zchunk,
    int nwaves) {
  qggmrf_body<false, P2, ACC>(f, grad, nullptr, nz, n, k, xt, yt, zchunk, nwaves, 0.0);
}

// with the value: the extra accumulations need more registers
template <bool P2>
__global__ __launch_bounds__(64 * QG_WAVES) __attribute__((amdgpu_waves_per_eu(2))) void k_qggmrf_value(
    const float* __restrict__ f, float* __restrict__ grad, double* __restrict__ value, int nz, int n, QgConst k,
    int xt, int yt, int zchunk, int nwaves, double value_scale) {
  qggmrf_body<true, P2, true>(f, grad, value, nz, n, k, xt, yt, zchunk, nwaves, value_scale);
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
// With cand, x' is also stored there (the monotone step evaluates it).  With
// gp, the gradient is g + gp (a second part computed elsewhere), stored back
// into g.
__global__ __launch_bounds__(256) void k_mbir_dot(const float* __restrict__ x, const float* __restrict__ y,
                                                  float* __restrict__ g, size_t count, float inv_L,
                                                  int nonneg, double* state, float* __restrict__ cand,
                                                  const float* __restrict__ gp) {
  __shared__ double red[256];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double acc = 0.0;
  int nf = 0;
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256) {
    float gi = g[i];
    if (gp) {
      gi += gp[i];
      g[i] = gi;
    }
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
                         float scale, hipStream_t st, bool accumulate) {
  if (value) hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, value, 0.0);
  QgConst k;
  const double inv_sigma = 1.0 / double(pr.sigma);
  k.e = 2.f - pr.p;
  k.elog = float(double(k.e) * std::log2(inv_sigma));
  k.c = pr.c;
  const float w[3] = {pr.w_face, pr.w_edge, pr.w_corner};
  for (int c = 0; c < 3; ++c) {
    const double a = double(scale) * 2.0 * double(pr.lambda) * inv_sigma * inv_sigma * double(w[c]);
    k.ap[c] = float(a * double(pr.p));
    k.a2c[c] = float(a * 2.0 * double(pr.c));
    k.w[c] = w[c];
  }
  // H = lambda sum over ordered pairs = 2 lambda sum over unordered pairs
  const double value_scale = 2.0 * double(pr.lambda) * inv_sigma * inv_sigma;
  const int xt = (n + OWN - 1) / OWN, yt = (n + TY - 1) / TY;
  // enough z-chunks for about eight wavefronts per SIMD
  const long strips = long(xt) * yt;
  const int chunks = int(std::max<long>(1, std::min<long>(nz, (8192 + strips - 1) / strips)));
  const int zchunk = (nz + chunks - 1) / chunks;
  const int nzc = (nz + zchunk - 1) / zchunk;
  const long nwaves = strips * nzc;
  const dim3 grid(unsigned((nwaves + QG_WAVES - 1) / QG_WAVES));
  const bool p2 = pr.p == 2.f;
  const int nw = int(nwaves);
  const dim3 block(64 * QG_WAVES);
  if (value) {
    if (p2) hipLaunchKernelGGL(k_qggmrf_value<true>, grid, block, 0, st, f, grad, value, nz, n, k, xt, yt, zchunk, nw, value_scale);
    else hipLaunchKernelGGL(k_qggmrf_value<false>, grid, block, 0, st, f, grad, value, nz, n, k, xt, yt, zchunk, nw, value_scale);
  } else {
    if (accumulate) {
      if (p2) hipLaunchKernelGGL((k_qggmrf<true, true>), grid, block, 0, st, f, grad, nz, n, k, xt, yt, zchunk, nw);
      else hipLaunchKernelGGL((k_qggmrf<false, true>), grid, block, 0, st, f, grad, nz, n, k, xt, yt, zchunk, nw);
    } else {
      if (p2) hipLaunchKernelGGL((k_qggmrf<true, false>), grid, block, 0, st, f, grad, nz, n, k, xt, yt, zchunk, nw);
      else hipLaunchKernelGGL((k_qggmrf<false, false>), grid, block, 0, st, f, grad, nz, n, k, xt, yt, zchunk, nw);
    }
  }
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

hipError_t launch_mbir_update(float* x, float* x_prev, float* y, float* g, size_t count, float inv_L,
                              int nonneg, int restart, double* state, hipStream_t st, bool add_x_prev) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, state + kStDot, 0.0);
  hipLaunchKernelGGL(k_mbir_dot, dim3(2048), dim3(256), 0, st, x, y, g, count, inv_L, nonneg, state,
                     static_cast<float*>(nullptr), add_x_prev ? static_cast<const float*>(x_prev) : nullptr);
  hipLaunchKernelGGL(k_mbir_finalize, dim3(1), dim3(1), 0, st, state, restart, 0);
  hipLaunchKernelGGL(k_mbir_update, dim3(4096), dim3(256), 0, st, x, x_prev, y, g, count, inv_L, nonneg, state);
  return hipGetLastError();
}

hipError_t launch_mbir_candidate(const float* x, float* x_prev, const float* y, const float* g, size_t count,
                                 float inv_L, int nonneg, double* state, hipStream_t st) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(1), 0, st, state + kStDot, 0.0);
  hipLaunchKernelGGL(k_mbir_dot, dim3(2048), dim3(256), 0, st, x, y, const_cast<float*>(g), count, inv_L, nonneg,
                     state, x_prev, static_cast<const float*>(nullptr));
  return hipGetLastError();
}

hipError_t launch_mbir_finish_monotone(float* x, float* x_prev, float* y, size_t count, int restart, double* state,
                                       hipStream_t st) {
  hipLaunchKernelGGL(k_mbir_finalize, dim3(1), dim3(1), 0, st, state, restart, 1);
  hipLaunchKernelGGL(k_mbir_update_mono, dim3(4096), dim3(256), 0, st, x, x_prev, y, count,
                     static_cast<const double*>(state));
  return hipGetLastError();
}

// y = x + beta (x - x_prev) with the beta of the last finalised step: the
// extrapolated point of the accelerated-gradient iteration, formed when the
// iterates live elsewhere (host memory) and only x and x_prev are kept
__global__ __launch_bounds__(256) void k_mbir_extrapolate(float* __restrict__ y, const float* __restrict__ x,
                                                          const float* __restrict__ x_prev, size_t count,
                                                          const double* __restrict__ state) {
  const float beta = float(state[kStBeta]);
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256) {
    const float xn = x[i];
    y[i] = xn + beta * (xn - x_prev[i]);
  }
}

hipError_t launch_mbir_extrapolate(float* y, const float* x, const float* x_prev, size_t count, const double* state,
                                   hipStream_t st) {
  const size_t blocks = std::min<size_t>(4096, std::max<size_t>(1, (count + 255) / 256));
  hipLaunchKernelGGL(k_mbir_extrapolate, dim3(unsigned(blocks)), dim3(256), 0, st, y, x, x_prev, count, state);
  return hipGetLastError();
}

hipError_t launch_mbir_dot_accumulate(const float* x, const float* y, float* g, const float* gp, size_t count,
                                      float inv_L, int nonneg, double* state, float* cand, hipStream_t st) {
  hipLaunchKernelGGL(k_mbir_dot, dim3(2048), dim3(256), 0, st, x, y, g, count, inv_L, nonneg, state, cand, gp);
  return hipGetLastError();
}

hipError_t launch_mbir_finalize(double* state, int restart, hipStream_t st) {
  hipLaunchKernelGGL(k_mbir_finalize, dim3(1), dim3(1), 0, st, state, restart, 0);
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
