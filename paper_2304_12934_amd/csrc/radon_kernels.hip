// HIP kernels of the NUFFT Radon projector (forward chain F1-F4) and its
// exact transpose (adjoint chain A1-A4) for gfx950.
//
// Data layout of one slice in its workspace slot (complex = float2):
//   T    [G/2+1][N]            row transform of the slice, stored transposed
//                              in tiles of 4 kept frequencies x 2 rows
//   ext  [rows][cols]          oversampled half-plane spectrum qx in [0, G/2]
//                              plus `halo` rows on each side and `colpad`
//                              columns on each side, so that every WxW
//                              kernel footprint is a plain rectangle:
//                                row r  <-> qx = r - halo
//                                col p  <-> qy = p - colpad - G/2
//                              Halo cells hold copies (periodic qy) and
//                              conjugate mirrors (qx < 0 and qx > G/2, by
//                              Hermitian symmetry of a real slice).
//   yh   [n_angles][N_t/2+1]   half-line spectra (interpolated values in the
//                              forward chain, the adjoint input's in the adjoint)
//
// Forward (Sec. 2.2, eqs. "nufft"-"nufft3" in reverse order):
//   F1 k_fwd_rows   divide by phihat(x/G) phihat(y/G), zero-pad to G,
//                   R2C along x for two rows at once, write T transposed
//   F2 k_fwd_cols   C2C along y per kept qx, write ext (with halo cells)
//   F3 k_interp_tiles  WxW Kaiser-Bessel interpolation onto the half-lines
//                   k_j = j/N_t from LDS-staged grid tiles, into yh
//   F4 k_fwd_radial  the 1D inverse DFT along each line (Hermitian, two
//                   angles packed in one complex transform), real sinogram rows
//   (F3+F4 k_fwd_interp does both per angle pair, gathering from the grid)
// Adjoint (Sec. 3, eq. "transpose"): the transpose of every step in reverse:
//   A1 k_adj_radial  R2C of two sinogram rows, weights c_j/N_t
//   A2 k_spread_*    WxW spreading onto ext (LDS tiles, or plain atomics)
//   A3 k_adj_cols    fold halo cells back, inverse C2C along y, keep N rows
//   A4 k_adj_rows    inverse half-spectrum transform along x for two rows,
//                    deapodise, real output
//
// Every kernel takes its unit from a work list of (slice, unit) items built
// by the plan, so one launch covers a batch of slices of mixed sizes (one
// launch per FFT length); per-slice parameters come from a device-resident
// SliceDesc.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "fft.hpp"
#include "radon_kernels.hpp"

namespace nrk {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Coordinates of a polar point j on angle table entry (gx, gy): u = j*(gx, gy)
// in grid cells, first tap g0 = ceil(u - W/2) and the W weights
// phi(u - g0 - i) from the piecewise polynomial in z = u - g0 - (W-1)/2.
// The multiply and subtract are rounded separately so the host's spreading
// bins see the same g0.
template <int W, class KB>
__device__ __forceinline__ void point_taps(double gx, double gy, int j, const KB& kb, int& g0x,
                                           int& g0y, float* wx, float* wy) {
  constexpr int D = W + 2;
  const double ux = __dmul_rn(double(j), gx);
  const double uy = __dmul_rn(double(j), gy);
  const double fx = ceil(__dsub_rn(ux, 0.5 * W));
  const double fy = ceil(__dsub_rn(uy, 0.5 * W));
  g0x = int(fx);
  g0y = int(fy);
  const float zx = float(ux - fx - 0.5 * (W - 1));
  const float zy = float(uy - fy - 0.5 * (W - 1));
  // phi is even, so tap W-1-i at z is tap i at -z: with p_i = E_i + O_i split
  // into its even and odd powers, taps i and W-1-i are E_i(z) +- O_i(z), each
  // part a Horner sum in z^2 (half the work of two full Horner sums)
  const float tx = zx * zx, ty = zy * zy;
#pragma unroll
  for (int i = 0; i < (W + 1) / 2; ++i) {
    const float* c = kb.c + i * (D + 1);
    constexpr int KE = (D / 2) * 2, KO = ((D - 1) / 2) * 2 + 1;   // highest even and odd powers
    float ex = c[KE], ey = ex, ox = c[KO], oy = ox;
#pragma unroll
    for (int k = KE - 2; k >= 0; k -= 2) {
      ex = fmaf(ex, tx, c[k]);
      ey = fmaf(ey, ty, c[k]);
    }
#pragma unroll
    for (int k = KO - 2; k >= 1; k -= 2) {
      ox = fmaf(ox, tx, c[k]);
      oy = fmaf(oy, ty, c[k]);
    }
    ox *= zx;
    oy *= zy;
    wx[i] = ex + ox;
    wy[i] = ey + oy;
    if (W - 1 - i != i) {
      wx[W - 1 - i] = ex - ox;
      wy[W - 1 - i] = ey - oy;
    }
  }
}

// Pointers read from device memory are generic to the compiler, which then
// emits flat loads (slower to issue, and counted against the LDS wait counter
// too). Every buffer a slice descriptor points to is global memory, so the
// kernels see the descriptor with global-typed pointers.
struct DSlice {
  int N, Nt, na, G, H, rows, cols, tiles_x;
  int64_t vol_off, sino_off;
  const NR_G float* deapod;
  const NR_G float2* tw_G;
  const NR_G float2* tw_Nt;
  const NR_G float2* shift;
  const NR_G double* gxy;
  const NR_G int32_t* flip;
  NR_G float2* T;
  NR_G float2* ext;
  NR_G float2* yh;
  const NR_G int32_t* pts;
  const NR_G SpreadItem* items;
  const NR_G int32_t* zero_tiles;
  const NR_G int32_t* ipts;
  const NR_G SpreadItem* iitems;
  int itiles_x, rdisc, jbits;
};

// The slice descriptor by value (uniform: scalar loads).
__device__ __forceinline__ DSlice load_desc(const SliceDesc* p) {
  const SliceDesc s = *p;
  DSlice d;
  d.N = s.N, d.Nt = s.Nt, d.na = s.na, d.G = s.G, d.H = s.H, d.rows = s.rows, d.cols = s.cols;
  d.tiles_x = s.tiles_x;
  d.vol_off = s.vol_off, d.sino_off = s.sino_off;
  d.deapod = (const NR_G float*)s.deapod;
  d.tw_G = (const NR_G float2*)s.tw_G;
  d.tw_Nt = (const NR_G float2*)s.tw_Nt;
  d.shift = (const NR_G float2*)s.shift;
  d.gxy = (const NR_G double*)s.gxy;
  d.flip = (const NR_G int32_t*)s.flip;
  d.T = (NR_G float2*)s.T;
  d.ext = (NR_G float2*)s.ext;
  d.yh = (NR_G float2*)s.yh;
  d.pts = (const NR_G int32_t*)s.pts;
  d.items = (const NR_G SpreadItem*)s.items;
  d.zero_tiles = (const NR_G int32_t*)s.zero_tiles;
  d.ipts = (const NR_G int32_t*)s.ipts;
  d.iitems = (const NR_G SpreadItem*)s.iitems;
  d.itiles_x = s.itiles_x;
  d.rdisc = s.rdisc;
  d.jbits = s.jbits;
  return d;
}

// round to the nearest integer, halves up: one instruction (v_cvt_rpi_i32_f32
// computes floor(x + 0.5)) where __float2int_rn takes two; the spreading
// rounds each of its ~90 fixed-point contributions per point with it
__device__ __forceinline__ int round_half_up(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// Non-temporal stores, for a stage's large output written in whole
// contiguous rows that the next stage reads once: the forward column
// transform's grid rows and the adjoint spreading's tile rows (each measured
// faster to store and faster for the next stage to read back, when the
// batch's grids exceed the last-level cache; the launch's stream_stores
// says so).  The 16-byte pieces of T, 64 bytes apart, and the half-lines yh,
// which the spreading reads back in scattered order, measured slower with
// them; grids that fit in the last-level cache, slower too.
typedef float nr_v2f __attribute__((ext_vector_type(2)));
typedef float nr_v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_nt(NR_G float2* p, float2 v) {
  __builtin_nontemporal_store(nr_v2f{v.x, v.y}, reinterpret_cast<NR_G nr_v2f*>(p));
}
__device__ __forceinline__ void store_nt(NR_G float4* p, float4 v) {
  __builtin_nontemporal_store(nr_v4f{v.x, v.y, v.z, v.w}, reinterpret_cast<NR_G nr_v4f*>(p));
}
__device__ __forceinline__ void store_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }

template <int L>
__device__ __forceinline__ int wrap_index(int x) {   // x in [-L, 2L) -> [0, L)
  return x < 0 ? x + L : (x >= L ? x - L : x);
}

// Workgroup reductions of one float per thread (T threads, T/64 wavefronts):
// butterfly within each wavefront, then the per-wavefront results through
// `red` (T/64 floats of LDS).  Every thread gets the result; both contain a
// barrier.
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
  return x;
}
template <int T>
__device__ __forceinline__ float block_sum(float x, float* red, int tid) {
  x = wave_sum(x);
  __syncthreads();   // red may still be read from a previous reduction
  if ((tid & 63) == 0) red[tid >> 6] = x;
  __syncthreads();
  float r = 0.f;
#pragma unroll
  for (int w = 0; w < T / 64; ++w) r += red[w];
  return r;
}
template <int T>
__device__ __forceinline__ float block_max(float x, float* red, int tid) {
  x = wave_max(x);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = x;
  __syncthreads();
  float r = 0.f;
#pragma unroll
  for (int w = 0; w < T / 64; ++w) r = fmaxf(r, red[w]);
  return r;
}

// for (int n = tid; n < COUNT; n += T) with a compile-time trip count, so
// that the compiler unrolls it and issues all of its loads before waiting
#define NR_STRIDED(n, COUNT, T)                                                                       \
  _Pragma("unroll") for (int n##_it = 0, n = tid; n##_it < ((COUNT) + (T)-1) / (T); ++n##_it, n += (T)) \
    if ((COUNT) % (T) == 0 || n < (COUNT))

// LDS extents of the tiled interpolation and spreading (shared by their
// kernels and the persistent kernel).
template <int W>
struct InterpLds {
  static constexpr int RW = kInterpTileW + W + 1, RH = kInterpTileH + W + 1;
  // staged from one cell before the region (an even grid column), in pairs
  // of cells: RWP columns, an even count
  static constexpr int RWP = (RW + 2) / 2 * 2;
  static constexpr int RS = RWP | 1;   // odd row stride (in complex cells)
};
template <int W, int TW, int TH>
struct SpreadLds {
  static constexpr int AH = TH + 2 * W, AW = TW + 2 * W;   // tile with its apron
  static constexpr int TS = AW + 1;                         // odd row stride: columns of lanes spread over banks
  // one accumulator array: the real plane, then the imaginary plane; the
  // length rounded up to whole 16-byte groups for the vector clear
  static constexpr int ACC = (2 * AH * TS + 3) / 4 * 4;
};

// The transform kernels run one unit of their work list per workgroup (block
// b takes entry b; the forward columns, the interpolation and the spreading
// take two, see there); padding entries (slice < 0) and blocks past the list
// do nothing.
#define NR_FOR_EACH_UNIT(a, wi)                                                                    \
  if (const WorkItem wi = int(blockIdx.x) < (a).n_work ? (a).work[blockIdx.x] : WorkItem{-1, 0}; \
      wi.slice >= 0)


// T is stored in tiles of 4 kept frequencies x 2 rows: the row transform's
// 16-byte results (two rows at one q) then land 64 contiguous bytes per 4
// threads instead of one 16-byte piece per 20 KB row of T, at the price of
// 16-byte pieces 64 bytes apart in the column transforms (measured: rows
// -8 us, adjoint rows -5, columns +6, adjoint columns +3 per 2560^2 slice).
// Index of the float4 holding rows 2p, 2p+1 at q:
__device__ __forceinline__ size_t t4(int q, int p, int N) {
  return (size_t(q >> 2) * (N / 2) + p) * 4 + (q & 3);
}
// ---------------------------------------------------------------------------
// F1: rows (along x), two at a time, transposed store into T
// ---------------------------------------------------------------------------

template <int L, int T, class LA>
__device__ __forceinline__ void fwd_rows_unit(const LA& a, const WorkItem wi, float2* sbuf, const int tid) {
  const Lds s{sbuf};
  const DSlice d = load_desc(a.descs + wi.slice);
  constexpr int N = L / 2;   // G = 2N
  const int iy0 = 2 * wi.unit;
  const float* __restrict__ f0 = a.vol_in + d.vol_off + size_t(iy0) * N;
  const float d0 = d.deapod[iy0], d1 = d.deapod[iy0 + 1];
  // x = ix - N/2 sits at index x mod L; indices N/2 .. L - N/2 - 1 are the zero padding
  const NR_G float* __restrict__ dp = d.deapod;
  fft_lds_halfzero<L, T, false>(s, d.tw_G, tid, [&](int n) {
    const int ix = n < N / 2 ? n + N / 2 : n - (L - N / 2);
    const float dx = dp[ix];
    return make_float2(dx * d0 * f0[ix], dx * d1 * f0[N + ix]);
  });
  // split the two real transforms: A = (Z_q + conj Z_-q)/2, B = (Z_q - conj Z_-q)/(2i)
  NR_G float4* __restrict__ out = (NR_G float4*)d.T;
  NR_STRIDED(q, L / 2 + 1, T) {
    const float2 z1 = s[q], z2 = s[q == 0 ? 0 : L - q];
    float4 o;
    o.x = 0.5f * (z1.x + z2.x);
    o.y = 0.5f * (z1.y - z2.y);
    o.z = 0.5f * (z1.y + z2.y);
    o.w = 0.5f * (z2.x - z1.x);
    out[t4(q, iy0 >> 1, N)] = o;
  }
  __syncthreads();
}

template <int L>
__global__ __launch_bounds__(fft_threads(L)) void k_fwd_rows(LaunchArgs a) {
  __shared__ float2 sbuf[lds_elems<L>()];
  NR_FOR_EACH_UNIT(a, wi) fwd_rows_unit<L, fft_threads(L)>(a, wi, sbuf, int(threadIdx.x));
}

// ---------------------------------------------------------------------------
// F2: columns (along y) per kept qx, into the extended grid
// ---------------------------------------------------------------------------

// store v at natural frequency index n of a grid row (and its periodic copies)
template <int L>
__device__ __forceinline__ void store_row(NR_G float2* row, int colpad, int n, float2 v) {
  const int p = wrap_index<L>(n + L / 2) + colpad;
  row[p] = v;
  if (p >= L) row[p - L] = v;                            // left pad: qy < -L/2
  if (p < 2 * colpad) row[p + L] = v;                    // right pad: qy >= L/2
}

template <int L, int T, class LA>
__device__ __forceinline__ void fwd_cols_unit(const LA& a, const WorkItem wi, float2* sbuf, const int tid) {
  const Lds s{sbuf};
  const int halo = a.halo, colpad = a.colpad;
  const DSlice d = load_desc(a.descs + wi.slice);
  constexpr int N = L / 2;   // G = 2N
  const int cols = d.cols;
  const int qx = wi.unit;
  // y = iy - N/2 sits at index y mod L; row iy of column qx is half iy & 1
  // of the tile entry t4(qx, iy / 2)
  const NR_G float2* __restrict__ T2 = (const NR_G float2*)d.T;
  fft_first_pass_from<L, T, false, true>(s, tid, [&](int n) {
    const int iy = n < N / 2 ? n + N / 2 : n - (L - N / 2);
    return T2[2 * t4(qx, iy >> 1, N) + (iy & 1)];
  });
  NR_G float2* ext = d.ext;
  NR_G float2* row = ext + size_t(qx + halo) * cols;
  // rows qx = -s (s = 1..halo) hold conj(G[s][-qy]); rows qx = L/2 + s hold conj(G[L/2 - s][-qy])
  NR_G float2* m1 = (qx >= 1 && qx <= halo) ? ext + size_t(halo - qx) * cols : nullptr;
  NR_G float2* m2 = (qx >= L / 2 - halo && qx <= L / 2 - 1) ? ext + size_t(L - qx + halo) * cols : nullptr;
  fft_passes<L, T, false, 1>(s, d.tw_G, tid);
  // only |q| <= rdisc is ever read: the natural indices n in [0, lim] and
  // [L - lim, L) of this row (a cell's periodic copies lie farther out than
  // the cell itself, and mirror rows keep |q_y|).  Stored from LDS by every
  // thread: measured faster than storing from the last pass's registers,
  // which for L = 5120 leaves a fifth of the threads idle.
  const int r2 = d.rdisc * d.rdisc - qx * qx;
  const int lim = r2 <= 0 ? -1 : int(sqrtf(float(r2)));
  const bool full = lim >= L / 2;   // the whole row, q_y = -L/2 included
  const int cnt = full ? L : 2 * lim + 1;
  if (m1 || m2) {   // the few columns next to qx = 0 and G/2 also fill mirror rows
    for (int k = tid; k < cnt; k += T) {
      const int n = (full || k <= lim) ? k : L - cnt + k;
      const float2 v = s[n];
      store_row<L>(row, colpad, n, v);
      const int nm = n == 0 ? 0 : L - n;
      if (m1) store_row<L>(m1, colpad, nm, c_conj(v));
      if (m2) store_row<L>(m2, colpad, nm, c_conj(v));
    }
  } else {
    // the kept natural indices are one contiguous run of row positions
    // m = (n + L/2) mod L: [L/2 - lim, L/2 + lim], or the whole row
    const int m0 = full ? 0 : L / 2 - lim;
    NR_G float2* __restrict__ out = row + colpad + m0;
#pragma unroll 4
    for (int k = tid; k < cnt; k += T) {
      const int m = m0 + k;
      const float2 v = s[m < L / 2 ? m + L / 2 : m - L / 2];
      if (a.stream_stores)
        store_nt(&out[k], v);
      else
        out[k] = v;
    }
    // periodic copies: positions m in [L - colpad, L) also at m - L (left
    // pad), m in [0, colpad) also at m + L (right pad), when stored
    if (tid < 2 * colpad) {
      const int m = tid < colpad ? tid + L - colpad : tid - colpad;
      if (m >= m0 && m < m0 + cnt) row[tid < colpad ? tid : L + tid] = s[m < L / 2 ? m + L / 2 : m - L / 2];
    }
  }
  __syncthreads();
}

template <int L>
__global__ __launch_bounds__(fft_threads(L)) void k_fwd_cols(LaunchArgs a) {
  __shared__ float2 sbuf[lds_elems<L>()];
  // Launches of many columns (a.pair_units) take two per workgroup:
  // positions p and p + 8 of the XCD-interleaved list (both on this
  // workgroup's XCD), as two calls with a barrier between (a loop over the
  // two kept values live across them and doubled the VGPRs).  Measured on
  // 2560^2 slices in launches of 8: 40.0 -> 37.2 us per slice; launches of
  // one 1280^2 or 2048^2 slice (1281 or 2049 columns) ran slower with half
  // as many workgroups, and the same pairing made the row transforms and
  // the adjoint columns slower (21.7 -> 22.3, 24.4 -> 28.6, 34.0 -> 43.4 us).
  if (a.pair_units) {
    const int p0 = 16 * (int(blockIdx.x) >> 3) + (int(blockIdx.x) & 7), p1 = p0 + 8;
    const WorkItem w0 = p0 < a.n_work ? a.work[p0] : WorkItem{-1, 0};
    const WorkItem w1 = p1 < a.n_work ? a.work[p1] : WorkItem{-1, 0};
    if (w0.slice >= 0) fwd_cols_unit<L, fft_threads(L)>(a, w0, sbuf, int(threadIdx.x));
    __syncthreads();
    if (w1.slice >= 0) fwd_cols_unit<L, fft_threads(L)>(a, w1, sbuf, int(threadIdx.x));
  } else {
    NR_FOR_EACH_UNIT(a, wi) fwd_cols_unit<L, fft_threads(L)>(a, wi, sbuf, int(threadIdx.x));
  }
}

// ---------------------------------------------------------------------------
// F3 + F4: interpolation onto two half-lines and the radial inverse DFT
// ---------------------------------------------------------------------------

template <int W, class KB>
__device__ __forceinline__ float2 interp_point(const DSlice& d, int halo, int colpad, const KB& kb,
                                               int ang, int j) {
  int g0x, g0y;
  float wx[W], wy[W];
  point_taps<W>(d.gxy[2 * ang], d.gxy[2 * ang + 1], j, kb, g0x, g0y, wx, wy);
  const NR_G float2* __restrict__ p = d.ext + size_t(g0x + halo) * d.cols + (g0y + d.G / 2 + colpad);
  float2 acc = make_float2(0.f, 0.f);
#pragma unroll
  for (int i = 0; i < W; ++i) {
    float2 r = make_float2(0.f, 0.f);
#pragma unroll
    for (int l = 0; l < W; ++l) {
      const float2 v = p[l];
      r.x = fmaf(wy[l], v.x, r.x);
      r.y = fmaf(wy[l], v.y, r.y);
    }
    acc.x = fmaf(wx[i], r.x, acc.x);
    acc.y = fmaf(wx[i], r.y, acc.y);
    p += d.cols;
  }
  if (d.flip[ang]) acc.y = -acc.y;
  return acc;
}

// The two sinogram rows a0, a0 + 1 (the second when has1) from the packed
// inverse transform in s (real part: row a0, imaginary part: row a0 + 1):
// bin m (t = m - N_t/2) is output index t mod N_t.  With a.sino_sub the
// data b are subtracted as the rows are stored (the residual R f - b of the
// data term, Sec. 3 eq. "objfn"), so no separate pass re-reads them.
template <int L, int T, class LA>
__device__ __forceinline__ void store_sino_rows(const LA& a, const DSlice& d, int a0, bool has1, Lds s,
                                                int tid) {
  const size_t off = d.sino_off + size_t(a0) * L;
  float* __restrict__ o0 = a.sino_out + off;
  if (a.sino_sub) {
    const float* __restrict__ b0 = a.sino_sub + off;
    const float* __restrict__ b1 = has1 ? b0 + L : b0;   // loads stay unconditional
    NR_STRIDED(m, L, T) {
      const float2 z = s[wrap_index<L>(m + L / 2)];
      const float c0 = b0[m], c1 = b1[m];
      o0[m] = z.x - c0;
      if (has1) o0[L + m] = z.y - c1;
    }
  } else {
    NR_STRIDED(m, L, T) {
      const float2 z = s[wrap_index<L>(m + L / 2)];
      o0[m] = z.x;
      if (has1) o0[L + m] = z.y;
    }
  }
}

template <int L, int W, int T, class LA, class KB>
__device__ __forceinline__ void fwd_interp_unit(const LA& a, const KB& kb, const WorkItem wi, float2* sbuf, const int tid) {
  const Lds s{sbuf};
  const float inv = 1.0f / float(L);
  const DSlice d = load_desc(a.descs + wi.slice);
  const int a0 = 2 * wi.unit, a1 = a0 + 1;
  const bool has1 = a1 < d.na;
  // both half-lines per iteration (two independent gathers in flight), packed
  // as the Hermitian completions Z = X + iY
  for (int j = tid; j <= L / 2; j += T) {
    float2 X = c_scale(interp_point<W>(d, a.halo, a.colpad, kb, a0, j), inv);
    float2 Y = has1 ? c_scale(interp_point<W>(d, a.halo, a.colpad, kb, a1, j), inv) : make_float2(0.f, 0.f);
    if (j == 0 || j == L / 2) {   // the full line's sum is real: keep Re at k = 0 and k = -1/2
      X.y = 0.f;
      Y.y = 0.f;
    }
    s[j] = make_float2(X.x - Y.y, X.y + Y.x);
    if (j > 0 && j < L / 2) s[L - j] = make_float2(X.x + Y.y, Y.x - X.y);
  }
  __syncthreads();
  fft_lds<L, T, true>(s, d.tw_Nt, tid);
  // bin m (t = m - N_t/2) is output index t mod N_t
  store_sino_rows<L, T>(a, d, a0, has1, s, tid);
  __syncthreads();
}

template <int L, int W>
__global__ __launch_bounds__(fft_threads(L)) void k_fwd_interp(LaunchArgs a, KBArgs kb) {
  __shared__ float2 sbuf[lds_elems<L>()];
  NR_FOR_EACH_UNIT(a, wi) fwd_interp_unit<L, W, fft_threads(L)>(a, kb, wi, sbuf, int(threadIdx.x));
}

// The item's descriptor, entry, point codes and angle tables (slots past the
// item's end repeat its first point; items are never empty).
template <int T, int PER, class LA>
__device__ __forceinline__ void interp_fetch_points(const LA& a, const WorkItem wi, DSlice& d, SpreadItem& it,
                                                    int (&codes)[PER], double (&gx)[PER], double (&gy)[PER],
                                                    int (&fl)[PER], const int tid) {
  d = load_desc(a.descs + wi.slice);
  it = d.iitems[wi.unit];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + k * T;
    codes[k] = d.ipts[it.begin + (e < it.end - it.begin ? e : 0)];
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int ang = codes[k] >> d.jbits;
    gx[k] = d.gxy[2 * ang];
    gy[k] = d.gxy[2 * ang + 1];
    fl[k] = d.flip[ang];
  }
}

// The tile region of an item: its first row and (even) first column, one
// cell before the tile's margin, so that every 16-byte load takes two cells
// of a row (grid rows are 64-byte aligned and hold an even number of cells).
// Thread tid loads pairs tid, tid + T, ... of the region into registers;
// staged cells off the grid are never read by a point, so the address is
// clamped and the load kept unconditional.
template <int W, int T>
struct InterpStage {
  static constexpr int PAIRS = InterpLds<W>::RWP / 2;
  static constexpr int N = (InterpLds<W>::RH * PAIRS + T - 1) / T;
};
template <int W, int T>
__device__ __forceinline__ void interp_stage_load(const DSlice& d, const SpreadItem& it, float4 (&v)[InterpStage<W, T>::N],
                                                  const int tid) {
  constexpr int TW = kInterpTileW, TH = kInterpTileH, PAIRS = InterpStage<W, T>::PAIRS;
  constexpr int COUNT = InterpLds<W>::RH * PAIRS;
  const int r0 = (it.tile / d.itiles_x) * TH - 1, c0 = (it.tile % d.itiles_x) * TW - 2;
  const NR_G float4* __restrict__ ext4 = reinterpret_cast<const NR_G float4*>(d.ext);
#pragma unroll
  for (int z = 0; z < InterpStage<W, T>::N; ++z) {
    const int c = min(tid + z * T, COUNT - 1);
    const int rl = c / PAIRS, pl = c % PAIRS;
    const int r = min(max(r0 + rl, 0), d.rows - 1);
    const int cc = min(max(c0 + 2 * pl, 0), d.cols - 2);
    v[z] = ext4[(size_t(r) * d.cols + cc) >> 1];
  }
}
template <int W, int T>
__device__ __forceinline__ void interp_stage_store(float2* reg, const float4 (&v)[InterpStage<W, T>::N], const int tid) {
  constexpr int PAIRS = InterpStage<W, T>::PAIRS, RS = InterpLds<W>::RS;
  constexpr int COUNT = InterpLds<W>::RH * PAIRS;
#pragma unroll
  for (int z = 0; z < InterpStage<W, T>::N; ++z) {
    const int c = tid + z * T;
    if (COUNT % T == 0 || c < COUNT) {
      const int rl = c / PAIRS, pl = c % PAIRS;
      reg[rl * RS + 2 * pl] = make_float2(v[z].x, v[z].y);
      reg[rl * RS + 2 * pl + 1] = make_float2(v[z].z, v[z].w);
    }
  }
}

// Every thread interpolates its points from the staged tile (the same sums,
// in the same order, as interp_point) into the half-line buffer yh, scaled
// by 1/N_t.
template <int W, int T, int PER, class LA, class KB>
__device__ __forceinline__ void interp_compute(const LA& a, const KB& kb, const DSlice& d, const SpreadItem& it,
                                               const int (&codes)[PER], const double (&gx)[PER],
                                               const double (&gy)[PER], const int (&fl)[PER], const float2* reg,
                                               const int tid) {
  constexpr int TW = kInterpTileW, TH = kInterpTileH, RS = InterpLds<W>::RS;
  const int r0 = (it.tile / d.itiles_x) * TH - 1, c0 = (it.tile % d.itiles_x) * TW - 2;
  const int rb = a.halo - r0, cb = d.G / 2 + a.colpad - c0;
  const float inv = 1.0f / float(d.Nt);
  const int count = it.end - it.begin;   // at most kMaxChunk
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (k * T >= count) break;          // uniform over the workgroup
    if (tid + k * T >= count) continue;
    const int code = codes[k];
    const int j = code & ((1 << d.jbits) - 1);
    int g0x, g0y;
    float wx[W], wy[W];
    point_taps<W>(gx[k], gy[k], j, kb, g0x, g0y, wx, wy);
    const int o = (g0x + rb) * RS + (g0y + cb);
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < W; ++i) {
      float2 r = make_float2(0.f, 0.f);
#pragma unroll
      for (int l = 0; l < W; ++l) {
        const float2 v = reg[o + i * RS + l];
        r.x = fmaf(wy[l], v.x, r.x);
        r.y = fmaf(wy[l], v.y, r.y);
      }
      acc.x = fmaf(wx[i], r.x, acc.x);
      acc.y = fmaf(wx[i], r.y, acc.y);
    }
    if (fl[k]) acc.y = -acc.y;
    d.yh[__umul24(uint32_t(code >> d.jbits), uint32_t(d.H)) + j] = c_scale(acc, inv);
  }
}

// F3 from LDS tiles: one work item = one interpolation tile and a range of the
// points whose first tap lies in it.  The workgroup stages the tile with the
// W-1 cells the footprints reach past it and a one-cell margin on each side,
// then every thread interpolates its points from LDS.
// The staged cells are complex values with an odd row stride (neighbouring
// lanes take neighbouring points of one line, about two cells apart): a
// point's taps along a row are read two cells per LDS instruction, which
// measured 2 % faster than separate real and imaginary planes.
template <int W, class LA, class KB>
__device__ __forceinline__ void interp_tiles_unit(const LA& a, const KB& kb, const WorkItem wi, float2* reg, const int tid) {
  constexpr int T = 256, PER = kMaxChunk / T;
  DSlice d;
  SpreadItem it;
  int codes[PER], fl[PER];
  double gx[PER], gy[PER];
  float4 stg[InterpStage<W, T>::N];
  interp_fetch_points<T>(a, wi, d, it, codes, gx, gy, fl, tid);
  interp_stage_load<W, T>(d, it, stg, tid);
  interp_stage_store<W, T>(reg, stg, tid);
  __syncthreads();
  interp_compute<W, T>(a, kb, d, it, codes, gx, gy, fl, reg, tid);
}

// Two work items per workgroup, b and n-1-b of the heaviest-first list: both
// items' point loads (descriptor, entry, codes, angle tables: a chain of
// dependent round trips) are issued at once, so the second item's chain is
// hidden behind the first item's staging and interpolation; the second tile
// is staged after the first is interpolated.  Measured on 2560^2 slices,
// 1024 angles: 35.9 -> 32.5 us per slice (b with b + gridDim.x), 32.25 with
// the heavy-light pairing; staging the second tile into registers up front
// as well took 102 VGPRs (four workgroups per CU instead of six) and ran
// 36.2 us.
template <int W>
__global__ __launch_bounds__(256) void k_interp_tiles(LaunchArgs a, KBArgs kb) {
  constexpr int T = 256, PER = kMaxChunk / T;
  __shared__ float2 reg[InterpLds<W>::RH * InterpLds<W>::RS];
  const int tid = int(threadIdx.x);
  const int b0 = int(blockIdx.x), b1 = a.n_work - 1 - b0;
  const WorkItem w0 = b0 < a.n_work ? a.work[b0] : WorkItem{-1, 0};
  const WorkItem w1 = b1 > b0 ? a.work[b1] : WorkItem{-1, 0};
  DSlice d0, d1;
  SpreadItem i0, i1;
  int c0[PER], f0[PER], c1[PER], f1[PER];
  double x0[PER], y0[PER], x1[PER], y1[PER];
  float4 s0[InterpStage<W, T>::N], s1[InterpStage<W, T>::N];
  if (w0.slice >= 0) interp_fetch_points<T>(a, w0, d0, i0, c0, x0, y0, f0, tid);
  if (w1.slice >= 0) interp_fetch_points<T>(a, w1, d1, i1, c1, x1, y1, f1, tid);
  if (w0.slice >= 0) interp_stage_load<W, T>(d0, i0, s0, tid);
  if (w0.slice >= 0) {
    interp_stage_store<W, T>(reg, s0, tid);
    __syncthreads();
    interp_compute<W, T>(a, kb, d0, i0, c0, x0, y0, f0, reg, tid);
  }
  if (w1.slice >= 0) {
    interp_stage_load<W, T>(d1, i1, s1, tid);
    __syncthreads();   // the first tile's reads are done
    interp_stage_store<W, T>(reg, s1, tid);
    __syncthreads();
    interp_compute<W, T>(a, kb, d1, i1, c1, x1, y1, f1, reg, tid);
  }
}

// F4 after k_interp_tiles: per pair of angles, the Hermitian completions of
// the two half-lines packed as Z = X + iY, the inverse DFT along the line and
// the real sinogram rows.
template <int L, int T, class LA>
__device__ __forceinline__ void fwd_radial_unit(const LA& a, const WorkItem wi, float2* sbuf, const int tid) {
  const Lds s{sbuf};
  constexpr int H = L / 2 + 1;
  const DSlice d = load_desc(a.descs + wi.slice);
  const int a0 = 2 * wi.unit, a1 = a0 + 1;
  const bool has1 = a1 < d.na;
  const NR_G float2* __restrict__ x0 = d.yh + size_t(a0) * H;
  const NR_G float2* __restrict__ x1 = has1 ? x0 + H : x0;   // loads stay unconditional
  NR_STRIDED(j, H, T) {
    float2 X = x0[j], Y = x1[j];
    if (!has1) Y = make_float2(0.f, 0.f);
    if (d.shift) {   // rotation axis at bin L/2 + c: evaluate the line at t - c
      const float2 p = d.shift[j];
      X = c_mul(X, p);
      Y = c_mul(Y, p);
    }
    if (j == 0 || j == L / 2) {   // the full line's sum is real: keep Re at k = 0 and k = -1/2
      X.y = 0.f;
      Y.y = 0.f;
    }
    s[j] = make_float2(X.x - Y.y, X.y + Y.x);
    if (j > 0 && j < L / 2) s[L - j] = make_float2(X.x + Y.y, Y.x - X.y);
  }
  __syncthreads();
  fft_lds<L, T, true>(s, d.tw_Nt, tid);
  store_sino_rows<L, T>(a, d, a0, has1, s, tid);
  __syncthreads();
}

template <int L>
__global__ __launch_bounds__(fft_threads(L)) void k_fwd_radial(LaunchArgs a) {
  __shared__ float2 sbuf[lds_elems<L>()];
  NR_FOR_EACH_UNIT(a, wi) fwd_radial_unit<L, fft_threads(L)>(a, wi, sbuf, int(threadIdx.x));
}

// ---------------------------------------------------------------------------
// A1: radial transform of two sinogram rows
// ---------------------------------------------------------------------------

// Filtered back-projection weight of half-line index j of an L-point line:
// (pi/n_angles) |k| B(k) with k = j/L cycles per pixel and B = 1 (ramp) or
// 1/(1 + (k/cutoff)^(2 order)) (Butterworth).
template <class LA>
__device__ __forceinline__ float fbp_weight(const LA& a, int j, int L, int n_angles) {
  const float k = float(j) / float(L);
  float w = k;
  if (a.fbp_filter == 1) {
    const float x = k * a.fbp_inv_cutoff, x2 = x * x;
    float pw = 1.f;
    for (int i = 0; i < a.fbp_order; ++i) pw *= x2;
    w = k / (1.f + pw);
  }
  return w * (3.14159265358979f / float(n_angles));
}

template <int L, int T, class LA>
__device__ __forceinline__ void adj_radial_unit(const LA& a, const WorkItem wi, float2* sbuf, const int tid) {
  const Lds s{sbuf};

  const DSlice d = load_desc(a.descs + wi.slice);
  const int a0 = 2 * wi.unit, a1 = a0 + 1;
  const bool has1 = a1 < d.na;
  const float* __restrict__ y0 = a.sino_in + d.sino_off + size_t(a0) * L;
  const float* __restrict__ y1 = has1 ? y0 + L : y0;   // loads stay unconditional
  NR_STRIDED(m, L, T) {
    const float b = y1[m];
    s[wrap_index<L>(m + L / 2)] = make_float2(y0[m], has1 ? b : 0.f);
  }
  __syncthreads();
  fft_lds<L, T, false>(s, d.tw_Nt, tid);
  const int H = L / 2 + 1;
  NR_G float2* __restrict__ o0 = d.yh + size_t(a0) * H;
  const float inv = 1.0f / float(L);
  NR_STRIDED(j, H, T) {
    const float2 z1 = s[j], z2 = s[j == 0 ? 0 : L - j];
    float w = (j == 0 || j == L / 2) ? inv : 2.0f * inv;
    if (a.fbp_filter >= 0) w *= fbp_weight(a, j, L, d.na);
    float2 A = make_float2(0.5f * w * (z1.x + z2.x), 0.5f * w * (z1.y - z2.y));
    float2 B = make_float2(0.5f * w * (z1.y + z2.y), 0.5f * w * (z2.x - z1.x));
    if (d.shift) {   // transpose of the forward's phase
      const float2 q = c_conj(d.shift[j]);
      A = c_mul(A, q);
      B = c_mul(B, q);
    }
    o0[j] = A;
    if (has1) o0[H + j] = B;
  }
  __syncthreads();
}

template <int L>
__global__ __launch_bounds__(fft_threads(L)) void k_adj_radial(LaunchArgs a) {
  __shared__ float2 sbuf[lds_elems<L>()];
  NR_FOR_EACH_UNIT(a, wi) adj_radial_unit<L, fft_threads(L)>(a, wi, sbuf, int(threadIdx.x));
}

// ---------------------------------------------------------------------------
// A2: spreading (type-1 gridding) onto the extended grid
// ---------------------------------------------------------------------------

__global__ void k_fill_zero(float4* p, size_t n4) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += size_t(gridDim.x) * blockDim.x)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// clear the tiles that several work items accumulate into
template <int TW, int TH, class LA>
__device__ __forceinline__ void spread_zero_unit(const LA& a, const WorkItem wi, const int tid) {

  const DSlice d = load_desc(a.descs + wi.slice);
  const int t = d.zero_tiles[wi.unit];
  const int r0 = (t / d.tiles_x) * TH, c0 = (t % d.tiles_x) * TW;
  NR_G float2* ext = d.ext;
  for (int c = tid; c < TW * TH; c += 256) {
    const int r = r0 + c / TW, cc = c0 + c % TW;
    if (r < d.rows && cc < d.cols) ext[size_t(r) * d.cols + cc] = make_float2(0.f, 0.f);
  }
}

template <int TW, int TH>
__global__ __launch_bounds__(256) void k_spread_zero(LaunchArgs a) {
  NR_FOR_EACH_UNIT(a, wi) spread_zero_unit<TW, TH>(a, wi, int(threadIdx.x));
}

// One work item = one grid tile (TH rows x TW columns) and a range of the
// points whose footprint touches it.  The tile accumulates in LDS in 32-bit
// fixed point with integer LDS atomics: on gfx950 float LDS atomics run
// about 40x slower than integer ones.  The item's scale q = 2^30/(M b), with
// M the largest |component| of its values and b the most of its points that
// touch any one cell (from the plan), bounds every cell's final sum by 2^30
// (|phi| <= 1), so the wrapped 32-bit partial sums are exact modulo 2^32 and
// the final sum is exact up to the rounding of each contribution to 1/q.
// (One 64-bit atomic per tap carrying both components measured 15% slower
// than two 32-bit ones.)
// The LDS tile carries a W-cell apron on every side, which holds the whole
// footprint of every listed point, so each point adds its W x W taps with no
// bounds test (no divergence); the apron is dropped at the end.  Single-item
// tiles are then stored plainly (every cell, zeros included); shared tiles
// are added with global float atomics.
// A spreading item's points are held in registers between the loads and the
// accumulation, as five arrays (gathered in one aggregate they were placed in
// scratch memory): slot k of thread tid is entry tid + k*T of the item.
#define NR_SPREAD_PTS(p) p##_code, p##_v, p##_gx, p##_gy, p##_fl
#define NR_SPREAD_PTS_DECL(p, PER) \
  int p##_code[PER];               \
  float2 p##_v[PER];               \
  double p##_gx[PER], p##_gy[PER]; \
  int p##_fl[PER]

// First loads of an item: its descriptor, its entry and its point codes.
// Slots past the item's end repeat its first point; an empty item (a tile no
// point touches, which still writes its zeros) reads no point list at all
// and uses point 0.  A code is (angle << jbits) | j: a shift and a mask take
// it apart, where dividing an index a*H + j by H cost about 20 VALU slots per
// point.
template <int T, int PER, class LA>
__device__ __forceinline__ void spread_fetch_codes(const LA& a, const WorkItem wi, DSlice& d, SpreadItem& it,
                                                   int (&code)[PER], const int tid) {
  d = load_desc(a.descs + wi.slice);
  it = d.items[wi.unit];
  const int count = it.end - it.begin;   // at most kMaxChunk
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + k * T;
    code[k] = count > 0 ? d.pts[it.begin + (e < count ? e : 0)] : 0;
  }
}

// Second loads: each point's value and its angle's entries.
template <int PER>
__device__ __forceinline__ void spread_fetch_values(const DSlice& d, const int (&code)[PER], float2 (&v)[PER],
                                                    double (&gx)[PER], double (&gy)[PER], int (&fl)[PER]) {
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int ang = code[k] >> d.jbits;
    v[k] = d.yh[__umul24(uint32_t(ang), uint32_t(d.H)) + (code[k] & ((1 << d.jbits) - 1))];
    gx[k] = d.gxy[2 * ang];
    gy[k] = d.gxy[2 * ang + 1];
    fl[k] = d.flip[ang];
  }
}

template <int W, int TW, int TH, int T, int PER, class LA, class KB>
__device__ __forceinline__ void spread_accumulate(const LA& a, const KB& kb, const DSlice& d, const SpreadItem& it,
                                                  const int (&code)[PER], const float2 (&v)[PER],
                                                  const double (&gx)[PER], const double (&gy)[PER],
                                                  const int (&fl)[PER], int* acc, float* red, int& nonfinite,
                                                  const int tid) {
  static_assert(PER == kMaxChunk / T, "slots per thread");
  constexpr int AH = SpreadLds<W, TW, TH>::AH, TS = SpreadLds<W, TW, TH>::TS, ACC = SpreadLds<W, TW, TH>::ACC;
  int* const acc_re = acc;             // acc: ACC ints, 16-byte aligned
  int* const acc_im = acc + AH * TS;   // T threads; red holds T/64 floats
  const int count = it.end - it.begin;
  const NR_G float2* __restrict__ yh = d.yh;
  NR_STRIDED(c, ACC / 4, T) reinterpret_cast<int4*>(acc)[c] = make_int4(0, 0, 0, 0);
  const int r0 = (it.tile / d.tiles_x) * TH, c0 = (it.tile % d.tiles_x) * TW;
  // apron coordinates of grid cell (row g0x + halo, column g0y + G/2 + colpad)
  const int rbase = a.halo - r0 + W, cbase = d.G / 2 + a.colpad - c0 + W;
  // k = 0 of every angle sits at the origin: their sum is spread once, in
  // float32 when the tile is written out, so that it does not enter the
  // item's fixed-point scale (with many angles it is far larger than any
  // single point value and would coarsen every other contribution)
  float dc = 0.f;
  if (it.flags & kItemDC) {
    float sum = 0.f;
    for (int ang = tid; ang < d.na; ang += T) sum += yh[size_t(ang) * d.H].x;
    dc = block_sum<T>(sum, red, tid);
  }
  // fixed-point scale of this item; a non-finite value (which the integer
  // conversion would turn into 0) poisons the whole tile with NaN instead
  float m = 0.f;
  bool bad = !isfinite(dc);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (tid + k * T < count) {
      m = fmaxf(m, fmaxf(fabsf(v[k].x), fabsf(v[k].y)));
      bad |= !isfinite(v[k].x) || !isfinite(v[k].y);
    }
  }
  if (tid == 0) nonfinite = 0;
  const float mmax = block_max<T>(m, red, tid);   // synchronises: the tile is cleared
  if (bad) nonfinite = 1;
  // 2^30 / (M b) through the hardware reciprocal (within 1 ulp: the sums keep
  // a factor of 2 of headroom below 2^31)
  const float q = mmax > 0.f ? 1073741824.0f * __builtin_amdgcn_rcpf(mmax * float(it.bound)) : 0.f;
  // one point per round, taken from slot 0 of copies that rotate down by one
  // slot each round: compile-time indices only (a chain of selects on the
  // round number was turned into an indexed load from scratch memory), and
  // the taps are unrolled once
  int rc[PER], rf[PER];
  float2 rv[PER];
  double rx[PER], ry[PER];
#pragma unroll
  for (int z = 0; z < PER; ++z) {
    rc[z] = code[z];
    rf[z] = fl[z];
    rv[z] = v[z];
    rx[z] = gx[z];
    ry[z] = gy[z];
  }
#pragma unroll 1
  for (int k = 0; k < PER; ++k) {
    if (k * T >= count) break;          // uniform over the workgroup
    const int p = rc[0], f = rf[0];
    float2 u = rv[0];
    const double px = rx[0], py = ry[0];
#pragma unroll
    for (int z = 0; z + 1 < PER; ++z) {
      rc[z] = rc[z + 1];
      rf[z] = rf[z + 1];
      rv[z] = rv[z + 1];
      rx[z] = rx[z + 1];
      ry[z] = ry[z + 1];
    }
    if (tid + k * T < count) {
      const int j = p & ((1 << d.jbits) - 1);
      if (f) u.y = -u.y;
      u.x *= q;
      u.y *= q;
      int g0x, g0y;
      float wx[W], wy[W];
      point_taps<W>(px, py, j, kb, g0x, g0y, wx, wy);
      const int base = (g0x + rbase) * TS + (g0y + cbase);
#pragma unroll
      for (int i = 0; i < W; ++i) {
        const float vx = wx[i] * u.x, vy = wx[i] * u.y;
#pragma unroll
        for (int l = 0; l < W; ++l) {
          atomicAdd(&acc_re[base + i * TS + l], round_half_up(vx * wy[l]));
          atomicAdd(&acc_im[base + i * TS + l], round_half_up(vy * wy[l]));
        }
      }
    }
  }
  __syncthreads();
  const bool shared_tile = it.flags & kItemAtomic;
  const float inv_q = nonfinite ? __int_as_float(0x7fc00000) : (q > 0.f ? __builtin_amdgcn_rcpf(q) : 0.f);
  // the origin's W x W footprint in apron coordinates (DC items only)
  int dcx = 0, dcy = 0;
  float dwx[W], dwy[W];
  const bool has_dc = it.flags & kItemDC;
  if (has_dc) {
    point_taps<W>(0.0, 0.0, 0, kb, dcx, dcy, dwx, dwy);
    dcx += rbase;
    dcy += cbase;
  }
  // a thread writes one column of the tile, every T/TW-th row: its grid and
  // LDS addresses advance by constant strides
  static_assert(T % TW == 0 && TH % (T / TW) == 0, "tile shape");
  constexpr int STEP = T / TW;
  const int cl = tid % TW, rl0 = tid / TW;
  const int cc = c0 + cl;
  NR_G float2* dst = d.ext + size_t(r0 + rl0) * d.cols + cc;
  const size_t dstep = size_t(STEP) * d.cols;
  const bool col_ok = cc < d.cols;
#pragma unroll
  for (int s = 0; s < TH / STEP; ++s) {
    const int rl = rl0 + s * STEP;
    if (col_ok && r0 + rl < d.rows) {
      const int ai = (rl + W) * TS + cl + W;
      float re = float(acc_re[ai]) * inv_q;
      const float im = float(acc_im[ai]) * inv_q;
      if (has_dc) {
        const int i = rl + W - dcx, l = cl + W - dcy;
        if (i >= 0 && i < W && l >= 0 && l < W) {
          float wi = 0.f, wl = 0.f;
#pragma unroll
          for (int k = 0; k < W; ++k) {   // compile-time register indices
            if (k == i) wi = dwx[k];
            if (k == l) wl = dwy[k];
          }
          re += dc * wi * wl;
        }
      }
      if (shared_tile) {
        atomicAdd((NR_G float*)&dst->x, re);
        atomicAdd((NR_G float*)&dst->y, im);
      } else {
        if (a.stream_stores)
          store_nt(dst, make_float2(re, im));
        else
          *dst = make_float2(re, im);
      }
    }
    dst += dstep;
  }
  __syncthreads();
}

// one work item: loads, then accumulation
template <int W, int TW, int TH, int T, class LA, class KB>
__device__ __forceinline__ void spread_tiles_unit(const LA& a, const KB& kb, const WorkItem wi, int* acc, float* red, int& nonfinite, const int tid) {
  constexpr int PER = kMaxChunk / T;
  DSlice d;
  SpreadItem it;
  NR_SPREAD_PTS_DECL(p, PER);
  spread_fetch_codes<T>(a, wi, d, it, p_code, tid);
  spread_fetch_values(d, NR_SPREAD_PTS(p));
  spread_accumulate<W, TW, TH, T>(a, kb, d, it, NR_SPREAD_PTS(p), acc, red, nonfinite, tid);
}

// Two work items per workgroup: b and n-1-b of the list, which is sorted
// heaviest first, so that every workgroup pairs a heavy item (bound by its
// taps) with a light one (bound by its tile stores) and the launch keeps a
// like mix of both from start to end.  An item's loads form a chain of four
// dependent round trips (work entry, descriptor and item, point codes,
// values); both items' chains run at once and the second item's values
// arrive while the first item accumulates.  Measured on 2560^2 slices, 1024
// angles: 44.8 -> 44.1 us per slice for the pairing, 44.1 -> 42.0 with
// non-temporal tile stores; 512 or 1024 threads per tile were slower (47.2,
// 62.1 us).
constexpr int kSpreadThreads = 256;
template <int W, int TW, int TH>
__global__ __launch_bounds__(kSpreadThreads) void k_spread_tiles(LaunchArgs a, KBArgs kb) {
  constexpr int T = kSpreadThreads;
  __shared__ __attribute__((aligned(16))) int acc[SpreadLds<W, TW, TH>::ACC];
  __shared__ float red[T / 64];
  __shared__ int nonfinite;
  const int tid = int(threadIdx.x);
  const int b0 = int(blockIdx.x), b1 = a.n_work - 1 - b0;
  const WorkItem w0 = b0 < a.n_work ? a.work[b0] : WorkItem{-1, 0};
  const WorkItem w1 = b1 > b0 ? a.work[b1] : WorkItem{-1, 0};
  constexpr int PER = kMaxChunk / T;
  DSlice d0, d1;
  SpreadItem i0, i1;
  NR_SPREAD_PTS_DECL(p0, PER);
  NR_SPREAD_PTS_DECL(p1, PER);
  if (w0.slice >= 0) spread_fetch_codes<T>(a, w0, d0, i0, p0_code, tid);
  if (w1.slice >= 0) spread_fetch_codes<T>(a, w1, d1, i1, p1_code, tid);
  if (w0.slice >= 0) spread_fetch_values(d0, NR_SPREAD_PTS(p0));
  if (w1.slice >= 0) spread_fetch_values(d1, NR_SPREAD_PTS(p1));
  if (w0.slice >= 0) spread_accumulate<W, TW, TH, T>(a, kb, d0, i0, NR_SPREAD_PTS(p0), acc, red, nonfinite, tid);
  if (w1.slice >= 0) spread_accumulate<W, TW, TH, T>(a, kb, d1, i1, NR_SPREAD_PTS(p1), acc, red, nonfinite, tid);
}

// Reference spreading: one thread per polar point of one slice, global float
// atomics straight into the (cleared) extended grid.  Slow; a cross-check.
template <int W>
__global__ __launch_bounds__(256) void k_spread_atomic(const SliceDesc* descs, int slice, int halo, int colpad,
                                                       KBArgs kb) {
  const DSlice d = load_desc(descs + slice);
  const int pid = blockIdx.x * 256 + threadIdx.x;
  if (pid >= d.na * d.H) return;
  const int ang = pid / d.H, j = pid - ang * d.H;
  float2 v = d.yh[pid];
  if (d.flip[ang]) v.y = -v.y;
  int g0x, g0y;
  float wx[W], wy[W];
  point_taps<W>(d.gxy[2 * ang], d.gxy[2 * ang + 1], j, kb, g0x, g0y, wx, wy);
  NR_G float2* p = d.ext + size_t(g0x + halo) * d.cols + (g0y + d.G / 2 + colpad);
  for (int i = 0; i < W; ++i)
    for (int l = 0; l < W; ++l) {
      atomicAdd(&p[size_t(i) * d.cols + l].x, wx[i] * wy[l] * v.x);
      atomicAdd(&p[size_t(i) * d.cols + l].y, wx[i] * wy[l] * v.y);
    }
}

// ---------------------------------------------------------------------------
// A3: fold the halo cells, inverse transform along y, keep N rows
// ---------------------------------------------------------------------------

// sum of a main cell and its periodic copy in the padded columns
template <int L>
__device__ __forceinline__ float2 load_folded(const NR_G float2* row, int colpad, int n) {
  const int p = wrap_index<L>(n + L / 2) + colpad;
  float2 v = row[p];
  if (p >= L) v = c_add(v, row[p - L]);
  if (p < 2 * colpad) v = c_add(v, row[p + L]);
  return v;
}

template <int L, int T, class LA>
__device__ __forceinline__ void adj_cols_unit(const LA& a, const WorkItem wi, float2* sbuf, const int tid) {
  const Lds s{sbuf};
  const int halo = a.halo, colpad = a.colpad;
  const DSlice d = load_desc(a.descs + wi.slice);
  const int qx = wi.unit;
  const int cols = d.cols;
  constexpr int N = L / 2;   // G = 2N
  const NR_G float2* ext = d.ext;
  const NR_G float2* row = ext + size_t(qx + halo) * cols;
  const NR_G float2* m1 = (qx >= 1 && qx <= halo) ? ext + size_t(halo - qx) * cols : nullptr;
  const NR_G float2* m2 = (qx >= L / 2 - halo && qx <= L / 2 - 1) ? ext + size_t(L - qx + halo) * cols : nullptr;
  // natural index n (q_y = n, or n - L from L/2 on) gathers the cell, its
  // periodic copies (n within colpad of L/2) and, for the columns next to
  // qx = 0 and G/2, the conjugate mirror rows.  Nothing is spread farther
  // than rdisc from the origin (nor onto any copy of such a cell), so those
  // cells are zero and not read.
  const int r2 = d.rdisc * d.rdisc - qx * qx;
  // Cells with |q_y| >= L/2 - colpad have periodic copies to fold in; a
  // column whose disc stops short of them, and that has no mirror rows (all
  // but a few), reads each cell once.
  const int lim = r2 < 0 ? -1 : int(sqrtf(float(r2)));
  if (m1 || m2 || lim >= L / 2 - colpad) {
    fft_first_pass_from<L, T, true, false>(s, tid, [&](int n) {
      const int qy = n < L / 2 ? n : n - L;
      if (qy * qy > r2) return make_float2(0.f, 0.f);
      float2 v = load_folded<L>(row, colpad, n);
      const int nm = n == 0 ? 0 : L - n;
      if (m1) v = c_add(v, c_conj(load_folded<L>(m1, colpad, nm)));
      if (m2) v = c_add(v, c_conj(load_folded<L>(m2, colpad, nm)));
      return v;
    });
  } else {
    const NR_G float2* __restrict__ mid = row + colpad + L / 2;   // the cell of q_y = 0
    fft_first_pass_from<L, T, true, false>(s, tid, [&](int n) {
      const int qy = n < L / 2 ? n : n - L;
      if (qy * qy > r2) return make_float2(0.f, 0.f);
      const float2 v = mid[qy];
      return v;
    });
  }
  // only y = iy - N/2 in [-N/2, N/2) is kept: natural indices [0, N/2) and
  // [L - N/2, L); row iy of column qx is half iy & 1 of tile entry t4(qx, iy / 2)
  NR_G float2* __restrict__ T2 = (NR_G float2*)d.T;
  fft_lds_store_out<L, T, true, 1>(s, d.tw_G, tid, [&](int n, float2 v) {
    const int iy = n < N / 2 ? n + N / 2 : n - (L - N / 2);
    T2[2 * t4(qx, iy >> 1, N) + (iy & 1)] = v;
  });
  __syncthreads();
}

template <int L>
__global__ __launch_bounds__(fft_threads(L)) void k_adj_cols(LaunchArgs a) {
  __shared__ float2 sbuf[lds_elems<L>()];
  NR_FOR_EACH_UNIT(a, wi) adj_cols_unit<L, fft_threads(L)>(a, wi, sbuf, int(threadIdx.x));
}

// ---------------------------------------------------------------------------
// A4: transpose of the row R2C: a'(x) = Re sum_{q=0}^{G/2} T'[q] e^{2 pi i q x/G}
// ---------------------------------------------------------------------------

template <int L, int T, class LA>
__device__ __forceinline__ void adj_rows_unit(const LA& a, const WorkItem wi, float2* sbuf, const int tid) {
  const Lds s{sbuf};

  const DSlice d = load_desc(a.descs + wi.slice);
  constexpr int N = L / 2;   // G = 2N
  const int iy0 = 2 * wi.unit;
  const NR_G float4* __restrict__ in = (const NR_G float4*)d.T;
  // Hermitian completion with doubled real parts at q = 0 and G/2, two rows
  // packed: index n <= L/2 takes entry q = n as X + iY, index L - q the
  // conjugate-symmetric combination of the same entry
  fft_first_pass_from<L, T, true, false>(s, tid, [&](int n) {
    const int q = n <= L / 2 ? n : L - n;
    const float4 t = in[t4(q, iy0 >> 1, N)];
    float2 X = make_float2(t.x, t.y), Y = make_float2(t.z, t.w);
    if (q == 0 || q == L / 2) {
      X = make_float2(2.f * X.x, 0.f);
      Y = make_float2(2.f * Y.x, 0.f);
    }
    return n <= L / 2 ? make_float2(X.x - Y.y, X.y + Y.x) : make_float2(X.x + Y.y, Y.x - X.y);
  });
  const float d0 = 0.5f * d.deapod[iy0], d1 = 0.5f * d.deapod[iy0 + 1];
  float* __restrict__ g0 = a.vol_out + d.vol_off + size_t(iy0) * N;
  const NR_G float* __restrict__ dp = d.deapod;
  // x = ix - N/2 in [-N/2, N/2) is kept: natural indices [0, N/2) and [L - N/2, L)
  fft_lds_store_out<L, T, true, 1>(s, d.tw_G, tid, [&](int n, float2 z) {
    const int ix = n < N / 2 ? n + N / 2 : n - (L - N / 2);
    const float dx = dp[ix];
    g0[ix] = dx * d0 * z.x;
    g0[N + ix] = dx * d1 * z.y;
  });
  __syncthreads();
}

template <int L>
__global__ __launch_bounds__(fft_threads(L)) void k_adj_rows(LaunchArgs a) {
  __shared__ float2 sbuf[lds_elems<L>()];
  NR_FOR_EACH_UNIT(a, wi) adj_rows_unit<L, fft_threads(L)>(a, wi, sbuf, int(threadIdx.x));
}

// ---------------------------------------------------------------------------
// M4: a batch's whole forward + adjoint chain in one persistent launch
// ---------------------------------------------------------------------------
//
// A resident grid of 256-thread workgroups; each workgroup reads the id of the
// XCD it runs on and takes tickets from that XCD's queue (an atomic counter).
// A unit waits (one thread, bounded) until every unit of the stage before it
// in its slice's chain has finished: units are counted per (slice, stage)
// after their stores have completed.  A slice's units all run on one XCD, so
// producer and consumer share that XCD's L2 (vector L1 is write-through): the
// producer waits for its stores before counting, the consumer invalidates its
// L1 after the wait, and no L2 writeback or invalidate is needed.  A wait
// that exceeds the spin limit (or sees another's) sets the error flag and the
// workgroup stops taking tickets, so every workgroup exits.

constexpr int kPersistThreads = 256;

// kernel-argument (constant) address space: loads through it are scalar
#ifdef __HIP_DEVICE_COMPILE__
#define NR_C __attribute__((address_space(4)))
#else
#define NR_C
#endif

template <int W>
struct PersistLds {
  static constexpr int FFT = 4096 * int(sizeof(float2));
  static constexpr int SPREAD = SpreadLds<W, 64, 32>::ACC * int(sizeof(int));
  static constexpr int INTERP = InterpLds<W>::RH * InterpLds<W>::RS * int(sizeof(float2));
  static constexpr int BYTES = FFT > SPREAD ? (FFT > INTERP ? FFT : INTERP) : (SPREAD > INTERP ? SPREAD : INTERP);
};

__device__ __forceinline__ int xcc_id() {
  int x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
  return x & (kPersistQueues - 1);
}

#define NR_PERSIST_LENGTHS(X) X(128) X(256) X(512) X(1024) X(2048) X(4096)

template <int W, class LA, class KB>
__device__ __forceinline__ void persist_unit(const LA& a, const KB& kb, int stage, int L, WorkItem wi,
                                             char* lds, float* red, int& nonfinite, const int tid) {
  float2* f2 = reinterpret_cast<float2*>(lds);
  constexpr int T = kPersistThreads;
  switch (StageKind(stage)) {
    case StageKind::FwdRows:
      switch (L) {
#define NR_CASE(l) case l: fwd_rows_unit<l, T>(a, wi, f2, tid); return;
        NR_PERSIST_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      return;
    case StageKind::FwdCols:
      switch (L) {
#define NR_CASE(l) case l: fwd_cols_unit<l, T>(a, wi, f2, tid); return;
        NR_PERSIST_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      return;
    case StageKind::FwdInterp: {
      interp_tiles_unit<W>(a, kb, wi, reinterpret_cast<float2*>(lds), tid);
      return;
    }
    case StageKind::FwdRadial:
      switch (L) {
#define NR_CASE(l) case l: fwd_radial_unit<l, T>(a, wi, f2, tid); return;
        NR_PERSIST_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      return;
    case StageKind::AdjRadial:
      switch (L) {
#define NR_CASE(l) case l: adj_radial_unit<l, T>(a, wi, f2, tid); return;
        NR_PERSIST_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      return;
    case StageKind::SpreadZero:
      spread_zero_unit<64, 32>(a, wi, tid);
      return;
    case StageKind::Spread: {
      spread_tiles_unit<W, 64, 32, kPersistThreads>(a, kb, wi, reinterpret_cast<int*>(lds), red, nonfinite, tid);
      return;
    }
    case StageKind::AdjCols:
      switch (L) {
#define NR_CASE(l) case l: adj_cols_unit<l, T>(a, wi, f2, tid); return;
        NR_PERSIST_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      return;
    case StageKind::AdjRows:
      switch (L) {
#define NR_CASE(l) case l: adj_rows_unit<l, T>(a, wi, f2, tid); return;
        NR_PERSIST_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      return;
    default:
      return;
  }
}

template <int W>
__global__ __launch_bounds__(kPersistThreads) void k_persistent(PersistLaunch args) {
  __shared__ __attribute__((aligned(16))) char lds[PersistLds<W>::BYTES];
  __shared__ float red[kPersistThreads / 64];
  __shared__ int nonfinite;
  __shared__ int s_ticket, s_verdict;
  // the arguments are read through the kernel-argument segment itself (the
  // kernel's only parameter starts it), so no copy of them is made
  const NR_C PersistLaunch* P = (const NR_C PersistLaunch*)__builtin_amdgcn_kernarg_segment_ptr();
  const PersistArgs p = P->p;
  const int q = xcc_id();
  const int q0 = p.qoff[q], qn = p.qoff[q + 1] - q0;
  const bool lead = threadIdx.x == 0;
  // Every loop and every barrier below runs in workgroup-uniform control flow
  // (loop exits come through readfirstlane of a value one thread published
  // in LDS); the only divergent code is single stores and loads of thread 0,
  // each fenced off by barriers.  A loop whose body mixes a divergent region
  // and barriers can otherwise be restructured so that lanes of one
  // wavefront loop back to a barrier without the lane that owns the ticket.
  for (;;) {
    __syncthreads();   // the previous unit's reads of LDS and of s_ticket are done
    // one ticket per workgroup: thread 0 adds 1, the others 0 (no branch)
    const int mine = atomicAdd(&p.tickets[q], lead ? 1 : 0);
    if (lead) s_ticket = mine;
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_ticket);
    if (t >= qn) break;
    const PersistEntry e = p.entries[q0 + t];
    const int c = p.dep[(e.slice - p.first_slice) * kPersistStages + e.stage];
    if (c >= 0) {
      // wait, bounded, until the previous stage of this slice has finished:
      // verdict 1 = go, 2 = give up (spin limit, or another gave up)
      const int need = p.need[c];
      int verdict = 0;
      for (int spin = 0; verdict == 0; ++spin) {
        if (lead) {
          int v = 0;
          if (__hip_atomic_load(&p.done[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) v = 1;
          else if (spin >= p.spin_limit || __hip_atomic_load(p.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            v = 2;
          s_verdict = v;
        }
        __syncthreads();
        verdict = __builtin_amdgcn_readfirstlane(s_verdict);
        __syncthreads();
        if (verdict == 0) __builtin_amdgcn_s_sleep(2);
      }
      if (verdict == 2) {
        if (lead) __hip_atomic_store(p.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    // the producers' stores are in this XCD's L2; drop stale lines from L1
    asm volatile("buffer_inv sc0" ::: "memory");
    // the launch and kernel arguments are read where each unit uses them
    // (scalar loads from the argument segment), not held in registers across
    // the loop: the laundered pointer is not loop-invariant to the compiler
    const NR_C PersistLaunch* ap = P;
    asm volatile("" : "+s"(ap));
    // the thread index is laundered too: index arithmetic derived from it is
    // recomputed per unit instead of being hoisted (and held) across the loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    persist_unit<W>(ap->a, ap->kb, e.stage, e.L, WorkItem{e.slice, e.unit}, lds, red, nonfinite, tid);
    // every wave's stores have reached L2 before the unit is counted
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    atomicAdd(&p.done[(e.slice - p.first_slice) * kPersistStages + e.stage], lead ? 1 : 0);
  }
}

// clears a batch's tickets and counters (before every persistent launch; a
// kernel, so that graph capture records no memset)
__global__ void k_persist_clear(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_fill_int(int* p, size_t n, int v) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

namespace {

// One workgroup per work entry, so the hardware dispatcher balances uneven
// units (grids capped at the resident capacity, striding over the list,
// measured slower on the spreading and transform stages).
template <class K, class... Args>
hipError_t launch(K kernel, int threads, int n, hipStream_t st, Args... args) {
  hipLaunchKernelGGL(kernel, dim3(std::max(1, n)), dim3(threads), 0, st, args...);
  return hipGetLastError();
}

}  // namespace

#define NR_LENGTHS(X) \
  X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192) X(80) X(160) X(320) X(640) X(1280) X(2560) X(5120)

template <int W>
hipError_t launch_spread(const LaunchArgs& a, const KBArgs& kb, int tw, int th, hipStream_t st, bool zero) {
#define NR_TILE(w, h)                                                               \
  if (tw == w && th == h)                                                           \
    return zero ? launch(k_spread_zero<w, h>, 256, a.n_work, st, a)                 \
                : launch(k_spread_tiles<W, w, h>, kSpreadThreads, (a.n_work + 1) / 2, st, a, kb);
  NR_TILE(64, 32)
  NR_TILE(32, 32)
  NR_TILE(64, 64)
  NR_TILE(128, 32)
#undef NR_TILE
  return hipErrorInvalidValue;
}

// forward column launches with at least this many columns run two per
// workgroup (at least about ten rounds of resident workgroups either way)
constexpr int kPairColumnsMin = 8192;

hipError_t launch_stage(StageKind stage, int L, const LaunchArgs& a, const KBArgs& kb, int W, int tile_w,
                        int tile_h, hipStream_t st) {
  if (a.n_work <= 0) return hipSuccess;
  switch (stage) {
    case StageKind::FwdRows:
      switch (L) {
#define NR_CASE(l) case l: return launch(k_fwd_rows<l>, fft_threads(l), a.n_work, st, a);
        NR_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      break;
    case StageKind::FwdCols: {
      LaunchArgs b = a;
      b.pair_units = a.n_work >= kPairColumnsMin ? 1 : 0;
      const int grid = b.pair_units ? (a.n_work + 15) / 16 * 8 : a.n_work;
      switch (L) {
#define NR_CASE(l) case l: return launch(k_fwd_cols<l>, fft_threads(l), grid, st, b);
        NR_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      break;
    }
    case StageKind::FwdInterp:
      if (L == 0) {   // tiled interpolation (the radial pass is its own stage)
        if (W == 6) return launch(k_interp_tiles<6>, 256, (a.n_work + 1) / 2, st, a, kb);
        if (W == 7) return launch(k_interp_tiles<7>, 256, (a.n_work + 1) / 2, st, a, kb);
        return launch(k_interp_tiles<8>, 256, (a.n_work + 1) / 2, st, a, kb);
      }
      switch (L) {
#define NR_CASE(l)                                                                          \
  case l:                                                                                   \
    if (W == 6) return launch(k_fwd_interp<l, 6>, fft_threads(l), a.n_work, st, a, kb);     \
    if (W == 7) return launch(k_fwd_interp<l, 7>, fft_threads(l), a.n_work, st, a, kb);     \
    return launch(k_fwd_interp<l, 8>, fft_threads(l), a.n_work, st, a, kb);
        NR_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      break;
    case StageKind::FwdRadial:
      switch (L) {
#define NR_CASE(l) case l: return launch(k_fwd_radial<l>, fft_threads(l), a.n_work, st, a);
        NR_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      break;
    case StageKind::AdjRadial:
      switch (L) {
#define NR_CASE(l) case l: return launch(k_adj_radial<l>, fft_threads(l), a.n_work, st, a);
        NR_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      break;
    case StageKind::SpreadZero:
    case StageKind::Spread: {
      const bool zero = stage == StageKind::SpreadZero;
      if (W == 6) return launch_spread<6>(a, kb, tile_w, tile_h, st, zero);
      if (W == 7) return launch_spread<7>(a, kb, tile_w, tile_h, st, zero);
      return launch_spread<8>(a, kb, tile_w, tile_h, st, zero);
    }
    case StageKind::AdjCols:
      switch (L) {
#define NR_CASE(l) case l: return launch(k_adj_cols<l>, fft_threads(l), a.n_work, st, a);
        NR_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      break;
    case StageKind::AdjRows:
      switch (L) {
#define NR_CASE(l) case l: return launch(k_adj_rows<l>, fft_threads(l), a.n_work, st, a);
        NR_LENGTHS(NR_CASE)
#undef NR_CASE
      }
      break;
    default:
      break;
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fill_int(int* p, size_t n, int v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3(unsigned(std::min<size_t>(1024, (n + 255) / 256))), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

int persist_blocks_per_cu(int W) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  if (W == 7) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<7>, kPersistThreads, 0);
  return e == hipSuccess ? n : 0;
}

hipError_t launch_persistent(const LaunchArgs& a, const PersistArgs& p, const KBArgs& kb, int W, int blocks,
                             int* clear, int clear_count, hipStream_t st) {
  if (W != 7 || blocks < kPersistQueues) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_persist_clear, dim3(std::max(1, std::min(64, (clear_count + 255) / 256))), dim3(256), 0, st,
                     clear, clear_count);
  hipLaunchKernelGGL(k_persistent<7>, dim3(blocks), dim3(kPersistThreads), 0, st, PersistLaunch{a, p, kb});
  return hipGetLastError();
}

hipError_t launch_spread_reference(const SliceDesc* d_descs, int slice, const SliceDesc& host_desc, int halo,
                                   int colpad, const KBArgs& kb, int W, hipStream_t st) {
  const size_t n4 = size_t(host_desc.rows) * host_desc.cols / 2;
  hipLaunchKernelGGL(k_fill_zero, dim3(1024), dim3(256), 0, st, reinterpret_cast<float4*>(host_desc.ext), n4);
  const int np = host_desc.na * host_desc.H;
  const dim3 g((np + 255) / 256);
  if (W == 6) hipLaunchKernelGGL(k_spread_atomic<6>, g, dim3(256), 0, st, d_descs, slice, halo, colpad, kb);
  else if (W == 7) hipLaunchKernelGGL(k_spread_atomic<7>, g, dim3(256), 0, st, d_descs, slice, halo, colpad, kb);
  else hipLaunchKernelGGL(k_spread_atomic<8>, g, dim3(256), 0, st, d_descs, slice, halo, colpad, kb);
  return hipGetLastError();
}

}  // namespace nrk
