// Workgroup-cooperative complex FFT in LDS for gfx950 (wave64).
//
// Stockham auto-sort (each pass reads with stride L/R and writes with stride
// Ns, so the result lands in natural order without a bit-reversal pass).  A
// pass loads every butterfly input of the thread into registers, waits at a
// barrier, then writes its outputs back over the same LDS buffer, so one
// L-point buffer is enough.  Radices: 8, 4, 2 for the power-of-two part
// (as many 8s as possible, the remainder as 4s), then 5 and 3; 4096 and 5120
// take three passes of radix 16 (16, 20).  Twiddles
// come from a table of exp(-2 pi i m/L), m < L, computed in float64 on the
// host and rounded once to float32.
#pragma once

#include <hip/hip_runtime.h>

// Buffers in global memory are typed as such in device code, which keeps
// their loads and stores off the flat path (the host pass sees plain pointers).
#ifdef __HIP_DEVICE_COMPILE__
#define NR_G __attribute__((address_space(1)))
#else
#define NR_G
#endif
using TwPtr = const NR_G float2*;

namespace nrk {

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }

// multiply by -i (forward transform) or +i (inverse transform)
template <bool INV>
__device__ __forceinline__ float2 mul_i(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// compile-time radix plan
// ---------------------------------------------------------------------------

constexpr int pow2_exponent(int v) {
  int e = 0;
  while (v > 1 && (v & 1) == 0) {
    v >>= 1;
    ++e;
  }
  return e;
}

constexpr int radix_of(int L, int p) {
  // three passes for the two longest transforms of the 2560^2 and 2048^2
  // workloads: radix 16 and 20 butterflies in registers, one LDS round trip
  // per pass
  if (L == 5120) return p == 0 ? 16 : (p == 1 ? 16 : (p == 2 ? 20 : 1));
  if (L == 4096) return p < 3 ? 16 : 1;
  int r[24] = {};
  int n = 0;
  const int e = pow2_exponent(L);
  const int k = e / 3, rem = e % 3;
  if (rem == 0) {
    for (int i = 0; i < k; ++i) r[n++] = 8;
  } else if (rem == 1) {
    if (k >= 1) {
      for (int i = 0; i < k - 1; ++i) r[n++] = 8;
      r[n++] = 4;
      r[n++] = 4;
    } else {
      r[n++] = 2;
    }
  } else {
    for (int i = 0; i < k; ++i) r[n++] = 8;
    r[n++] = 4;
  }
  int o = L >> e;
  while (o % 5 == 0) {
    r[n++] = 5;
    o /= 5;
  }
  while (o % 3 == 0) {
    r[n++] = 3;
    o /= 3;
  }
  return p < n ? r[p] : 1;
}

constexpr int num_passes(int L) {
  int n = 0;
  while (radix_of(L, n) > 1) ++n;
  return n;
}

constexpr int span_before(int L, int p) {
  int s = 1;
  for (int i = 0; i < p; ++i) s *= radix_of(L, i);
  return s;
}

constexpr bool radix_plan_complete(int L) { return span_before(L, num_passes(L)) == L; }

// ---------------------------------------------------------------------------
// small DFTs, X_k = sum_n x_n exp(-+2 pi i n k / R)
// ---------------------------------------------------------------------------

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float2 a = v[0], b = v[1];
    v[0] = c_add(a, b);
    v[1] = c_sub(a, b);
  }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float2 a0 = c_add(v[0], v[2]), a1 = c_sub(v[0], v[2]);
    const float2 a2 = c_add(v[1], v[3]), a3 = mul_i<INV>(c_sub(v[1], v[3]));
    v[0] = c_add(a0, a2);
    v[2] = c_sub(a0, a2);
    v[1] = c_add(a1, a3);
    v[3] = c_sub(a1, a3);
  }
};

template <bool INV>
struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    const float h = 0.70710678118654752440f;
    // W^1 = (1 -+ i)/sqrt(2), W^2 = -+i, W^3 = W^2 W^1
    const float2 o1 = INV ? make_float2((o[1].x - o[1].y) * h, (o[1].x + o[1].y) * h)
                          : make_float2((o[1].x + o[1].y) * h, (o[1].y - o[1].x) * h);
    const float2 o2 = mul_i<INV>(o[2]);
    const float2 o3t = INV ? make_float2((o[3].x - o[3].y) * h, (o[3].x + o[3].y) * h)
                           : make_float2((o[3].x + o[3].y) * h, (o[3].y - o[3].x) * h);
    const float2 o3 = mul_i<INV>(o3t);
    v[0] = c_add(e[0], o[0]);
    v[4] = c_sub(e[0], o[0]);
    v[1] = c_add(e[1], o1);
    v[5] = c_sub(e[1], o1);
    v[2] = c_add(e[2], o2);
    v[6] = c_sub(e[2], o2);
    v[3] = c_add(e[3], o3);
    v[7] = c_sub(e[3], o3);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float s3 = 0.86602540378443864676f;  // sin(2 pi/3)
    const float2 b = c_add(v[1], v[2]);
    const float2 t = make_float2(v[0].x - 0.5f * b.x, v[0].y - 0.5f * b.y);
    const float2 u = mul_i<INV>(c_scale(c_sub(v[1], v[2]), s3));
    v[0] = c_add(v[0], b);
    v[1] = c_add(t, u);
    v[2] = c_sub(t, u);
  }
};

template <bool INV>
struct Dft<5, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float c1 = 0.30901699437494742410f;   // cos(2 pi/5)
    const float c2 = -0.80901699437494742410f;  // cos(4 pi/5)
    const float s1 = 0.95105651629515357212f;   // sin(2 pi/5)
    const float s2 = 0.58778525229247312917f;   // sin(4 pi/5)
    const float2 b1 = c_add(v[1], v[4]), b2 = c_add(v[2], v[3]);
    const float2 d1 = c_sub(v[1], v[4]), d2 = c_sub(v[2], v[3]);
    const float2 t1 = make_float2(v[0].x + c1 * b1.x + c2 * b2.x, v[0].y + c1 * b1.y + c2 * b2.y);
    const float2 t2 = make_float2(v[0].x + c2 * b1.x + c1 * b2.x, v[0].y + c2 * b1.y + c1 * b2.y);
    const float2 u1 = mul_i<INV>(make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
    const float2 u2 = mul_i<INV>(make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
    v[0] = c_add(v[0], c_add(b1, b2));
    v[1] = c_add(t1, u1);
    v[4] = c_sub(t1, u1);
    v[2] = c_add(t2, u2);
    v[3] = c_sub(t2, u2);
  }
};

// cos and sin of 2 pi m / N for the composite butterflies below
template <int N>
struct UnitRoots;
template <>
struct UnitRoots<16> {
  static constexpr float c[16] = {1.f, 0.92387953251128674f, 0.70710678118654757f, 0.38268343236508984f,
                                  0.f, -0.38268343236508984f, -0.70710678118654757f, -0.92387953251128674f,
                                  -1.f, -0.92387953251128674f, -0.70710678118654757f, -0.38268343236508984f,
                                  0.f, 0.38268343236508984f, 0.70710678118654757f, 0.92387953251128674f};
  static constexpr float s[16] = {0.f, 0.38268343236508984f, 0.70710678118654757f, 0.92387953251128674f,
                                  1.f, 0.92387953251128674f, 0.70710678118654757f, 0.38268343236508984f,
                                  0.f, -0.38268343236508984f, -0.70710678118654757f, -0.92387953251128674f,
                                  -1.f, -0.92387953251128674f, -0.70710678118654757f, -0.38268343236508984f};
};
template <>
struct UnitRoots<20> {
  static constexpr float c[20] = {1.f, 0.95105651629515357f, 0.80901699437494742f, 0.58778525229247313f,
                                  0.30901699437494742f, 0.f, -0.30901699437494742f, -0.58778525229247313f,
                                  -0.80901699437494742f, -0.95105651629515357f, -1.f, -0.95105651629515357f,
                                  -0.80901699437494742f, -0.58778525229247313f, -0.30901699437494742f, 0.f,
                                  0.30901699437494742f, 0.58778525229247313f, 0.80901699437494742f,
                                  0.95105651629515357f};
  static constexpr float s[20] = {0.f, 0.30901699437494742f, 0.58778525229247313f, 0.80901699437494742f,
                                  0.95105651629515357f, 1.f, 0.95105651629515357f, 0.80901699437494742f,
                                  0.58778525229247313f, 0.30901699437494742f, 0.f, -0.30901699437494742f,
                                  -0.58778525229247313f, -0.80901699437494742f, -0.95105651629515357f, -1.f,
                                  -0.95105651629515357f, -0.80901699437494742f, -0.58778525229247313f,
                                  -0.30901699437494742f};
};

// a * exp(-+2 pi i m/N) for an index m that is a constant once the calling
// loops are unrolled (the quarter turns are sign swaps)
template <int N, bool INV>
__device__ __forceinline__ float2 mul_root(float2 a, int m) {
  m %= N;
  if (m == 0) return a;
  if (4 * m == N) return mul_i<INV>(a);
  if (2 * m == N) return make_float2(-a.x, -a.y);
  if (4 * m == 3 * N) return mul_i<!INV>(a);
  const float c = UnitRoots<N>::c[m], sn = INV ? UnitRoots<N>::s[m] : -UnitRoots<N>::s[m];
  return make_float2(a.x * c - a.y * sn, a.x * sn + a.y * c);
}

// N = P*Q point DFT from P- and Q-point ones: input n = Q*n1 + n2, output
// k = k1 + P*k2; DFT_P over n1 for each n2, twiddles W_N^(n2*k1), DFT_Q over
// n2 for each k1.
template <int P, int Q, bool INV>
struct DftPQ {
  __device__ __forceinline__ static void run(float2* v) {
    float2 y[Q][P];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) {
      float2 t[P];
#pragma unroll
      for (int n1 = 0; n1 < P; ++n1) t[n1] = v[Q * n1 + n2];
      Dft<P, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < P; ++k1) y[n2][k1] = mul_root<P * Q, INV>(t[k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
      float2 t[Q];
#pragma unroll
      for (int n2 = 0; n2 < Q; ++n2) t[n2] = y[n2][k1];
      Dft<Q, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) v[k1 + P * k2] = t[k2];
    }
  }
};

template <bool INV>
struct Dft<16, INV> : DftPQ<4, 4, INV> {};
template <bool INV>
struct Dft<20, INV> : DftPQ<5, 4, INV> {};

// ---------------------------------------------------------------------------
// LDS buffer of one transform.  Element i lives at i ^ ((i >> 4) & 15): an
// XOR swizzle within blocks of 16 elements (128 bytes), so that the stride-R
// writes of the early passes (R = 8, 16: lanes 64 or 128 bytes apart, all on
// the same banks unswizzled) and the contiguous reads of the others both
// spread over the banks.  Counters put bank conflicts at 56 % of the LDS
// cycles of the 5120-point column transform unswizzled; swizzled, the
// transforms run 0-2 % faster (LDS is not their limit).  A bijection within
// each block, so L (a multiple of 16) elements still fill L slots.
// ---------------------------------------------------------------------------

template <int L>
constexpr int lds_elems() {
  return L;
}

struct Lds {
  float2* p;
  __device__ __forceinline__ float2& operator[](int i) const { return p[i ^ ((i >> 4) & 15)]; }
};

// ---------------------------------------------------------------------------
// one Stockham pass and the whole transform
// ---------------------------------------------------------------------------

// Twiddles of a radix-R pass: w^r for r = 1..R-1 with w = e^{-2 pi i k/(Ns R)}.
// For R >= 8 only w and w^B are read from the table (B = ceil(sqrt(R))):
// w^b (b < B) and w^{aB} follow by repeated products, and w^{aB+b} =
// w^{aB} w^b, so a twiddle carries at most (B - 2) + (A - 2) + 1 extra
// roundings, A = ceil(R / B) (5 at R = 16, 6 at R = 20; parity at 2560^2
// does not change).  The table loads were most of a transform's
// vector-memory instructions: all R - 1 per butterfly ran the 5120-point
// column transforms at 53 us per slice, 2 run them at 45.5.
constexpr int tw_split(int R) {
  int b = 1;
  while (b * b < R) ++b;
  return b;
}

// w[r - 1] = tw[r st], r = 1..R-1 (w = tw[st] is e^{-2 pi i st/L}), as above
template <int R>
__device__ __forceinline__ void radix_twiddles(TwPtr __restrict__ tw, int st, float2 (&w)[R - 1]) {
  if constexpr (R >= 8) {
    constexpr int B = tw_split(R);
    constexpr int A = (R - 1) / B + 1;
    float2 lo[B], hi[A];
    lo[1] = tw[st];
    hi[1] = tw[B * st];
#pragma unroll
    for (int b = 2; b < B; ++b) lo[b] = c_mul(lo[b - 1], lo[1]);
#pragma unroll
    for (int a = 2; a < A; ++a) hi[a] = c_mul(hi[a - 1], hi[1]);
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const int a = r / B, b = r % B;
      w[r - 1] = a == 0 ? lo[b] : (b == 0 ? hi[a] : c_mul(hi[a], lo[b]));
    }
  } else {
#pragma unroll
    for (int r = 1; r < R; ++r) w[r - 1] = tw[r * st];
  }
}

template <int L, int T, int P, bool INV>
__device__ __forceinline__ void fft_pass(Lds s, TwPtr __restrict__ tw, int tid) {
  constexpr int R = radix_of(L, P);
  constexpr int Ns = span_before(L, P);
  constexpr int NB = L / R;
  constexpr int PER = (NB + T - 1) / T;
  float2 v[PER][R];
  float2 w[PER][R - 1];
  // twiddles first (clamped index, no branch): their global loads overlap the
  // LDS reads and the barrier
  if constexpr (Ns > 1) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int j = (NB % T == 0 || tid + i * T < NB) ? tid + i * T : 0;
      const int k = j % Ns;
      radix_twiddles<R>(tw, k * (L / (Ns * R)), w[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = tid + i * T;
    if (NB % T == 0 || j < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = s[j + r * NB];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = tid + i * T;
    if (NB % T == 0 || j < NB) {
      const int k = j % Ns;
      if constexpr (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = c_mul(v[i][r], INV ? c_conj(w[i][r - 1]) : w[i][r - 1]);
      }
      Dft<R, INV>::run(v[i]);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) s[base + r * Ns] = v[i][r];
    }
  }
  __syncthreads();
}

template <int L, int T, bool INV, int P = 0, int END = num_passes(L)>
__device__ __forceinline__ void fft_passes(Lds s, TwPtr __restrict__ tw, int tid) {
  if constexpr (P < END) {
    fft_pass<L, T, P, INV>(s, tw, tid);
    fft_passes<L, T, INV, P + 1, END>(s, tw, tid);
  }
}

// In-place length-L transform of the LDS buffer s by T threads.  Forward:
// X_k = sum_n x_n exp(-2 pi i nk/L); inverse: the + sign, unnormalised.
// The caller must have synchronised after filling s; on return s holds the
// result and the workgroup has synchronised.
template <int L, int T, bool INV>
__device__ __forceinline__ void fft_lds(Lds s, TwPtr __restrict__ tw, int tid) {
  static_assert(radix_plan_complete(L), "FFT length must be 2^a * 3^b * 5^c");
  fft_passes<L, T, INV>(s, tw, tid);
}

// First pass of a transform whose inputs come from load(n) (natural index
// n) straight into registers; the pass writes the LDS buffer and the
// workgroup synchronises.  With HALF, the input is a length-L/2 signal
// zero-padded to L and centred (non-zero only at natural indices [0, L/4)
// and [3L/4, L)): the zeros of each first-pass butterfly sit at fixed
// positions and are not loaded.
template <int L, int T, bool INV, bool HALF, class Load>
__device__ __forceinline__ void fft_first_pass_from(Lds s, int tid, Load&& load) {
  constexpr int R = radix_of(L, 0);
  static_assert(!HALF || (R % 4 == 0 && L % 4 == 0), "the first radix must split the zero padding evenly");
  constexpr int NB = L / R;
  constexpr int PER = (NB + T - 1) / T;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = tid + i * T;
    if (NB % T == 0 || j < NB) {
      // input r of butterfly j is index j + r NB: with HALF, below L/4 for
      // r < R/4, at or above 3L/4 for r >= 3R/4, padding in between
      float2 v[R];
#pragma unroll
      for (int r = 0; r < R; ++r)
        v[r] = (!HALF || r < R / 4 || r >= 3 * R / 4) ? load(j + r * NB) : make_float2(0.f, 0.f);
      Dft<R, INV>::run(v);
#pragma unroll
      for (int r = 0; r < R; ++r) s[j * R + r] = v[r];
    }
  }
  __syncthreads();
}

// Transform of a length-L/2 signal zero-padded to L and centred, its input
// from load(n): the first pass as fft_first_pass_from with HALF, the rest as
// in fft_lds.  No LDS fill precedes it; on return s holds the result and the
// workgroup has synchronised.
template <int L, int T, bool INV, class Load>
__device__ __forceinline__ void fft_lds_halfzero(Lds s, TwPtr __restrict__ tw, int tid, Load&& load) {
  static_assert(radix_plan_complete(L), "FFT length must be 2^a * 3^b * 5^c");
  fft_first_pass_from<L, T, INV, true>(s, tid, load);
  fft_passes<L, T, INV, 1>(s, tw, tid);
}

// Transform whose last pass hands its outputs straight from registers to
// store(n, value) (natural index n) instead of writing the LDS buffer; with
// HALF only the outputs at [0, L/4) and [3L/4, L) (the centred half of the
// result) are handed over.  Passes START to the last but one run as in
// fft_lds (START = 1 after fft_first_pass_from).  Expects s to hold the
// input of pass START and the workgroup synchronised; leaves s holding the
// input of the last pass, and the caller must synchronise before writing s
// again.
template <int L, int T, bool INV, int START = 0, bool HALF = true, class Store>
__device__ __forceinline__ void fft_lds_store_out(Lds s, TwPtr __restrict__ tw, int tid, Store&& store) {
  static_assert(radix_plan_complete(L), "FFT length must be 2^a * 3^b * 5^c");
  constexpr int P = num_passes(L) - 1;
  constexpr int R = radix_of(L, P);
  constexpr int Ns = span_before(L, P);
  static_assert(Ns * R == L && P >= 1 && START <= P, "a transform of at least two passes");
  fft_passes<L, T, INV, START, P>(s, tw, tid);
  constexpr int PER = (Ns + T - 1) / T;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    // butterfly j of the last pass reads j + r Ns and yields outputs j + r Ns
    const int j = tid + i * T;
    if (Ns % T == 0 || j < Ns) {
      float2 v[R], w[R - 1];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = s[j + r * Ns];
      radix_twiddles<R>(tw, j, w);
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = c_mul(v[r], INV ? c_conj(w[r - 1]) : w[r - 1]);
      Dft<R, INV>::run(v);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int n = j + r * Ns;
        if (!HALF || n < L / 4 || n >= L - L / 4) store(n, v[r]);
      }
    }
  }
}

// threads per transform for a length-L FFT.  For 5·2^a lengths five
// wavefronts split the radix-8 and radix-4 passes evenly (2560: 320 radix-8
// butterflies per pass; 5120: 640 and 1280), where four would leave the last
// round of each pass partly idle.
constexpr int fft_threads(int L) {
  return (L == 2560 || L == 5120) ? 320 : (L >= 2048 ? 256 : (L >= 512 ? 128 : 64));
}

}  // namespace nrk
