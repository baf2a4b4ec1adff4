// Host-side plan construction (pure C++; see plan.hpp).
//
// Compiled with floating-point contraction off: the spreading bins below and
// the device kernels must compute identical grid coordinates from the same
// float64 tables (one rounded multiply, one rounded subtract, ceil).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>

namespace nr {

static const int kFftLengths[] = {16,  32,  64,  128,  256,  512,  1024, 2048, 4096, 8192,
                                  80,  160, 320, 640,  1280, 2560, 5120};

bool fft_length_supported(int L) {
  for (int v : kFftLengths)
    if (v == L) return true;
  return false;
}

bool spread_tile_supported(int w, int h) {
  return (w == 64 && h == 32) || (w == 32 && h == 32) || (w == 64 && h == 64) || (w == 128 && h == 32);
}

// ---------------------------------------------------------------------------
// Kaiser-Bessel kernel
// ---------------------------------------------------------------------------

// Modified Bessel function of the first kind, order 0: the power series
// sum_k ((x/2)^2)^k / (k!)^2, summed until the terms stop contributing.
double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= q / (double(k) * double(k));
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return sum;
}

double KaiserBessel::phi(double u) const {
  const double r = 2.0 * u / W;
  if (std::fabs(r) > 1.0) return 0.0;
  return bessel_i0(beta * std::sqrt(1.0 - r * r)) / i0beta;
}

// Continuous Fourier transform of phi: for the window I0(beta sqrt(1-(x/a)^2))
// on |x| <= a it is 2a sinh(sqrt(beta^2 - (2 pi a xi)^2)) / sqrt(beta^2 - (2 pi a xi)^2)
// (sin/sqrt past the cut-off), here with a = W/2 and the 1/I0(beta) normalisation.
double KaiserBessel::phihat(double xi) const {
  const double t = M_PI * W * xi;
  const double d = beta * beta - t * t;
  double v;
  if (d > 1e-12) {
    const double r = std::sqrt(d);
    v = W * std::sinh(r) / r;
  } else if (d < -1e-12) {
    const double r = std::sqrt(-d);
    v = W * std::sin(r) / r;
  } else {
    v = W;
  }
  return v / i0beta;
}

// Chebyshev interpolation of each tap weight w_i(z) = phi(z + (W-1)/2 - i) on
// z in [-1/2, 1/2] at D+1 Chebyshev points, converted to monomials in z.
static std::vector<double> fit_tap(const KaiserBessel& kb, int i, int D) {
  const int n = D + 1;
  std::vector<double> fk(n), c(n, 0.0);
  for (int k = 0; k < n; ++k) {
    const double t = std::cos(M_PI * (k + 0.5) / n);   // t in [-1,1], z = t/2
    fk[k] = kb.phi(0.5 * t + 0.5 * (kb.W - 1) - i);
  }
  for (int m = 0; m < n; ++m) {
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += fk[k] * std::cos(M_PI * m * (k + 0.5) / n);
    c[m] = (m == 0 ? 1.0 : 2.0) * s / n;
  }
  // Chebyshev series in t -> monomials in t (T_{m+1} = 2 t T_m - T_{m-1}).
  std::vector<double> Tm1(n, 0.0), Tm(n, 0.0), mono(n, 0.0);
  Tm1[0] = 1.0;                 // T_0
  if (n > 1) Tm[1] = 1.0;       // T_1
  for (int k = 0; k < n; ++k) mono[k] += c[0] * Tm1[k];
  if (n > 1)
    for (int k = 0; k < n; ++k) mono[k] += c[1] * Tm[k];
  for (int m = 2; m < n; ++m) {
    std::vector<double> Tn(n, 0.0);
    for (int k = 0; k < n; ++k) {
      if (k > 0) Tn[k] += 2.0 * Tm[k - 1];
      Tn[k] -= Tm1[k];
    }
    for (int k = 0; k < n; ++k) mono[k] += c[m] * Tn[k];
    Tm1 = Tm;
    Tm = Tn;
  }
  // t = 2 z: coefficient of z^k is mono[k] * 2^k
  for (int k = 0; k < n; ++k) mono[k] *= std::ldexp(1.0, k);
  return mono;
}

void KaiserBessel::init(int width, double beta_in) {
  W = width;
  const double sigma = 2.0;
  beta = beta_in > 0 ? beta_in
                     : M_PI * std::sqrt((W / sigma) * (W / sigma) * (sigma - 0.5) * (sigma - 0.5) - 0.8);
  i0beta = bessel_i0(beta);
  // degree W + 2: the fit error then sits at the float32 rounding of the
  // coefficients (a few 1e-8 of phi(0)) for the default shapes
  D = W + 2;
  coef.assign(size_t(W) * (D + 1), 0.0f);
  // phi is even: tap W-1-i at z equals tap i at -z.  The upper taps take the
  // lower taps' coefficients with the odd powers negated, exactly as the
  // kernels evaluate them (in mirrored pairs).
  for (int i = 0; i < (W + 1) / 2; ++i) {
    std::vector<double> m = fit_tap(*this, i, D);
    for (int k = 0; k <= D; ++k) {
      coef[size_t(i) * (D + 1) + k] = float(m[k]);
      coef[size_t(W - 1 - i) * (D + 1) + k] = (k % 2 ? -1.0f : 1.0f) * float(m[k]);
    }
  }
}

double KaiserBessel::phi_poly(double u) const {
  // locate the tap of u in the convention of plan.hpp for a point at 0: taps
  // sit at offsets d = z + (W-1)/2 - i with z in (-1/2, 1/2]
  const double h = 0.5 * (W - 1);
  for (int i = 0; i < W; ++i) {
    const double z = u - h + i;
    if (z > -0.5 && z <= 0.5) {
      double acc = coef[size_t(i) * (D + 1) + D];
      for (int k = D - 1; k >= 0; --k) acc = acc * z + coef[size_t(i) * (D + 1) + k];
      return acc;
    }
  }
  return 0.0;
}

double KaiserBessel::max_poly_error() const {
  double e = 0.0;
  for (int s = 0; s <= 4000; ++s) {
    const double u = -0.5 * W + 1e-9 + (W - 2e-9) * s / 4000.0;
    e = std::max(e, std::fabs(phi_poly(u) - phi(u)));
  }
  return e;
}

// ---------------------------------------------------------------------------
// spreading bins
// ---------------------------------------------------------------------------

int disc_radius(const Plan& plan, const Geom& g) {
  // the polar points reach |u| = (N_t/2)(G/N_t) = G/2 cells; their taps
  // W/2 cells further (one cell of margin on top)
  return g.G / 2 + (plan.kb.W + 1) / 2 + 2;
}

void build_spread_bins(const Plan& plan, Geom& g) {
  const int W = plan.kb.W;
  const int na = g.key.n_angles;
  // tile shape from the tuning (compiled shapes only); edge tiles are partial
  g.tile_w = plan.tune.tile_w;
  g.tile_h = plan.tune.tile_h;
  g.tiles_x = (g.cols + g.tile_w - 1) / g.tile_w;
  g.tiles_y = (g.rows + g.tile_h - 1) / g.tile_h;
  const int ntiles = g.tiles_x * g.tiles_y;
  const double halfW = 0.5 * W;
  // one-cell margin: a point is listed by every tile within one cell of its
  // footprint, so a last-bit difference in the device's coordinate cannot drop a tap
  const int margin = 1;
  std::vector<int32_t> count(ntiles + 1, 0);
  auto for_tiles = [&](int a, int j, auto&& fn) {
    const double ux = double(j) * g.gxy[2 * a];
    const double uy = double(j) * g.gxy[2 * a + 1];
    const int g0x = int(std::ceil(ux - halfW));
    const int g0y = int(std::ceil(uy - halfW));
    const int r0 = std::max(0, g0x + plan.halo - margin);
    const int r1 = std::min(g.rows - 1, g0x + plan.halo + W - 1 + margin);
    const int c0 = std::max(0, g0y + g.G / 2 + plan.colpad - margin);
    const int c1 = std::min(g.cols - 1, g0y + g.G / 2 + plan.colpad + W - 1 + margin);
    for (int ty = r0 / g.tile_h; ty <= r1 / g.tile_h; ++ty)
      for (int tx = c0 / g.tile_w; tx <= c1 / g.tile_w; ++tx) fn(ty * g.tiles_x + tx);
  };
  for (int a = 0; a < na; ++a)
    for (int j = 1; j < g.H; ++j) for_tiles(a, j, [&](int t) { count[t + 1]++; });
  for (int t = 0; t < ntiles; ++t) count[t + 1] += count[t];
  g.tile_start = count;
  g.pts.assign(size_t(count[ntiles]), 0);
  std::vector<int32_t> fill(count.begin(), count.end() - 1);
  for (int a = 0; a < na; ++a)
    for (int j = 1; j < g.H; ++j)
      for_tiles(a, j, [&](int t) { g.pts[size_t(fill[t]++)] = (a << g.jbits) | j; });
  // work items: at most `chunk` points each; tiles cut into several items
  // accumulate with atomics into a grid region cleared beforehand
  const int chunk = plan.tune.chunk;
  // the k = 0 point of every angle sits at the origin: it is summed over the
  // angles once and spread by the first item of each tile its footprint touches
  const int d0 = int(std::ceil(-halfW));
  const int dr0 = d0 + plan.halo, dr1 = d0 + plan.halo + W - 1;
  const int dc0 = d0 + g.G / 2 + plan.colpad, dc1 = dc0 + W - 1;
  g.items.clear();
  g.zero_tiles.clear();
  // The adjoint column transform reads only cells whose natural frequency
  // (mirror rows folded back, periodic columns wrapped) lies within rdisc of
  // the origin.  A tile without points and without such a cell is neither
  // written nor read, so it gets no work item.
  const int64_t rd2 = int64_t(disc_radius(plan, g)) * disc_radius(plan, g);
  auto unread = [&](int ty, int tx) {
    for (int r = ty * g.tile_h; r < std::min(g.rows, (ty + 1) * g.tile_h); ++r) {
      int qx = r - plan.halo;
      qx = qx < 0 ? -qx : (qx > g.G / 2 ? g.G - qx : qx);
      for (int c = tx * g.tile_w; c < std::min(g.cols, (tx + 1) * g.tile_w); ++c) {
        const int qy = ((c - plan.colpad) % g.G + g.G) % g.G - g.G / 2;
        if (int64_t(qx) * qx + int64_t(qy) * qy <= rd2) return false;
      }
    }
    return true;
  };
  std::vector<int32_t> cell_count(size_t(g.tile_w) * g.tile_h);
  for (int t = 0; t < ntiles; ++t) {
    const int b = g.tile_start[t], e = g.tile_start[t + 1];
    const int ty = t / g.tiles_x, tx = t % g.tiles_x;
    if (e == b && unread(ty, tx)) continue;
    const int n_items = std::max(1, (e - b + chunk - 1) / chunk);
    const bool has_dc = ty * g.tile_h <= dr1 && (ty + 1) * g.tile_h > dr0 &&
                        tx * g.tile_w <= dc1 && (tx + 1) * g.tile_w > dc0;
    if (n_items > 1) g.zero_tiles.push_back(t);
    for (int k = 0; k < n_items; ++k) {
      const int ib = b + int((int64_t(e - b) * k) / n_items);
      const int ie = b + int((int64_t(e - b) * (k + 1)) / n_items);
      // largest number of this item's points that touch one cell: bounds the
      // magnitude of every cell's sum for the kernel's fixed-point scale
      std::fill(cell_count.begin(), cell_count.end(), 0);
      int cmax = 0;
      for (int q = ib; q < ie; ++q) {
        const int a = g.pts[size_t(q)] >> g.jbits, j = g.pts[size_t(q)] & ((1 << g.jbits) - 1);
        const int g0x = int(std::ceil(double(j) * g.gxy[2 * a] - halfW));
        const int g0y = int(std::ceil(double(j) * g.gxy[2 * a + 1] - halfW));
        const int rr0 = g0x + plan.halo - ty * g.tile_h, cc0 = g0y + g.G / 2 + plan.colpad - tx * g.tile_w;
        for (int i = std::max(0, rr0); i < std::min(g.tile_h, rr0 + W); ++i)
          for (int l = std::max(0, cc0); l < std::min(g.tile_w, cc0 + W); ++l)
            cmax = std::max(cmax, ++cell_count[size_t(i) * g.tile_w + l]);
      }
      // (the origin's k = 0 sum is added in float32 at write-out, outside the
      // fixed-point sums)
      const int flags = (n_items > 1 ? kItemAtomic : 0) | (has_dc && k == 0 ? kItemDC : 0);
      g.items.push_back({t, ib, ie, flags, cmax + 1});
    }
  }
  // heaviest items first so the long ones start early
  std::stable_sort(g.items.begin(), g.items.end(), [](const SpreadItem& x, const SpreadItem& y) {
    return (x.end - x.begin) > (y.end - y.begin);
  });
}

void build_interp_bins(const Plan& plan, Geom& g) {
  const int W = plan.kb.W;
  const int na = g.key.n_angles;
  const int TW = kInterpTileW, TH = kInterpTileH;
  g.itiles_x = (g.cols + TW - 1) / TW;
  g.itiles_y = (g.rows + TH - 1) / TH;
  const int ntiles = g.itiles_x * g.itiles_y;
  const double halfW = 0.5 * W;
  // the tile of the first tap (g0x, g0y) in grid row/column coordinates; the
  // same double arithmetic as the kernels, which stage a one-cell margin anyway
  auto tile_of = [&](int a, int j) {
    const int g0x = int(std::ceil(double(j) * g.gxy[2 * a] - halfW));
    const int g0y = int(std::ceil(double(j) * g.gxy[2 * a + 1] - halfW));
    const int r = g0x + plan.halo, c = g0y + g.G / 2 + plan.colpad;
    return (r / TH) * g.itiles_x + c / TW;
  };
  std::vector<int32_t> start(size_t(ntiles) + 1, 0);
  for (int a = 0; a < na; ++a)
    for (int j = 0; j < g.H; ++j) start[size_t(tile_of(a, j)) + 1]++;
  for (int t = 0; t < ntiles; ++t) start[size_t(t) + 1] += start[size_t(t)];
  g.ipts.assign(size_t(start[size_t(ntiles)]), 0);
  std::vector<int32_t> fill(start.begin(), start.end() - 1);
  // angle-major within a tile: neighbouring threads take neighbouring points of one line
  for (int a = 0; a < na; ++a)
    for (int j = 0; j < g.H; ++j) g.ipts[size_t(fill[size_t(tile_of(a, j))]++)] = (a << g.jbits) | j;
  const int chunk = plan.tune.chunk;
  g.iitems.clear();
  for (int t = 0; t < ntiles; ++t) {
    const int b = start[size_t(t)], e = start[size_t(t) + 1];
    if (e == b) continue;
    const int n_items = (e - b + chunk - 1) / chunk;
    for (int k = 0; k < n_items; ++k) {
      const int ib = b + int((int64_t(e - b) * k) / n_items);
      const int ie = b + int((int64_t(e - b) * (k + 1)) / n_items);
      g.iitems.push_back({t, ib, ie, 0, 0});
    }
  }
  std::stable_sort(g.iitems.begin(), g.iitems.end(), [](const SpreadItem& x, const SpreadItem& y) {
    return (x.end - x.begin) > (y.end - y.begin);
  });
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

nr_status build_plan(const nr_slice* slices, int32_t n_slices, const double* angles,
                     const nr_nufft* params, Plan& plan, std::string& err) {
  if (!slices || n_slices <= 0 || !angles) {
    err = "slices/angles must be non-null and n_slices > 0";
    return NR_INVALID_ARG;
  }
  double sigma = params ? params->sigma : 2.0;
  int width = params ? params->width : 7;
  double beta = params ? params->beta : 0.0;
  if (sigma == 0.0) sigma = 2.0;
  if (width == 0) width = 7;
  if (sigma != 2.0) {
    err = "only oversampling sigma = 2 is built";
    return NR_UNSUPPORTED_SIZE;
  }
  if (width < 6 || width > 8) {
    err = "kernel width must be 6, 7 or 8";
    return NR_UNSUPPORTED_SIZE;
  }
  if (!(beta <= 0.0 || (beta > 1.0 && beta < 100.0))) {
    err = "beta must be <= 0 (default shape) or in (1, 100)";
    return NR_INVALID_ARG;
  }
  plan.sigma = sigma;
  plan.kb.init(width, beta);
  if (plan.kb.max_poly_error() > 1e-6) {
    err = "kernel shape beta gives a polynomial fit error above 1e-6";
    return NR_UNSUPPORTED_SIZE;
  }
  // taps of a point reach ceil(W/2) cells beyond the half-plane's edges
  plan.halo = (width + 1) / 2;
  plan.colpad = 4;                 // covers W <= 8 on both ends; keeps rows 64-byte aligned
  plan.slices.assign(slices, slices + n_slices);

  int64_t max_angle = 0;
  for (int s = 0; s < n_slices; ++s) {
    const nr_slice& sl = slices[s];
    if (sl.n < 8 || (sl.n & 1) || sl.n_det < 8 || (sl.n_det & 1) || sl.n_angles < 1) {
      err = "slice " + std::to_string(s) + ": need even n >= 8, even n_det >= 8, n_angles >= 1";
      return NR_INVALID_ARG;
    }
    if (sl.vol_off < 0 || sl.sino_off < 0 || sl.angle_off < 0) {
      err = "slice " + std::to_string(s) + ": negative offset";
      return NR_INVALID_ARG;
    }
    if (!std::isfinite(sl.center) || std::fabs(sl.center) > 0.5 * sl.n_det) {
      err = "slice " + std::to_string(s) + ": center must be finite with |center| <= n_det/2";
      return NR_INVALID_ARG;
    }
    // the kernels' point codes (angle << bits of n_det/2) | radial index are
    // 31-bit, and angle * (n_det/2 + 1) is formed with 24-bit multiplies
    int jb = 0;
    while ((1 << jb) < sl.n_det / 2 + 1) ++jb;
    if (int64_t(sl.n_angles) >= (int64_t(1) << std::min(24, 31 - jb))) {
      err = "slice " + std::to_string(s) + ": n_angles must be below 2^24 and below 2^31 / 2^ceil(log2(n_det/2 + 1))";
      return NR_UNSUPPORTED_SIZE;
    }
    const int G = int(sigma * sl.n);
    if (!fft_length_supported(G) || !fft_length_supported(sl.n_det)) {
      err = "slice " + std::to_string(s) + ": FFT length " + std::to_string(G) + " or " +
            std::to_string(sl.n_det) + " is not built (2^a 16..8192 or 5*2^a 80..5120)";
      return NR_UNSUPPORTED_SIZE;
    }
    max_angle = std::max(max_angle, sl.angle_off + sl.n_angles);
  }
  plan.angles.assign(angles, angles + max_angle);
  for (int64_t i = 0; i < max_angle; ++i)
    if (!std::isfinite(plan.angles[size_t(i)])) {
      err = "angle " + std::to_string(i) + " is not finite";
      return NR_INVALID_ARG;
    }

  std::map<GeomKey, int> geom_index;
  plan.slice_geom.resize(n_slices);
  for (int s = 0; s < n_slices; ++s) {
    const nr_slice& sl = slices[s];
    GeomKey key{sl.n, sl.n_det, sl.n_angles, sl.angle_off};
    auto it = geom_index.find(key);
    if (it != geom_index.end()) {
      plan.slice_geom[s] = it->second;
      continue;
    }
    Geom g;
    g.key = key;
    g.G = int(sigma * sl.n);
    g.H = sl.n_det / 2 + 1;
    while ((1 << g.jbits) < g.H) ++g.jbits;
    g.rows = g.G / 2 + 1 + 2 * plan.halo;
    g.cols = g.G + 2 * plan.colpad;
    g.gxy.resize(size_t(2) * sl.n_angles);
    g.flip.resize(sl.n_angles);
    for (int a = 0; a < sl.n_angles; ++a) {
      const double th = plan.angles[size_t(sl.angle_off + a)];
      double cx = std::cos(th), cy = std::sin(th);
      // conjugate symmetry of the spectrum of a real slice: points with a
      // negative first coordinate are read at -u and conjugated
      const int fl = cx < 0.0 ? 1 : 0;
      if (fl) {
        cx = -cx;
        cy = -cy;
      }
      g.gxy[2 * a] = double(g.G) * cx / double(sl.n_det);
      g.gxy[2 * a + 1] = double(g.G) * cy / double(sl.n_det);
      g.flip[a] = fl;
    }
    plan.slice_geom[s] = int(plan.geoms.size());
    geom_index[key] = int(plan.geoms.size());
    plan.geoms.push_back(std::move(g));
  }

  // tables: deapodisation per N, twiddles per FFT length
  for (const Geom& g : plan.geoms) {
    const int n = g.key.n;
    if (!plan.deapod.count(n)) {
      std::vector<float> d(n);
      for (int i = 0; i < n; ++i) d[i] = float(1.0 / plan.kb.phihat(double(i - n / 2) / g.G));
      plan.deapod[n] = d;
    }
    for (int L : {g.G, g.key.n_det}) {
      if (plan.twiddle.count(L)) continue;
      std::vector<f2> tw(L);
      for (int m = 0; m < L; ++m) {
        const double ph = -2.0 * M_PI * double(m) / double(L);
        tw[m] = {float(std::cos(ph)), float(std::sin(ph))};
      }
      plan.twiddle[L] = tw;
    }
  }
  // rotation-axis phases exp(-2 pi i k_j c) on the half-line k_j = j/N_t,
  // one table per distinct (N_t, c) with c != 0
  for (const nr_slice& sl : plan.slices) {
    const std::pair<int, double> key{sl.n_det, sl.center};
    if (sl.center == 0.0 || plan.shift.count(key)) continue;
    const int H = sl.n_det / 2 + 1;
    std::vector<f2> ph(H);
    for (int j = 0; j < H; ++j) {
      // reduce j*c/N_t modulo 1 in float64 before the trigonometry
      double turns = std::fmod(double(j) * sl.center, double(sl.n_det)) / double(sl.n_det);
      ph[j] = {float(std::cos(2.0 * M_PI * turns)), float(-std::sin(2.0 * M_PI * turns))};
    }
    plan.shift[key] = ph;
  }

  return NR_OK;
}

// ---------------------------------------------------------------------------
// batches, work lists and the workspace layout
// ---------------------------------------------------------------------------

namespace {

// Append `n` logical units of (slice, unit) pairs for one launch.  With
// `xcd`, position p = 8k + x holds logical unit x*ceil(n/8) + k (padding
// beyond n), so that a grid-stride loop over a grid that is a multiple of 8
// gives each XCD (block b runs on XCD b % 8) a contiguous run of units.
void append_units(std::vector<WorkItem>& out, const std::vector<WorkItem>& logical, bool xcd) {
  if (!xcd) {
    out.insert(out.end(), logical.begin(), logical.end());
    return;
  }
  const size_t n = logical.size();
  const size_t per = (n + 7) / 8;
  for (size_t p = 0; p < 8 * per; ++p) {
    const size_t x = p % 8, k = p / 8;
    const size_t l = x * per + k;
    out.push_back(l < n ? logical[l] : WorkItem{-1, 0});
  }
}

}  // namespace

nr_status layout_plan(Plan& plan, std::string& err) {
  if (plan.laid_out) return NR_OK;
  const Tuning& tu = plan.tune;
  if (!spread_tile_supported(tu.tile_w, tu.tile_h)) {
    err = "spreading tile " + std::to_string(tu.tile_w) + "x" + std::to_string(tu.tile_h) +
          " is not built (64x32, 32x32, 64x64, 128x32)";
    return NR_UNSUPPORTED_SIZE;
  }
  if (tu.chunk < 64 || tu.chunk > kMaxChunk) {
    err = "chunk must be in [64, " + std::to_string(kMaxChunk) + "]";
    return NR_INVALID_ARG;
  }
  for (Geom& g : plan.geoms) {
    if (g.bins_tile_w != tu.tile_w || g.bins_tile_h != tu.tile_h || g.bins_chunk != tu.chunk) {
      build_spread_bins(plan, g);
      g.bins_tile_w = tu.tile_w;
      g.bins_tile_h = tu.tile_h;
      g.bins_chunk = tu.chunk;
    }
    if (tu.interp_mode == 0) {
      if (g.ibins_chunk != tu.chunk) {
        build_interp_bins(plan, g);
        g.ibins_chunk = tu.chunk;
      }
    } else {
      g.itiles_x = g.itiles_y = 0;
      g.ipts.clear();
      g.iitems.clear();
      g.ibins_chunk = -1;
    }
  }

  const int ns = int(plan.slices.size());
  // per-slice scratch: T (its q rows rounded up to a multiple of 4), ext and
  // yh, each 256-byte aligned
  auto scratch_bytes = [&](const Geom& g, size_t& t_off, size_t& ext_off, size_t& yh_off) {
    t_off = 0;
    ext_off = align_up(size_t((g.G / 2 + 4) / 4 * 4) * g.key.n * sizeof(f2), 256);
    yh_off = align_up(ext_off + size_t(g.rows) * g.cols * sizeof(f2), 256);
    return align_up(yh_off + size_t(g.key.n_angles) * g.H * sizeof(f2), 256);
  };
  if (tu.batch < 0 || tu.batch_mb < 0) {
    err = "batch and batch_mb must be >= 0";
    return NR_INVALID_ARG;
  }
  if (tu.streams < 1 || tu.streams > 8) {
    err = "streams must be in [1, 8]";
    return NR_INVALID_ARG;
  }
  // batches: consecutive slices while their scratch fits the budget (a slice
  // larger than the budget runs alone); a budget of one slot's size keeps each
  // slice's grids resident in the 256 MB last-level cache between stages
  const size_t budget = size_t(tu.batch_mb) << 20;
  plan.batches.clear();
  plan.work.clear();
  plan.slot_area = 0;
  plan.n_slots = 0;
  for (int b0 = 0; b0 < ns;) {
    Batch bt;
    size_t used = 0;
    for (int s = b0; s < ns; ++s) {
      const Geom& g = plan.geoms[size_t(plan.slice_geom[size_t(s)])];
      size_t t_off, e_off, y_off;
      const size_t need = scratch_bytes(g, t_off, e_off, y_off);
      if (!bt.slices.empty() && (used + need > budget || (tu.batch > 0 && int(bt.slices.size()) >= tu.batch)))
        break;
      bt.slices.push_back(s);
      bt.slot_off.push_back(used);
      used += need;
    }
    b0 += int(bt.slices.size());
    bt.bytes = used;
    plan.slot_area = std::max(plan.slot_area, used);
    plan.n_slots = std::max(plan.n_slots, int(bt.slices.size()));
    // FFT lengths present in this batch
    std::vector<int> Gs, Nts;
    for (int s : bt.slices) {
      const Geom& g = plan.geoms[size_t(plan.slice_geom[size_t(s)])];
      if (std::find(Gs.begin(), Gs.end(), g.G) == Gs.end()) Gs.push_back(g.G);
      if (std::find(Nts.begin(), Nts.end(), g.key.n_det) == Nts.end()) Nts.push_back(g.key.n_det);
    }
    auto add = [&](std::vector<StageLaunch>& seq, Stage st, int L, bool by_G, bool xcd, auto&& units) {
      std::vector<WorkItem> logical;
      for (int s : bt.slices) {
        const Geom& g = plan.geoms[size_t(plan.slice_geom[size_t(s)])];
        if (L > 0 && (by_G ? g.G : g.key.n_det) != L) continue;
        units(s, g, logical);
      }
      if (logical.empty()) return;
      StageLaunch sl{st, L, plan.work.size() * sizeof(WorkItem), 0};
      append_units(plan.work, logical, xcd);
      sl.n_work = int(plan.work.size() * sizeof(WorkItem) - sl.work_off) / int(sizeof(WorkItem));
      seq.push_back(sl);
    };
    auto row_pairs = [](int s, const Geom& g, std::vector<WorkItem>& v) {
      for (int u = 0; u < g.key.n / 2; ++u) v.push_back({s, u});
    };
    auto columns = [](int s, const Geom& g, std::vector<WorkItem>& v) {
      for (int u = 0; u <= g.G / 2; ++u) v.push_back({s, u});
    };
    auto angle_pairs = [](int s, const Geom& g, std::vector<WorkItem>& v) {
      for (int u = 0; u < (g.key.n_angles + 1) / 2; ++u) v.push_back({s, u});
    };
    for (int G : Gs) add(bt.fwd, Stage::FwdRows, G, true, true, row_pairs);
    // columns XCD-interleaved: the four columns of a tile of T share its lines
    for (int G : Gs) add(bt.fwd, Stage::FwdCols, G, true, true, columns);
    // items of heavy tiles (near the origin) first, over every slice of the batch
    auto heaviest_first = [&](Stage st, auto&& items_of) {
      std::vector<WorkItem> logical;
      std::vector<int> weight;
      for (int s : bt.slices) {
        const Geom& g = plan.geoms[size_t(plan.slice_geom[size_t(s)])];
        const std::vector<SpreadItem>& its = items_of(g);
        for (int u = 0; u < int(its.size()); ++u) {
          logical.push_back({s, u});
          weight.push_back(its[size_t(u)].end - its[size_t(u)].begin);
        }
      }
      if (logical.empty()) return std::vector<StageLaunch>{};
      std::vector<size_t> order(logical.size());
      for (size_t i = 0; i < order.size(); ++i) order[i] = i;
      std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return weight[a] > weight[b]; });
      std::vector<WorkItem> sorted;
      for (size_t i : order) sorted.push_back(logical[i]);
      StageLaunch sl{st, 0, plan.work.size() * sizeof(WorkItem), int(sorted.size())};
      append_units(plan.work, sorted, false);
      return std::vector<StageLaunch>{sl};
    };
    if (tu.interp_mode == 0) {
      for (const StageLaunch& sl : heaviest_first(Stage::FwdInterp, [](const Geom& g) -> const std::vector<SpreadItem>& {
             return g.iitems;
           }))
        bt.fwd.push_back(sl);
      for (int L : Nts) add(bt.fwd, Stage::FwdRadial, L, false, true, angle_pairs);
    } else {
      for (int L : Nts) add(bt.fwd, Stage::FwdInterp, L, false, true, angle_pairs);
    }
    for (int L : Nts) add(bt.adj, Stage::AdjRadial, L, false, false, angle_pairs);
    add(bt.adj, Stage::SpreadZero, 0, true, false, [](int s, const Geom& g, std::vector<WorkItem>& v) {
      for (int u = 0; u < int(g.zero_tiles.size()); ++u) v.push_back({s, u});
    });
    // spreading items of the whole batch, heaviest first (every tile has at
    // least one item, so the launch always exists)
    for (const StageLaunch& sl : heaviest_first(Stage::Spread, [](const Geom& g) -> const std::vector<SpreadItem>& {
           return g.items;
         }))
      bt.adj.push_back(sl);
    for (int G : Gs) add(bt.adj, Stage::AdjCols, G, true, true, columns);
    for (int G : Gs) add(bt.adj, Stage::AdjRows, G, true, true, row_pairs);
    plan.batches.push_back(std::move(bt));
  }

  // persistent launches: per batch, each slice's units go to one of
  // kPersistQueues queues (one per XCD; slices assigned largest first to the
  // least loaded queue by their forward + adjoint model bytes), stage-major
  // in chain order within a queue; each unit waits for the whole previous
  // non-empty stage of its slice
  plan.pentries.clear();
  plan.ptables.clear();
  plan.psync_ints = 1;   // the error flag
  if (tu.persistent) {
    if (plan.kb.W != 7 || tu.tile_w != 64 || tu.tile_h != 32 || tu.interp_mode != 0) {
      err = "persistent launches need kernel width 7, the 64x32 spreading tile and interp_mode 0";
      return NR_UNSUPPORTED_SIZE;
    }
    for (const Geom& g : plan.geoms)
      if (!persist_length_supported(g.G) || !persist_length_supported(g.key.n_det)) {
        err = "persistent launches are built for FFT lengths 128..4096 (powers of two); slice has G = " +
              std::to_string(g.G) + ", N_t = " + std::to_string(g.key.n_det);
        return NR_UNSUPPORTED_SIZE;
      }
    const Stage chain[] = {Stage::FwdRows, Stage::FwdCols, Stage::FwdInterp, Stage::FwdRadial, Stage::AdjRadial,
                           Stage::SpreadZero, Stage::Spread, Stage::AdjCols, Stage::AdjRows};
    for (Batch& bt : plan.batches) {
      const int n = int(bt.slices.size());
      const int first = bt.slices.front();
      // queue of each slice
      std::vector<int> order(size_t(n), 0), queue_of(size_t(n), 0);
      std::vector<double> bytes(size_t(n), 0.0), load(kPersistQueues, 0.0);
      for (int k = 0; k < n; ++k) {
        const Geom& g = plan.geoms[size_t(plan.slice_geom[size_t(bt.slices[size_t(k)])])];
        const double N = g.key.n, half = g.G / 2 + 1, na = g.key.n_angles, H = g.H, nt = g.key.n_det;
        bytes[size_t(k)] = 8 * N * N + 32 * N * half + g.G * half * (24.0 + 2.0 * M_PI) + 32 * na * H + 8 * na * nt;
        order[size_t(k)] = k;
      }
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return bytes[size_t(x)] > bytes[size_t(y)]; });
      for (int k : order) {
        const size_t qi = size_t(std::min_element(load.begin(), load.end()) - load.begin());
        queue_of[size_t(k)] = int(qi);
        load[qi] += bytes[size_t(k)];
      }
      std::vector<std::vector<PersistEntry>> queues(kPersistQueues);
      std::vector<int32_t> need(size_t(n) * kPersistStages, 0), dep(size_t(n) * kPersistStages, -1);
      for (int pass = 0; pass < 2; ++pass)
        for (const StageLaunch& sl : pass == 0 ? bt.fwd : bt.adj) {
          const WorkItem* w = plan.work.data() + sl.work_off / sizeof(WorkItem);
          for (int i = 0; i < sl.n_work; ++i) {
            if (w[i].slice < 0) continue;
            const int k = w[i].slice - first;
            queues[size_t(queue_of[size_t(k)])].push_back({w[i].slice, int(sl.stage), w[i].unit, sl.L});
            need[size_t(k) * kPersistStages + size_t(sl.stage)] += 1;
          }
        }
      for (int k = 0; k < n; ++k) {
        int prev = -1;
        for (Stage st : chain) {
          const size_t c = size_t(k) * kPersistStages + size_t(st);
          dep[c] = prev < 0 ? -1 : int32_t(size_t(k) * kPersistStages + size_t(prev));
          if (need[c] > 0) prev = int(st);
        }
      }
      bt.pe_first = plan.pentries.size();
      bt.pt_off = plan.ptables.size();
      int32_t q0 = 0;
      for (int qi = 0; qi < kPersistQueues; ++qi) {
        plan.ptables.push_back(q0);
        q0 += int32_t(queues[size_t(qi)].size());
        plan.pentries.insert(plan.pentries.end(), queues[size_t(qi)].begin(), queues[size_t(qi)].end());
      }
      plan.ptables.push_back(q0);
      plan.ptables.insert(plan.ptables.end(), need.begin(), need.end());
      plan.ptables.insert(plan.ptables.end(), dep.begin(), dep.end());
      bt.ps_off = plan.psync_ints;
      plan.psync_ints += kPersistQueues + size_t(n) * kPersistStages;
    }
  }

  // workspace layout
  size_t off = 0;
  for (auto& kv : plan.deapod) {
    plan.off_deapod[kv.first] = off;
    off = align_up(off + kv.second.size() * sizeof(float), 256);
  }
  for (auto& kv : plan.twiddle) {
    plan.off_twiddle[kv.first] = off;
    off = align_up(off + kv.second.size() * sizeof(f2), 256);
  }
  for (auto& kv : plan.shift) {
    plan.off_shift[kv.first] = off;
    off = align_up(off + kv.second.size() * sizeof(f2), 256);
  }
  for (Geom& g : plan.geoms) {
    g.off_gxy = off;
    off = align_up(off + g.gxy.size() * sizeof(double), 256);
    g.off_flip = off;
    off = align_up(off + g.flip.size() * sizeof(int32_t), 256);
    g.off_pts = off;
    off = align_up(off + std::max<size_t>(1, g.pts.size()) * sizeof(int32_t), 256);
    g.off_items = off;
    off = align_up(off + g.items.size() * sizeof(SpreadItem), 256);
    g.off_zero = off;
    off = align_up(off + std::max<size_t>(1, g.zero_tiles.size()) * sizeof(int32_t), 256);
    g.off_ipts = off;
    off = align_up(off + std::max<size_t>(1, g.ipts.size()) * sizeof(int32_t), 256);
    g.off_iitems = off;
    off = align_up(off + std::max<size_t>(1, g.iitems.size()) * sizeof(SpreadItem), 256);
  }
  plan.off_desc = off;
  off = align_up(off + size_t(ns) * sizeof(SliceDesc), 256);
  plan.off_work = off;
  off = align_up(off + std::max<size_t>(1, plan.work.size()) * sizeof(WorkItem), 256);
  plan.off_pentries = off;
  off = align_up(off + std::max<size_t>(1, plan.pentries.size()) * sizeof(PersistEntry), 256);
  plan.off_ptables = off;
  off = align_up(off + std::max<size_t>(1, plan.ptables.size()) * sizeof(int32_t), 256);
  plan.off_psync = off;
  off = align_up(off + plan.psync_ints * sizeof(int32_t), 256);
  // batches round-robin over the lanes; each lane has its own scratch area
  plan.n_lanes = std::max(1, std::min(tu.streams, int(plan.batches.size())));
  for (size_t b = 0; b < plan.batches.size(); ++b) plan.batches[b].lane = int(b % size_t(plan.n_lanes));
  plan.off_slot = off;
  plan.ws_bytes = plan.off_slot + size_t(plan.n_lanes) * plan.slot_area;
  plan.laid_out = true;
  return NR_OK;
}

bool persist_length_supported(int L) { return L >= 128 && L <= 4096 && (L & (L - 1)) == 0; }

std::vector<SliceDesc> slice_descs(const Plan& plan, char* d_ws) {
  std::vector<SliceDesc> out(plan.slices.size());
  for (const Batch& bt : plan.batches) {
    for (size_t k = 0; k < bt.slices.size(); ++k) {
      const int s = bt.slices[k];
      const nr_slice& sl = plan.slices[size_t(s)];
      const Geom& g = plan.geoms[size_t(plan.slice_geom[size_t(s)])];
      SliceDesc d{};
      d.N = sl.n;
      d.Nt = sl.n_det;
      d.na = sl.n_angles;
      d.G = g.G;
      d.H = g.H;
      d.rows = g.rows;
      d.cols = g.cols;
      d.tiles_x = g.tiles_x;
      d.n_items = int(g.items.size());
      d.n_zero = int(g.zero_tiles.size());
      d.slot = int(k);
      d.vol_off = sl.vol_off;
      d.sino_off = sl.sino_off;
      d.deapod = reinterpret_cast<const float*>(d_ws + plan.off_deapod.at(sl.n));
      d.tw_G = reinterpret_cast<const float*>(d_ws + plan.off_twiddle.at(g.G));
      d.tw_Nt = reinterpret_cast<const float*>(d_ws + plan.off_twiddle.at(sl.n_det));
      d.shift = sl.center == 0.0
                    ? nullptr
                    : reinterpret_cast<const float*>(d_ws + plan.off_shift.at({sl.n_det, sl.center}));
      d.gxy = reinterpret_cast<const double*>(d_ws + g.off_gxy);
      d.flip = reinterpret_cast<const int32_t*>(d_ws + g.off_flip);
      char* slot = d_ws + plan.off_slot + size_t(bt.lane) * plan.slot_area + bt.slot_off[k];
      const size_t ext_off = align_up(size_t((g.G / 2 + 4) / 4 * 4) * g.key.n * sizeof(f2), 256);
      const size_t yh_off = align_up(ext_off + size_t(g.rows) * g.cols * sizeof(f2), 256);
      d.T = reinterpret_cast<float*>(slot);
      d.ext = reinterpret_cast<float*>(slot + ext_off);
      d.yh = reinterpret_cast<float*>(slot + yh_off);
      d.pts = reinterpret_cast<const int32_t*>(d_ws + g.off_pts);
      d.items = reinterpret_cast<const SpreadItem*>(d_ws + g.off_items);
      d.zero_tiles = reinterpret_cast<const int32_t*>(d_ws + g.off_zero);
      d.itiles_x = g.itiles_x;
      d.rdisc = disc_radius(plan, g);
      d.jbits = g.jbits;
      d.ipts = reinterpret_cast<const int32_t*>(d_ws + g.off_ipts);
      d.iitems = reinterpret_cast<const SpreadItem*>(d_ws + g.off_iitems);
      out[size_t(s)] = d;
    }
  }
  return out;
}

}  // namespace nr
