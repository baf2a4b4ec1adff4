// Host-side plan: geometry validation, Kaiser-Bessel tables, per-angle
// coordinate tables, spreading bins, batched work lists and the workspace
// layout.  Pure C++ (no HIP) so it can be built and tested without a GPU.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "layout.hpp"
#include "nufftradon.h"

namespace nr {

// FFT lengths compiled into the device library: 2^a (16..8192) and 5*2^a (80..5120).
bool fft_length_supported(int L);

// Spreading tile shapes compiled into the device library (width x height).
bool spread_tile_supported(int w, int h);

struct f2 {
  float x, y;
};

// Kaiser-Bessel kernel phi(u) = I0(beta*sqrt(1-(2u/W)^2)) / I0(beta) on |u| <= W/2
// (Sec. 2.2: the compact spreading kernel of eq. "nufft2"), its continuous
// Fourier transform (divided out in eq. "nufft3"), and a piecewise polynomial
// of the W tap weights for the device.
struct KaiserBessel {
  int W = 7;
  double beta = 0.0;
  int D = 0;                   // polynomial degree
  std::vector<float> coef;     // [W][D+1], coefficient of z^k for tap i
  double i0beta = 1.0;

  void init(int width, double beta_in);   // beta_in <= 0: Beatty shape for sigma = 2
  double phi(double u) const;              // float64 series
  double phihat(double xi) const;          // closed form
  double phi_poly(double u) const;         // device polynomial (evaluated in float64)
  double max_poly_error() const;
};

double bessel_i0(double x);

// Tap convention shared by host tables and kernels: for a coordinate u (grid
// units) the first tap is g0 = ceil(u - W/2); tap i sits at g0 + i with offset
// d_i = u - g0 - i = z + (W-1)/2 - i, where z = u - g0 - (W-1)/2 lies in (-1/2, 1/2].

struct GeomKey {
  int n, n_det, n_angles;
  int64_t angle_off;
  bool operator<(const GeomKey& o) const {
    return std::tie(n, n_det, n_angles, angle_off) < std::tie(o.n, o.n_det, o.n_angles, o.angle_off);
  }
};

struct Geom {
  GeomKey key;
  int G = 0;            // oversampled grid size (sigma * N)
  int H = 0;            // half-line points N_t/2 + 1
  int jbits = 0;        // point codes (a << jbits) | j: the bits of j < H
  int rows = 0;         // extended grid rows G/2 + 1 + 2*halo
  int cols = 0;         // extended grid row length G + 2*colpad
  std::vector<double> gxy;          // per angle: (G cos/N_t, G sin/N_t), sign-flipped so that x >= 0
  std::vector<int32_t> flip;        // per angle: 1 if the spectrum value is conjugated
  // spreading bins (tile-major point lists; points j >= 1 only)
  int tile_w = 0, tile_h = 0, tiles_x = 0, tiles_y = 0;
  std::vector<int32_t> pts;         // point codes (a << jbits) | j, grouped by tile
  std::vector<int32_t> tile_start;  // tiles_x*tiles_y + 1 offsets into pts
  std::vector<SpreadItem> items;
  std::vector<int32_t> zero_tiles;  // tiles written by atomic items: cleared first
  // interpolation bins (every point j >= 0 once, by the tile of its first tap)
  int itiles_x = 0, itiles_y = 0;
  std::vector<int32_t> ipts;
  std::vector<SpreadItem> iitems;
  // tuning the bins were last built for (layouts that change only the
  // batching reuse them)
  int bins_tile_w = -1, bins_tile_h = -1, bins_chunk = -1, ibins_chunk = -1;
  // workspace offsets (bytes)
  size_t off_gxy = 0, off_flip = 0, off_pts = 0, off_items = 0, off_zero = 0, off_ipts = 0, off_iitems = 0;
};

// Tunable execution parameters: none changes results beyond float32 rounding
// (the order of the spreading sums).
struct Tuning {
  int tile_w = 64, tile_h = 32;   // spreading tile
  int chunk = 1024;               // most points per spreading item
  int batch = 0;                  // most slices per batched launch (0: no limit)
  int batch_mb = 160;             // scratch budget of one batch in MiB (a lone slice may exceed it)
  int spread_mode = 0;            // 0: LDS tiles, 1: global atomics (reference)
  int interp_mode = 0;            // 0: LDS tiles + radial pass, 1: direct gathers per angle pair
  int streams = 2;                // batches run round-robin on this many concurrent streams
  int persistent = 0;             // 1: a forward + adjoint pass runs each batch as one persistent launch
};

// Stages of the forward chain (FwdRows, FwdCols, FwdInterp, FwdRadial) and of the
// adjoint chain (AdjRadial, SpreadZero, Spread, AdjCols, AdjRows).
enum class Stage : int {
  FwdRows = 0, FwdCols, FwdInterp, AdjRadial, Spread, AdjCols, AdjRows, SpreadZero, FwdRadial, Count
};

// One kernel launch of a batch: every unit of `stage` over the batch's
// slices whose FFT length is L, listed at work_off in the workspace.
struct StageLaunch {
  Stage stage;
  int L;
  size_t work_off;    // bytes
  int n_work;         // entries (XCD padding included)
};

// The MI355X's last-level cache (Infinity Cache), 256 MiB.  A batch whose
// scratch grids exceed it has its stages store their large row outputs with
// non-temporal stores (the next stage finds them in HBM either way); a batch
// that fits keeps plain stores, so that the next stage reads from the cache.
constexpr size_t kLastLevelCacheBytes = size_t(256) << 20;

struct Batch {
  int lane = 0;                   // stream (and scratch area) the batch runs on
  size_t bytes = 0;               // scratch bytes of its slices (T, ext, yh)
  std::vector<int> slices;
  std::vector<size_t> slot_off;   // scratch offset of each slice inside its lane's slot area
  std::vector<StageLaunch> fwd, adj;
  // persistent launch (Tuning::persistent): entries [pe_first, pe_first + n)
  // in Plan::pentries; at pt_off in Plan::ptables the kPersistQueues + 1
  // queue offsets, then need[] and dep[] (kPersistStages per slice); at
  // ps_off in the sync area the tickets (kPersistQueues) and done counters
  size_t pe_first = 0, pt_off = 0, ps_off = 0;
};

struct Plan {
  std::vector<nr_slice> slices;
  std::vector<int> slice_geom;
  std::vector<Geom> geoms;
  std::vector<double> angles;       // copy of every referenced angle (indexed by angle_off + a)
  KaiserBessel kb;
  double sigma = 2.0;
  int halo = 0;                     // grid rows beyond the half-plane on each side
  int colpad = 0;                   // grid columns beyond the period on each side

  std::map<int, std::vector<float>> deapod;   // N -> 1/phihat((i - N/2)/G)
  std::map<int, size_t> off_deapod;
  std::map<int, std::vector<f2>> twiddle;     // L -> exp(-2 pi i m / L)
  std::map<int, size_t> off_twiddle;
  std::map<std::pair<int, double>, std::vector<f2>> shift;   // (N_t, c) -> exp(-2 pi i j c / N_t), j <= N_t/2
  std::map<std::pair<int, double>, size_t> off_shift;

  Tuning tune;
  bool laid_out = false;
  std::vector<Batch> batches;
  std::vector<WorkItem> work;       // every work list, concatenated
  size_t off_desc = 0, off_work = 0, off_slot = 0;
  size_t slot_area = 0;             // bytes of the largest batch's scratch (one area per lane)
  int n_lanes = 1;                  // concurrent streams in use (at most the number of batches)
  int n_slots = 0;                  // most slices in one batch
  size_t ws_bytes = 0;
  // persistent launches: every batch's entries, its tables, the sync area
  // (int32: the error flag at 0, then each batch's tickets and counters)
  std::vector<PersistEntry> pentries;
  std::vector<int32_t> ptables;
  size_t psync_ints = 0;
  size_t off_pentries = 0, off_ptables = 0, off_psync = 0;

  void* d_ws = nullptr;
  size_t d_ws_bytes = 0;
};

// Geometry, kernel and FFT tables; returns NR_OK or an error status with a message.
nr_status build_plan(const nr_slice* slices, int32_t n_slices, const double* angles,
                     const nr_nufft* params, Plan& plan, std::string& err);

// Spreading bins (for the current tuning), batches, work lists and the
// workspace layout.  Idempotent until the tuning changes.
nr_status layout_plan(Plan& plan, std::string& err);

// FFT lengths the persistent kernel is built for (128..4096, powers of two).
bool persist_length_supported(int L);

// Per-slice descriptors with absolute pointers into the workspace at d_ws.
std::vector<SliceDesc> slice_descs(const Plan& plan, char* d_ws);

// Radius (grid cells, from the origin of the spectrum) beyond which no
// spreading tap lands and no interpolation tap reads.
int disc_radius(const Plan& plan, const Geom& g);

// Fills the spreading bins of one geometry (called by layout_plan).
void build_spread_bins(const Plan& plan, Geom& g);

// Fills the interpolation bins of one geometry (called by layout_plan).
void build_interp_bins(const Plan& plan, Geom& g);

}  // namespace nr
