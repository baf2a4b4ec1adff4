// Launch interface of the projector kernels (host side of radon_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "layout.hpp"

namespace nrk {

// Everything one slice's kernels need, by value.
struct SliceArgs {
  const float* vol_in;     // forward input  f[N][N]
  float* vol_out;          // adjoint output g[N][N]
  const float* sino_in;    // adjoint input  y[na][Nt]
  float* sino_out;         // forward output s[na][Nt]
  int N, Nt, na, G, H;
  int rows, cols, halo, colpad;
  const float* deapod;     // [N] 1/phihat((i - N/2)/G)
  const float2* tw_G;      // [G] exp(-2 pi i m/G)
  const float2* tw_Nt;     // [Nt] exp(-2 pi i m/Nt)
  const double* gxy;       // [na][2] grid step per radial index
  const int* flip;         // [na] conjugate flag
  float2* T;               // [G/2+1][N]
  float2* ext;             // [rows][cols]
  float2* yh;              // [na][H]
  const int* pts;          // spreading point lists
  const SpreadItem* items;
  const int* zero_tiles;
  int n_items, n_zero;
  int tile_w, tile_h, tiles_x;
};

// Kaiser-Bessel tap polynomials: c[i*(W+3) + k] is the z^k coefficient of tap i.
struct KBArgs {
  float c[8 * 11];
};

// Stages of the forward chain (FwdRows, FwdCols, FwdInterp) and of the
// adjoint chain (AdjRadial, Spread, AdjCols, AdjRows), launched in that order.
enum class Stage : int { FwdRows = 0, FwdCols, FwdInterp, AdjRadial, Spread, AdjCols, AdjRows, Count };

// spread_mode 0: LDS tiles (default), 1: plain global atomics (reference)
hipError_t launch_stage(Stage stage, const SliceArgs& a, const KBArgs& kb, int W, int spread_mode, hipStream_t st);

}  // namespace nrk
