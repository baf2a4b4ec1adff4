// Launch interface of the projector kernels (host side of radon_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "layout.hpp"

namespace nrk {

// Arguments of one stage launch (by value).
struct LaunchArgs {
  const SliceDesc* descs;   // device array, one per slice of the plan
  const WorkItem* work;     // device work list of this launch
  int n_work;
  int halo, colpad;
  const float* vol_in;      // caller buffers (+ per-slice offsets)
  float* vol_out;
  const float* sino_in;
  float* sino_out;
  const float* sino_sub;    // subtracted from the forward's output (residual R f - b) when not null
  int fbp_filter;           // adjoint radial weight: -1 none, 0 ramp, 1 ramp x Butterworth
  int fbp_order;
  float fbp_inv_cutoff;
};

// Kaiser-Bessel tap polynomials: c[i*(W+3) + k] is the z^k coefficient of tap i.
struct KBArgs {
  float c[8 * 11];
};

// The stage kernels (same order as nr::Stage).
enum class StageKind : int { FwdRows = 0, FwdCols, FwdInterp, AdjRadial, Spread, AdjCols, AdjRows, SpreadZero, FwdRadial };

// One grid-stride launch of `stage` over its work list; L = FFT length of the
// slices in the list (unused by the spreading stages).
hipError_t launch_stage(StageKind stage, int L, const LaunchArgs& a, const KBArgs& kb, int W, int tile_w,
                        int tile_h, hipStream_t st);

// Reference spreading of one slice (clear + one thread per point with
// global float atomics); host_desc is the host copy of that slice's descriptor.
hipError_t launch_spread_reference(const SliceDesc* d_descs, int slice, const SliceDesc& host_desc, int halo,
                                   int colpad, const KBArgs& kb, int W, hipStream_t st);

}  // namespace nrk
