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
  int stream_stores;        // 1: the forward columns and the spreading store their rows non-temporally
  int pair_units;           // set by launch_stage: 1 when the forward columns run two units per workgroup
};

// Arguments of a persistent launch (one batch): the per-XCD queues of
// entries, their offsets, the dependency tables of the batch's slices
// (first_slice .. first_slice + n - 1) and the cleared counters.
struct PersistArgs {
  const PersistEntry* entries;
  const int32_t* qoff;       // kPersistQueues + 1 offsets into entries
  const int32_t* need;       // [slice][stage]: units of that stage
  const int32_t* dep;        // [slice][stage]: counter to wait for (-1: none)
  int32_t* tickets;          // kPersistQueues, cleared before the launch
  int32_t* done;             // [slice][stage], cleared before the launch
  int32_t* error;            // set when a wait gives up (not cleared by the launch)
  int first_slice;
  int spin_limit;
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

// Everything a persistent launch reads, as the kernel's single argument.
struct PersistLaunch {
  LaunchArgs a;
  PersistArgs p;
  KBArgs kb;
};

// Persistent launch of a batch's forward + adjoint chain (W = 7, spreading
// tile 64x32, FFT lengths 128..4096): clears `clear_count` ints at `clear`
// (the tickets and counters), then runs `blocks` resident workgroups.
hipError_t launch_persistent(const LaunchArgs& a, const PersistArgs& p, const KBArgs& kb, int W, int blocks,
                             int* clear, int clear_count, hipStream_t st);
// resident workgroups of the persistent kernel per CU (0 if W is not built)
int persist_blocks_per_cu(int W);
// p[0 .. n) = v
hipError_t launch_fill_int(int* p, size_t n, int v, hipStream_t st);

// Reference spreading of one slice (clear + one thread per point with
// global float atomics); host_desc is the host copy of that slice's descriptor.
hipError_t launch_spread_reference(const SliceDesc* d_descs, int slice, const SliceDesc& host_desc, int halo,
                                   int colpad, const KBArgs& kb, int W, hipStream_t st);

}  // namespace nrk
