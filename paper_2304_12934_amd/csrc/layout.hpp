// Plain structs shared by the host plan and the device kernels.
#pragma once

#include <cstdint>

// Spreading work item: a grid tile and a contiguous range of its point list.
struct SpreadItem {
  int32_t tile;         // tile index (row-major over tiles)
  int32_t begin, end;   // range in the geometry's point-index list
  int32_t flags;        // bit 0: tile shared by several items (accumulate with atomics)
                        // bit 1: this item also spreads the k = 0 point of every angle
  int32_t bound;        // most points of this item that touch any one cell of the tile
};
enum { kItemAtomic = 1, kItemDC = 2 };

// Interpolation tiles: a point belongs to the tile holding its first tap; the
// kernel stages the tile plus W + 1 cells (the footprint and a one-cell
// margin on each side) of the grid in LDS.  Interpolation items reuse
// SpreadItem with flags = bound = 0.
constexpr int kInterpTileW = 64, kInterpTileH = 32;

// Most points per spreading or interpolation work item (the kernels keep an
// item's points in registers, kMaxChunk / 256 per thread).
constexpr int kMaxChunk = 1024;

// One slice as the kernels see it (device resident, filled at bind time).
// Complex buffers are float pairs.
struct SliceDesc {
  int32_t N, Nt, na, G, H, rows, cols, tiles_x, n_items, n_zero, slot, itiles_x;
  int32_t rdisc;                  // cells of ext farther than rdisc from the origin are never read
  int32_t jbits;                  // point codes in pts/ipts: (angle << jbits) | radial index
  int64_t vol_off, sino_off;      // element offsets into the caller's buffers
  const float* deapod;            // [N] 1/phihat((i - N/2)/G)
  const float* tw_G;              // [G] exp(-2 pi i m/G)
  const float* tw_Nt;             // [Nt] exp(-2 pi i m/Nt)
  const float* shift;             // [Nt/2+1] exp(-2 pi i j c/Nt) for a rotation axis at bin Nt/2 + c; null if c = 0
  const double* gxy;              // [na][2] grid step per radial index (sign-flipped)
  const int32_t* flip;            // [na] conjugate flag
  float* T;                       // [G/2+1][N] complex, in tiles of 4 q x 2 rows
  float* ext;                     // [rows][cols] complex
  float* yh;                      // [na][H] complex
  const int32_t* pts;             // spreading point lists (tile-major)
  const SpreadItem* items;        // spreading work items of this slice's geometry
  const int32_t* zero_tiles;      // tiles written by several items
  const int32_t* ipts;            // interpolation point lists (tile-major, every point once)
  const SpreadItem* iitems;       // interpolation work items (tile, point range)
};

// One unit of work of a stage launch: (slice index in the plan, unit index
// within the slice: a row pair, a column, an angle pair, a spreading item...).
// slice < 0 marks padding.
struct WorkItem {
  int32_t slice, unit;
};

// Persistent launch: one kernel runs a batch's whole forward + adjoint chain.
// An entry names one unit of one stage (nr::Stage numbering) of one slice;
// the entries form one queue per XCD (each slice's units all in the queue of
// the XCD it is assigned to), stage-major within a queue, so that every unit
// depends only on units earlier in its own queue.
struct PersistEntry {
  int32_t slice, stage, unit, L;
};
constexpr int kPersistStages = 9;   // dependency counters per slice, indexed by stage
constexpr int kPersistQueues = 8;   // one queue per XCD

