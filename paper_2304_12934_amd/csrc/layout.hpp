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
