// XCD-aware block order for kernels whose rows gather from rows a grid side away.
//
// The MI355X's 256 compute units sit in 8 XCDs, each with its own L2, and a launch's
// workgroups are dispatched round-robin over the XCDs. A block that gathers x from rows one
// grid side away therefore reads lines that another XCD brought in (a side of 4095 rows is
// about 16 blocks of 256 rows). xcd_block maps the dispatched block i to a logical block so
// that every XCD covers one contiguous range of logical blocks; the map is a bijection on
// [0, G), so a kernel that uses it for its row range and for its per-block outputs computes
// exactly what it computes in dispatch order.
#pragma once

#include "gabp_internal.h"   // kXcds

namespace gabp {

__device__ __forceinline__ int xcd_block(int i, int G) {
  const int x = i % kXcds, k = i / kXcds, q = G / kXcds, r = G % kXcds;
  return x * q + min(x, r) + k;
}

// Tile of a tiled launch (one workgroup per tile, G = tiles_x * tiles_y tiles, row-major)
// that dispatched block b works on. The tiles are taken in strip-major order -- strips of
// `strip` tile columns (the last one narrower if strip does not divide tiles_x), each walked
// row by row -- and every XCD takes one contiguous run of that order (xcd_block). A tile
// reads the edge rows of its left, right, upper and lower neighbours as its halo; in this
// order those neighbours run at about the same time on the same XCD, so the halo's lines
// are found in that XCD's L2 instead of being fetched again (round-robin dispatch puts
// consecutive tiles on different XCDs). A bijection on [0, G).
__device__ __forceinline__ int tile_of_block(int b, int G, int tiles_x, int strip) {
  const int o = xcd_block(b, G);
  const int tiles_y = G / tiles_x;
  const int full = tiles_x / strip * strip;     // tile columns in whole strips
  if (o < full * tiles_y) {
    const int span = strip * tiles_y;            // tiles per whole strip
    const int st = o / span, rem = o - st * span;
    return (rem / strip) * tiles_x + st * strip + rem % strip;
  }
  const int wl = tiles_x - full, rem = o - full * tiles_y;
  return (rem / wl) * tiles_x + full + rem % wl;
}

}  // namespace gabp
