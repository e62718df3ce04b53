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

namespace gabp {

constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_block(int i, int G) {
  const int x = i % kXcds, k = i / kXcds, q = G / kXcds, r = G % kXcds;
  return x * q + min(x, r) + k;
}

}  // namespace gabp
