// Workgroup numbering across the XCDs of gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rts {
// Workgroups are dealt to the 8 XCDs in turn (workgroup w to XCD w mod 8),
// each XCD with its own L2.  This renumbering gives each XCD one contiguous
// range of workgroup indices, so that neighbouring particles, which gather
// the same neighbour data, share an L2.  A bijection of [0, g).
constexpr uint32_t kXcds = 8;
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t g) {
  const uint32_t q = g / kXcds, r = g % kXcds;  // XCDs below r hold q + 1 workgroups
  const uint32_t x = b % kXcds, k = b / kXcds;
  return (x < r ? x * (q + 1u) : r * (q + 1u) + (x - r) * q) + k;
}

}  // namespace rts
