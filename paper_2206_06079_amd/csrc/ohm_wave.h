// Wave-level helpers (64-wide wavefronts): lane shifts, run detection and
// segmented sums used to merge equal updates of adjacent lanes before they
// reach memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ohm {

// The tile a block of a tiled launch of nb blocks walks.  The device deals
// a launch's blocks to its 8 XCDs round-robin (block b to XCD b % 8), and
// each XCD has its own L2; this mapping gives every XCD a contiguous eighth
// of the tiles instead, so that neighbouring tiles of a scan, which share
// the voxels, regions and accumulator lines near their sensor, meet in one
// L2.  A bijection on [0, nb); the first nb % 8 XCDs take one tile more.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nb) {
  constexpr uint32_t kXcds = 8;
  const uint32_t per = nb / kXcds, rem = nb % kXcds, x = b % kXcds;
  return x * per + (x < rem ? x : rem) + b / kXcds;
}

// value of lane (l - 1); lane 0 receives `fill` (DPP wave_shr:1)
__device__ __forceinline__ uint32_t wave_shr1(uint32_t v, uint32_t fill) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, 0x138, 0xf, 0xf, false);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Butterfly min / max over the wave (every lane must take part; lanes with
// nothing to contribute pass the identity).  One LDS atomic per wave after
// this is far cheaper than one per lane to a shared address, which the
// compiler would serialise lane by lane.
__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(v, off);
    v = o < v ? o : v;
  }
  return v;
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

// Runs of equal ids over adjacent lanes.  Every lane learns whether it heads
// its run, whether it ends it, and (at the head) the run length.
struct LaneRuns {
  bool head, tail;
  uint32_t len;  // valid at the head
};

__device__ __forceinline__ LaneRuns lane_runs(uint32_t id, uint32_t lane) {
  const uint32_t prev = wave_shr1(id, ~id);
  const bool head = (lane == 0) || (prev != id);
  const unsigned long long heads = __ballot(head);
  const unsigned long long above = lane == 63 ? 0ull : (heads >> (lane + 1));
  LaneRuns r;
  r.head = head;
  r.tail = (lane == 63) || (above & 1ull);
  r.len = above ? (uint32_t)__builtin_ctzll(above) + 1u : 64u - lane;
  return r;
}

// Inclusive segmented sum over runs (segments start at heads); the run's last
// lane (tail) holds the run total.
template <typename T>
__device__ __forceinline__ T segmented_sum(T v, bool head, uint32_t lane) {
  uint32_t f = head ? 1u : 0u;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T vu = __shfl_up(v, off);
    const uint32_t fu = __shfl_up(f, off);
    if (lane >= (uint32_t)off && !f) {
      v += vu;
      f |= fu;
    }
  }
  return v;
}

}  // namespace ohm
