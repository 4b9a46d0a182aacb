// Region allocation and the per-block region cache ("LDS-staged region
// keys").  Before a block walks its rays voxel by voxel it walks them region
// by region (the same exact walk with 2^(F+5) cells), gathers the distinct
// regions in LDS, and resolves each once: allocating a slot from the pool
// when the region is new and, in count mode, listing it for the scan's
// finalize.  The voxel walk then finds slots in LDS, so its inner loop
// issues no global loads.  This replaces the paper's CPU-side region walk
// (Sec. III-B, last paragraph) with a GPU pass fused into the walk kernel.
//
// When the bounding box of the regions the block's rays can enter holds at
// most kRegionWindow regions (coherent tiles: a few to a few dozen regions),
// the regions live in a dense LDS window over that box, so a lookup is one
// LDS read at a computed index; otherwise in an LDS hash set.
#pragma once

#include "ohm_device.h"
#include "ohm_wave.h"

namespace ohm {

constexpr int kRegionCacheLog2 = 9;  // 512 entries per block
constexpr int kRegionCacheSize = 1 << kRegionCacheLog2;
constexpr int kRegionWindow = 1024;   // dense window entries per block
constexpr int32_t kSlotNotCached = -4;
constexpr int32_t kWindowMarked = -5;  // window entry of a region some ray enters, not yet resolved
constexpr int kAllocSpinLimit = 1 << 20;  // bounded wait for a slot another block is publishing

// A block stages its regions either in the dense window or in the hash set
// (never both), so the two share their LDS.
struct RegionCache {
  union {
    struct {
      int32_t key[kRegionCacheSize];
      int32_t slot[kRegionCacheSize];
    };
    int32_t win[kRegionWindow];  // dense window: slot per region of the box, kSlotEmpty where no ray enters
  };
  int32_t lo[3], hi[3];        // region bounding box of the block's rays
};

// The block's choice of lookup structure, held in registers by every thread.
struct RegionWindow {
  int32_t x0, y0, z0;  // box origin (region coordinates)
  int32_t wx, wy;      // box extent in x and y
  uint32_t vol;        // entries in use
  bool on;             // the box fits the window
};

__device__ __forceinline__ uint32_t region_hash(int32_t r) {
  return ((uint32_t)r * 0x9E3779B1u) >> (32 - kRegionCacheLog2);
}

// Insert region r; false when the probe budget is exhausted.
__device__ __forceinline__ bool rc_insert(RegionCache& rc, int32_t r) {
  uint32_t h = region_hash(r);
  for (int p = 0; p < 16; ++p) {
    int32_t k = __hip_atomic_load(rc.key + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (k == kSlotEmpty) {
      const int32_t old = atomicCAS(rc.key + h, kSlotEmpty, r);
      k = old == kSlotEmpty ? r : old;
    }
    if (k == r) return true;
    h = (h + 1) & (kRegionCacheSize - 1);
  }
  return false;
}

__device__ __forceinline__ int32_t rc_find(const RegionCache& rc, int32_t r) {
  uint32_t h = region_hash(r);
  for (int p = 0; p < 16; ++p) {
    const int32_t k = rc.key[h];
    if (k == r) return rc.slot[h];
    if (k == kSlotEmpty) return kSlotNotCached;
    h = (h + 1) & (kRegionCacheSize - 1);
  }
  return kSlotNotCached;
}

__device__ __forceinline__ void append_touched(const DevMap& m, uint32_t parity, int32_t slot) {
  const uint32_t idx = atomicAdd(m.hdr + kHdrTouched0 + parity, 1u);
  m.touched[(size_t)parity * m.capacity + idx] = (uint32_t)slot;
}

// Slot of region r, allocating it when new.  With kTouch the slot is listed
// once per scan (tag) in the touched list of `parity`.  Returns a negative
// value when the pool is exhausted (updates to the region are dropped).
template <bool kTouch>
__device__ int32_t resolve_region(const DevMap& m, int32_t r, uint32_t tag, uint32_t parity) {
  int32_t slot = __hip_atomic_load(m.table + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (slot == kSlotEmpty) {
    const int32_t old = atomicCAS(m.table + r, kSlotEmpty, kSlotClaimed);
    if (old == kSlotEmpty) {
      const uint32_t s = atomicAdd(m.hdr + kHdrPoolCount, 1u);
      slot = s < m.capacity ? (int32_t)s : kSlotExhausted;
      if (slot == kSlotExhausted) atomicOr(reinterpret_cast<int32_t*>(m.hdr + kHdrSticky), kStickyPoolExhausted);
      __hip_atomic_store(m.table + r, slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      slot = old;
    }
  }
  // another block claimed the region and is publishing its slot
  for (int spin = 0; slot == kSlotClaimed && spin < kAllocSpinLimit; ++spin) {
    __builtin_amdgcn_s_sleep(1);
    slot = __hip_atomic_load(m.table + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (slot == kSlotClaimed) {
    atomicOr(reinterpret_cast<int32_t*>(m.hdr + kHdrSticky), kStickySlotTimeout);
    return kSlotExhausted;
  }
  if (kTouch && slot >= 0) {
    if (__hip_atomic_load(m.stamp + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != tag &&
        atomicExch(m.stamp + slot, tag) != tag)
      append_touched(m, parity, slot);
  }
  return slot;
}

// Region-level walk of one prepared ray: calls f(rx, ry, rz) for every
// region the voxel walk can enter, in order.
template <typename F>
__device__ __forceinline__ void for_each_region(const DevMap& m, const Ray& r, F&& f) {
  int32_t k0[3], k1[3], lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    k0[a] = r.k0[a] >> kRegionLog2;
    k1[a] = r.k1[a] >> kRegionLog2;
    lo[a] = m.kmin[a] >> kRegionLog2;
    hi[a] = (m.kmax[a] - 1) >> kRegionLog2;
  }
  Walk w;
  walk_init(w, r.q0, r.q1, k0, k1, lo, hi, m.F + kRegionLog2);
  int32_t rx = k0[0], ry = k0[1], rz = k0[2];
  for (;;) {
    f(rx, ry, rz);
    if (w.total == 0) break;
    const int a = walk_step(w);
    const int32_t ra = a == 0 ? w.rem[0] : (a == 1 ? w.rem[1] : w.rem[2]);
    if (ra == 0 && ((w.clip >> a) & 1u)) break;
    rx += a == 0 ? w.sg[0] : 0;
    ry += a == 1 ? w.sg[1] : 0;
    rz += a == 2 ? w.sg[2] : 0;
  }
}

// Block prologue: every thread passes its prepared ray (ok = valid); on
// return the block's region cache maps each region its rays enter to its
// slot, and the returned window says how to look slots up.  Must be reached
// by every thread of the block.
template <bool kTouch>
__device__ RegionWindow stage_regions(const DevMap& m, RegionCache& rc, bool ok, const Ray& r, uint32_t tag,
                                      uint32_t parity) {
  if (threadIdx.x < 3) {
    rc.lo[threadIdx.x] = 0x7fffffff;
    rc.hi[threadIdx.x] = (int32_t)0x80000000;
  }
  __syncthreads();
  for (int a = 0; a < 3; ++a) {
    // the walk stays between the origin's region and the (clipped) end's
    const int32_t lo = m.kmin[a] >> kRegionLog2, hi = (m.kmax[a] - 1) >> kRegionLog2;
    const int32_t s0 = r.k0[a] >> kRegionLog2;
    int32_t s1 = r.k1[a] >> kRegionLog2;
    s1 = s1 < lo ? lo : (s1 > hi ? hi : s1);
    const int32_t bmin = wave_min_i32(ok ? (s0 < s1 ? s0 : s1) : 0x7fffffff);
    const int32_t bmax = wave_max_i32(ok ? (s0 < s1 ? s1 : s0) : (int32_t)0x80000000);
    if (lane_id() == 0 && bmin <= bmax) {
      atomicMin(&rc.lo[a], bmin);
      atomicMax(&rc.hi[a], bmax);
    }
  }
  __syncthreads();
  RegionWindow w;
  w.x0 = rc.lo[0];
  w.y0 = rc.lo[1];
  w.z0 = rc.lo[2];
  const bool any = rc.lo[0] <= rc.hi[0];
  const int64_t ex = any ? (int64_t)rc.hi[0] - rc.lo[0] + 1 : 0;
  const int64_t ey = any ? (int64_t)rc.hi[1] - rc.lo[1] + 1 : 0;
  const int64_t ez = any ? (int64_t)rc.hi[2] - rc.lo[2] + 1 : 0;
  w.on = ex <= kRegionWindow && ey <= kRegionWindow && ez <= kRegionWindow && ex * ey * ez <= kRegionWindow;
  const int64_t vol = w.on ? ex * ey * ez : 0;
  w.wx = (int32_t)ex;
  w.wy = (int32_t)ey;
  w.vol = w.on ? (uint32_t)vol : 0u;
  if (w.on)
    for (uint32_t h = threadIdx.x; h < w.vol; h += blockDim.x) rc.win[h] = kSlotEmpty;
  else
    for (int h = threadIdx.x; h < kRegionCacheSize; h += blockDim.x) rc.key[h] = kSlotEmpty;
  __syncthreads();
  if (ok)
    for_each_region(m, r, [&](int32_t rx, int32_t ry, int32_t rz) {
      if (w.on) {
        const uint32_t h = (uint32_t)(((rz - w.z0) * w.wy + (ry - w.y0)) * w.wx + (rx - w.x0));
        if (h < w.vol) rc.win[h] = kWindowMarked;  // always inside the box
      } else {
        const int32_t ri = region_index(m, rx, ry, rz);
        if (!rc_insert(rc, ri)) (void)resolve_region<kTouch>(m, ri, tag, parity);
      }
    });
  __syncthreads();
  if (w.on) {
    for (uint32_t h = threadIdx.x; h < w.vol; h += blockDim.x) {
      if (rc.win[h] != kWindowMarked) continue;
      const int32_t rx = w.x0 + (int32_t)(h % (uint32_t)w.wx);
      const int32_t ry = w.y0 + (int32_t)((h / (uint32_t)w.wx) % (uint32_t)w.wy);
      const int32_t rz = w.z0 + (int32_t)(h / ((uint32_t)w.wx * (uint32_t)w.wy));
      rc.win[h] = resolve_region<kTouch>(m, region_index(m, rx, ry, rz), tag, parity);
    }
  } else {
    for (int h = threadIdx.x; h < kRegionCacheSize; h += blockDim.x) {
      const int32_t ri = rc.key[h];
      rc.slot[h] = ri == kSlotEmpty ? kSlotExhausted : resolve_region<kTouch>(m, ri, tag, parity);
    }
  }
  __syncthreads();
  return w;
}

// Slot of the region holding key (kx, ky, kz): LDS first (window or hash
// set), the table as fallback.
__device__ __forceinline__ int32_t staged_slot(const DevMap& m, const RegionCache& rc, const RegionWindow& w,
                                               int32_t kx, int32_t ky, int32_t kz) {
  const int32_t rx = kx >> kRegionLog2, ry = ky >> kRegionLog2, rz = kz >> kRegionLog2;
  int32_t s = kSlotNotCached;
  if (w.on) {
    const uint32_t h = (uint32_t)(((rz - w.z0) * w.wy + (ry - w.y0)) * w.wx + (rx - w.x0));
    s = h < w.vol ? rc.win[h] : kSlotNotCached;
    s = s == kSlotEmpty ? kSlotNotCached : s;
  } else {
    s = rc_find(rc, region_index(m, rx, ry, rz));
  }
  if (s == kSlotNotCached) {
    s = __hip_atomic_load(m.table + region_index(m, rx, ry, rz), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s = s < kSlotExhausted ? kSlotExhausted : s;  // consume the load here
  }
  return s;
}

// Accumulate statistics of a block into the map's counters with one atomic
// per counter per block.
__device__ __forceinline__ void flush_stats(const DevMap& m, const uint32_t (&vals)[kStatCount]) {
  __shared__ uint32_t part[kStatCount];
  if (threadIdx.x < kStatCount) part[threadIdx.x] = 0;
  __syncthreads();
  uint32_t lane = lane_id();
#pragma unroll
  for (int c = 0; c < kStatCount; ++c) {
    // most counters are per-ray flags: a ballot count replaces the butterfly
    // sum, and counters that are zero across the wave cost one ballot
    const unsigned long long nz = __ballot(vals[c] != 0u);
    if (nz == 0ull) continue;
    const uint32_t s = __ballot(vals[c] > 1u) == 0ull ? (uint32_t)__popcll(nz) : wave_sum_u32(vals[c]);
    if (lane == 0 && s) atomicAdd(&part[c], s);
  }
  __syncthreads();
  if (threadIdx.x < kStatCount && part[threadIdx.x])
    atomicAdd(m.stats + threadIdx.x, (unsigned long long)part[threadIdx.x]);
}

}  // namespace ohm
