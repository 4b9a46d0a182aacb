// The per-ray voxel walk with its merged updates, shared by the per-scan and
// the batched integration kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ohm_device.h"
#include "ohm_regions.h"
#include "ohm_wave.h"

namespace ohm {

// ---------------------------------------------------------------------------
// voxel walk
// ---------------------------------------------------------------------------

enum : int { kSinkCount = 0, kSinkCas = 1, kSinkTraceCount = 2, kSinkTraceWrite = 3 };

// LDS hash table of the aggregating walk: 2^kWalkLdsLog2 (voxel, kind)
// entries of 8 bytes; 0 applies every merged update straight to global memory.
#ifndef OHM_WALK_LDS_LOG2
#define OHM_WALK_LDS_LOG2 0
#endif
constexpr int kWalkLdsLog2 = OHM_WALK_LDS_LOG2;

// Per-update clamp-add by compare-and-swap, retried until it lands.
__device__ __forceinline__ void cas_clamp_add(float* p, float delta, float lo, float hi) {
  uint32_t* u = reinterpret_cast<uint32_t*>(p);
  uint32_t old = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    float nv = fminf(fmaxf(__uint_as_float(old) + delta, lo), hi);
    uint32_t prev = atomicCAS(u, old, __float_as_uint(nv));
    if (prev == old) break;
    old = prev;
  }
}

constexpr uint32_t kLdsEmpty = 0xFFFFFFFFu;

// Adds v to entry `id` of the block's LDS hash table (open addressing,
// linear probing).  False when the probe budget runs out; the caller then
// applies the update to global memory itself.
template <int kLog2>
__device__ __forceinline__ bool lds_add(uint32_t* keys, float* vals, uint32_t id, float v) {
  uint32_t h = (id * 0x9E3779B1u) >> (32 - kLog2);
#pragma unroll 1
  for (int p = 0; p < 32; ++p) {
    uint32_t k = __hip_atomic_load(keys + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (k == kLdsEmpty) {
      const uint32_t old = atomicCAS(keys + h, kLdsEmpty, id);
      k = old == kLdsEmpty ? id : old;
    }
    if (k == id) {
      atomicAdd(vals + h, v);
      return true;
    }
    h = (h + 1) & ((1u << kLog2) - 1);
  }
  return false;
}

// The per-ray walk of one block: thread `i` of the scan handles ray r0 + i
// (i >= n: idle).  `origin` points at the scan's sensor position.  Must be
// reached by every thread of the block.
template <int kSink, bool kWeighted, int kLdsLog2>
__device__ __forceinline__ void walk_body(const DevMap& m, const float* __restrict__ origin,
                                          const float* __restrict__ samples, const float* __restrict__ weights,
                                          uint32_t r0, uint32_t n, uint32_t i, uint32_t tag, uint32_t parity,
                                          uint32_t* __restrict__ ray_counts, int32_t* __restrict__ ray_flags,
                                          const int64_t* __restrict__ ray_offsets, int32_t* __restrict__ updates) {
  constexpr bool kAccum = kSink == kSinkCount || kSink == kSinkCas;
  constexpr bool kLds = kAccum && kLdsLog2 > 0;
  constexpr int kEntries = kLds ? (1 << kLdsLog2) : 1;
  __shared__ uint32_t s_key[kEntries];
  __shared__ float s_val[kEntries];
  if (kLds) {
    for (int h = threadIdx.x; h < kEntries; h += blockDim.x) {
      s_key[h] = kLdsEmpty;
      s_val[h] = 0.f;
    }
    __syncthreads();
  }
  // applies a merged update of weight v to (voxel, kind) `id`
  auto emit = [&](uint32_t id, float v) {
    if (kLds && lds_add<kLds ? kLdsLog2 : 1>(s_key, s_val, id, v)) return;
    if (kSink == kSinkCount)
      unsafeAtomicAdd(m.acc + id, v);
    else
      cas_clamp_add(m.occ + (id >> 1), v * ((id & 1u) ? m.l_hit : m.l_miss), m.l_min, m.l_max);
  };
  const uint32_t lane = lane_id();
  const bool inrange = i < n;
  const size_t ray = (size_t)r0 + i;
  const float o[3] = {origin[0], origin[1], origin[2]};
  float e[3] = {0.f, 0.f, 0.f};
  if (inrange) {
    e[0] = samples[3 * ray + 0];
    e[1] = samples[3 * ray + 1];
    e[2] = samples[3 * ray + 2];
  }
  Ray r;
  int st = inrange ? prepare_ray(m, o, e, r) : kRayInvalid;
  bool alive = inrange && st == kRayOk;
  const float wt = (kWeighted && inrange) ? weights[ray] : 1.0f;

  __shared__ RegionCache rc;
  if (kAccum) stage_regions<kSink == kSinkCount>(m, rc, alive, r, tag, parity);

  Walk w;
  int32_t kx = 0, ky = 0, kz = 0;
  int32_t slot = -1;
  uint32_t lidx = 0;
  if (alive) {
    int32_t hi[3] = {m.kmax[0] - 1, m.kmax[1] - 1, m.kmax[2] - 1};
    walk_init(w, r.q0, r.q1, r.k0, r.k1, m.kmin, hi, m.F);
    kx = r.k0[0];
    ky = r.k0[1];
    kz = r.k0[2];
    if (kAccum) slot = staged_slot(m, rc, kx, ky, kz);
    lidx = local_index(kx, ky, kz);
  }
  uint32_t n_upd = 0, n_drop = 0, n_hit = 0;
  bool clipped = false;
  int64_t out_base = 0;
  if (kSink == kSinkTraceWrite && inrange) out_base = ray_offsets[ray];

  while (__ballot(alive)) {
    const bool last = alive && w.total == 0;
    const bool is_hit = last && !r.truncated;
    if (kAccum) {
      const bool has = alive && slot >= 0;
      const uint32_t id = has ? (((uint32_t)slot * (uint32_t)kRegionVoxels + lidx) << 1) | (is_hit ? 1u : 0u)
                              : (0xFFFFFFFFu - lane);
      const LaneRuns run = lane_runs(id, lane);
      if (!kWeighted) {
        if (has && run.head) emit(id, (float)run.len);
      } else {
        // the run's last lane holds the summed weight
        const float v = segmented_sum(has ? wt : 0.f, run.head, lane);
        if (has && run.tail) emit(id, v);
      }
      if (alive) {
        if (slot >= 0) {
          ++n_upd;
          n_hit += is_hit ? 1u : 0u;
        } else {
          ++n_drop;
        }
      }
    } else {
      if (alive) {
        if (kSink == kSinkTraceWrite) {
          int32_t* out = updates + 4 * (out_base + n_upd);
          out[0] = kx;
          out[1] = ky;
          out[2] = kz;
          out[3] = is_hit ? 1 : 0;
        }
        ++n_upd;
        n_hit += is_hit ? 1u : 0u;
      }
    }
    // advance
    if (alive) {
      if (last) {
        alive = false;
      } else {
        const int a = walk_step(w);
        const int32_t ra = a == 0 ? w.rem[0] : (a == 1 ? w.rem[1] : w.rem[2]);
        if (ra == 0 && ((w.clip >> a) & 1u)) {
          alive = false;
          clipped = true;
        } else {
          const int32_t sg = a == 0 ? w.sg[0] : (a == 1 ? w.sg[1] : w.sg[2]);
          kx += a == 0 ? sg : 0;
          ky += a == 1 ? sg : 0;
          kz += a == 2 ? sg : 0;
          const int32_t kn = a == 0 ? kx : (a == 1 ? ky : kz);
          const bool wrap = (kn & kRegionMask) == (sg > 0 ? 0 : kRegionMask);
          if (wrap) {
            if (kAccum) slot = staged_slot(m, rc, kx, ky, kz);
            lidx = local_index(kx, ky, kz);
          } else {
            lidx += (uint32_t)(a == 0 ? sg : (a == 1 ? sg * kRegionEdge : sg * kRegionEdge * kRegionEdge));
          }
        }
      }
    }
  }

  if (kSink == kSinkTraceCount || kSink == kSinkTraceWrite) {
    if (kSink == kSinkTraceCount && inrange) {
      int32_t flags = 0;
      if (st == kRayInvalid) flags |= 8;
      if (st == kRayOriginOob) flags |= 16;
      if (st == kRayOk) {
        flags |= r.truncated ? 1 : 0;
        flags |= clipped ? 2 : 0;
        flags |= n_hit ? 4 : 0;
      }
      ray_counts[ray] = n_upd;
      ray_flags[ray] = flags;
    }
    return;
  }
  if (kLds) {
    // flush the block's merged updates
    __syncthreads();
    for (int h = threadIdx.x; h < kEntries; h += blockDim.x) {
      const uint32_t k = s_key[h];
      if (k == kLdsEmpty) continue;
      const float v = s_val[h];
      if (kSink == kSinkCount)
        unsafeAtomicAdd(m.acc + k, v);
      else
        cas_clamp_add(m.occ + (k >> 1), v * ((k & 1u) ? m.l_hit : m.l_miss), m.l_min, m.l_max);
    }
  }
  uint32_t vals[kStatCount];
  vals[kStatRays] = inrange ? 1u : 0u;
  vals[kStatInvalid] = (inrange && st == kRayInvalid) ? 1u : 0u;
  vals[kStatOriginOob] = (inrange && st == kRayOriginOob) ? 1u : 0u;
  vals[kStatTruncated] = (st == kRayOk && inrange && r.truncated) ? 1u : 0u;
  vals[kStatClipped] = clipped ? 1u : 0u;
  vals[kStatHits] = n_hit;
  vals[kStatUpdates] = n_upd;
  vals[kStatDropped] = n_drop;
  flush_stats(m, vals);
}

}  // namespace ohm
