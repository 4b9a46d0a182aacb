// Segmented voxel walk kernel body: a block processes the segments (see
// ohm_seg_math.h) of a tile of 256 rays, segment level by segment level, with
// 256, 512 or 1024 threads.
//
// Why: one thread per whole ray leaves lanes idle behind the longest ray of
// their wave and, for a 131k-ray scan, keeps only two waves per SIMD.  With
// segments every lane works on at most K major steps, so waves stay full and
// a block can run several threads per ray.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ohm_device.h"
#include "ohm_regions.h"
#include "ohm_seg_math.h"
#include "ohm_walk_body.h"
#include "ohm_wave.h"

namespace ohm {

// Per-ray data a tile keeps in LDS.
struct TileRays {
  long long q0[3][kTileRays];
  long long q1[3][kTileRays];
  uint8_t nseg[kTileRays];
  uint8_t trunc[kTileRays];
  uint16_t level_base[kMaxLevels + 1];
  uint16_t wave_count[kMaxLevels][kTileRays / 64];
  uint8_t item_ray[kMaxItems];
  uint32_t max_seg;
};

// One block processes the tile of rays [tile0, tile0 + kTileRays) of a scan
// (n rays from r0).  Every thread of the block must call it.
template <int kSink, bool kWeighted>
__device__ void walk_tile(const DevMap& m, const float* __restrict__ origin, const float* __restrict__ samples,
                          const float* __restrict__ weights, uint32_t r0, uint32_t n, uint32_t tile0, int K,
                          uint32_t tag, uint32_t parity, uint32_t* __restrict__ ray_counts,
                          int32_t* __restrict__ ray_flags, const int64_t* __restrict__ ray_offsets,
                          int32_t* __restrict__ updates) {
  constexpr bool kAccum = kSink == kSinkCount || kSink == kSinkCas;
  __shared__ TileRays tr;
  __shared__ RegionCache rc;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = lane_id();
  // --- prologue: prepare the tile's rays (threads 0..255) ---
  bool ok = false;
  int st = kRayInvalid;
  Ray r;
  const uint32_t ti = tid;  // tile-local ray of this thread in the prologue
  const bool holds_ray = ti < (uint32_t)kTileRays;
  const bool inrange = holds_ray && tile0 + ti < n;
  if (tid == 0) tr.max_seg = 0;
  if (inrange) {
    const size_t ray = (size_t)r0 + tile0 + ti;
    const float o[3] = {origin[0], origin[1], origin[2]};
    const float e[3] = {samples[3 * ray + 0], samples[3 * ray + 1], samples[3 * ray + 2]};
    st = prepare_ray(m, o, e, r);
    ok = st == kRayOk;
  }
  __syncthreads();
  uint32_t nseg = 0;
  uint32_t total_upd = 0;
  bool clipped_ray = false;
  if (holds_ray) {
    if (ok) {
      Walk w;
      const int32_t hi[3] = {m.kmax[0] - 1, m.kmax[1] - 1, m.kmax[2] - 1};
      walk_init(w, r.q0, r.q1, r.k0, r.k1, m.kmin, hi, m.F);
      nseg = seg_count(w, r.q0, r.q1, K);
      // the end voxel lies outside the map exactly when some axis is clipped
      clipped_ray = w.clip != 0;
      total_upd = walk_voxels(w, r.q0, r.q1, m.F);
      for (int a = 0; a < 3; ++a) {
        tr.q0[a][ti] = r.q0[a];
        tr.q1[a][ti] = r.q1[a];
      }
      tr.trunc[ti] = r.truncated ? 1 : 0;
      atomicMax(&tr.max_seg, nseg);
    }
    tr.nseg[ti] = (uint8_t)nseg;
  }
  if (kAccum) stage_regions<kSink == kSinkCount>(m, rc, ok, r, tag, parity);
  else __syncthreads();
  // --- segment-major item list: level j holds the rays with nseg > j ---
  const uint32_t levels = tr.max_seg;
  const uint32_t wave = tid >> 6;
  for (uint32_t j = 0; j < levels; ++j) {
    if (holds_ray) {
      const unsigned long long bal = __ballot(nseg > j);
      if (lane == 0) tr.wave_count[j][wave] = (uint16_t)__popcll(bal);
    }
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (uint32_t j = 0; j < levels; ++j) {
      tr.level_base[j] = (uint16_t)acc;
      for (int w = 0; w < kTileRays / 64; ++w) {
        const uint32_t c = tr.wave_count[j][w];
        tr.wave_count[j][w] = (uint16_t)acc;  // now: this wave's offset
        acc += c;
      }
    }
    tr.level_base[levels] = (uint16_t)acc;
  }
  __syncthreads();
  for (uint32_t j = 0; j < levels; ++j) {
    if (holds_ray) {
      const unsigned long long bal = __ballot(nseg > j);
      if (nseg > j) {
        const unsigned long long below = lane == 0 ? 0ull : (bal & (~0ull >> (64 - lane)));
        tr.item_ray[tr.wave_count[j][wave] + __popcll(below)] = (uint8_t)ti;
      }
    }
  }
  __syncthreads();
  const uint32_t items = tr.level_base[levels];

  // --- per-ray trace outputs and statistics (prologue threads) ---
  if (kSink == kSinkTraceCount && inrange) {
    int32_t flags = 0;
    if (st == kRayInvalid) flags |= 8;
    if (st == kRayOriginOob) flags |= 16;
    if (st == kRayOk) {
      flags |= r.truncated ? 1 : 0;
      flags |= clipped_ray ? 2 : 0;
      flags |= (!r.truncated && !clipped_ray) ? 4 : 0;
    }
    const size_t ray = (size_t)r0 + tile0 + ti;
    ray_counts[ray] = ok ? total_upd : 0u;
    ray_flags[ray] = flags;
  }
  uint32_t n_upd = 0, n_drop = 0, n_hit = 0;

  // --- items: segment walks with lane-run merging ---
  const uint32_t rounds = (items + blockDim.x - 1) / blockDim.x;
  for (uint32_t round = 0; round < rounds; ++round) {
    const uint32_t it = round * blockDim.x + tid;
    bool alive = it < items;
    uint32_t ray_t = 0, level = 0;
    SegState s;
    float wt = 1.f;
    bool trunc = false;
    int32_t slot = -1;
    uint32_t lidx = 0;
    int64_t out_base = 0;
    if (alive) {
      ray_t = tr.item_ray[it];
      while (level + 1 < levels && tr.level_base[level + 1] <= it) ++level;
      const int64_t q0[3] = {tr.q0[0][ray_t], tr.q0[1][ray_t], tr.q0[2][ray_t]};
      const int64_t q1[3] = {tr.q1[0][ray_t], tr.q1[1][ray_t], tr.q1[2][ray_t]};
      seg_init(s, q0, q1, m, (int)level, K);
      trunc = tr.trunc[ray_t] != 0;
      alive = !s.empty;
      const size_t ray = (size_t)r0 + tile0 + ray_t;
      if (kWeighted) wt = weights[ray];
      if (kSink == kSinkTraceWrite) out_base = ray_offsets[ray] + s.pos;
      if (kAccum && alive) slot = staged_slot(m, rc, s.k[0], s.k[1], s.k[2]);
      lidx = local_index(s.k[0], s.k[1], s.k[2]);
    }
    int M_axis = 0;
    if (alive) {
      const int64_t q0[3] = {tr.q0[0][ray_t], tr.q0[1][ray_t], tr.q0[2][ray_t]};
      const int64_t q1[3] = {tr.q1[0][ray_t], tr.q1[1][ray_t], tr.q1[2][ray_t]};
      M_axis = ray_major_axis(q0, q1);
    }
    uint32_t local = 0;
    while (__ballot(alive)) {
      const bool last = alive && s.w.total == 0;
      const bool is_hit = last && !trunc;
      if (kAccum) {
        const bool has = alive && slot >= 0;
        const uint32_t id = has ? (((uint32_t)slot * (uint32_t)kRegionVoxels + lidx) << 1) | (is_hit ? 1u : 0u)
                                : (0xFFFFFFFFu - lane);
        const LaneRuns run = lane_runs(id, lane);
        float v = 1.f;
        bool emit_here;
        if (!kWeighted) {
          v = (float)run.len;
          emit_here = has && run.head;
        } else {
          v = segmented_sum(has ? wt : 0.f, run.head, lane);
          emit_here = has && run.tail;
        }
        if (emit_here) {
          if (kSink == kSinkCount)
            unsafeAtomicAdd(m.acc + id, v);
          else
            cas_clamp_add(m.occ + (id >> 1), v * ((id & 1u) ? m.l_hit : m.l_miss), m.l_min, m.l_max);
        }
        if (alive) {
          if (slot >= 0) {
            ++n_upd;
            n_hit += is_hit ? 1u : 0u;
          } else {
            ++n_drop;
          }
        }
      } else if (alive && kSink == kSinkTraceWrite) {
        int32_t* out = updates + 4 * (out_base + local);
        out[0] = s.k[0];
        out[1] = s.k[1];
        out[2] = s.k[2];
        out[3] = is_hit ? 1 : 0;
      }
      if (alive) {
        ++local;
        if (last) {
          alive = false;
        } else {
          const int a = seg_advance(s, M_axis);
          if (a < 0) {
            alive = false;
          } else {
            const int32_t sg = pick3(a, s.w.sg[0], s.w.sg[1], s.w.sg[2]);
            const int32_t kn = pick3(a, s.k[0], s.k[1], s.k[2]);
            if ((kn & kRegionMask) == (sg > 0 ? 0 : kRegionMask)) {
              if (kAccum) slot = staged_slot(m, rc, s.k[0], s.k[1], s.k[2]);
              lidx = local_index(s.k[0], s.k[1], s.k[2]);
            } else {
              lidx += (uint32_t)(a == 0 ? sg : (a == 1 ? sg * kRegionEdge : sg * kRegionEdge * kRegionEdge));
            }
          }
        }
      }
    }
  }
  if (kSink == kSinkTraceCount || kSink == kSinkTraceWrite) return;
  uint32_t vals[kStatCount];
  vals[kStatRays] = inrange ? 1u : 0u;
  vals[kStatInvalid] = (inrange && st == kRayInvalid) ? 1u : 0u;
  vals[kStatOriginOob] = (inrange && st == kRayOriginOob) ? 1u : 0u;
  vals[kStatTruncated] = (inrange && ok && r.truncated) ? 1u : 0u;
  vals[kStatClipped] = (inrange && ok && clipped_ray) ? 1u : 0u;
  vals[kStatHits] = n_hit;
  vals[kStatUpdates] = n_upd;
  vals[kStatDropped] = n_drop;
  flush_stats(m, vals);
}

}  // namespace ohm
