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

#include <type_traits>

#include "ohm_device.h"
#include "ohm_layers.h"
#include "ohm_regions.h"
#include "ohm_seg_math.h"
#include "ohm_wave.h"

namespace ohm {

// What a walk does with each voxel: count-mode accumulation, per-update CAS,
// or the per-ray trace outputs (voxel counts, then the voxel lists).
enum : int { kSinkCount = 0, kSinkCas = 1, kSinkTraceCount = 2, kSinkTraceWrite = 3 };

// Per-update clamp-add by compare-and-swap, retried until it lands.
__device__ __forceinline__ void cas_clamp_add(float* p, float delta, float lo, float hi) {
  uint32_t* u = reinterpret_cast<uint32_t*>(p);
  uint32_t old = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const float nv = fminf(fmaxf(__uint_as_float(old) + delta, lo), hi);
    const uint32_t prev = atomicCAS(u, old, __float_as_uint(nv));
    if (prev == old) break;
    old = prev;
  }
}

// Per-tile aggregation of updates: an LDS table of 2^kAggLog2 (update id ->
// summed weight) entries.  A merged update is added to the entry its id owns
// (claiming an empty one) among two probes; when both belong to other ids it
// is applied at once.  The table is applied with one atomic per entry when
// the tile ends, so the voxels that many rays of the tile cross cost one
// global atomic per tile instead of one per wave and step.  An id names one
// voxel and one kind (hit or miss), so an entry only sums increments of one
// sign; in per-update mode a clamp-add of that sum equals the clamp-adds of
// its parts in sequence.
//
// The table is laid out by 64-byte line of the accumulator: the 16 ids of a
// line (8 voxels along x, miss and hit) share one 16-entry group, at their
// position in the line, and the group is picked by hashing the line.  The
// end-of-tile flush, consecutive entries by consecutive lanes, then sends
// one wave's atomics to a few lines instead of 64 scattered ones: the memory
// side's atomic throughput is counted in lines, and scattered atomics are
// what bounds the walk once the voxel steps are cheap.  The second probe
// takes the same position in the next group.
constexpr int kAggLog2 = 12;
constexpr uint32_t kAggSize = 1u << kAggLog2;
constexpr uint32_t kAggEmpty = 0xFFFFFFFFu;  // above every update id (capacity <= kMaxCapacity)
constexpr uint32_t kAggLine = 16;            // ids per 64-byte accumulator line

__device__ __forceinline__ uint32_t agg_slot(uint32_t id) {
  const uint32_t group = ((id / kAggLine) * 0x9E3779B1u) >> (32 - (kAggLog2 - 4));
  return group * kAggLine + id % kAggLine;
}

// Claim-or-match entry h for id (k: its key as read before): true when the
// entry is (now) the id's.
__device__ __forceinline__ bool agg_own(uint32_t* keys, uint32_t h, uint32_t id, uint32_t k) {
  if (k == kAggEmpty) {
    const uint32_t old = atomicCAS(keys + h, kAggEmpty, id);
    k = old == kAggEmpty ? id : old;
  }
  return k == id;
}

// Second half of an insert whose first entry's key k = keys[agg_slot(id)]
// was read earlier: add v to the id's entry among the two probes.  False
// when both belong to other ids.
template <typename T>
__device__ __forceinline__ bool agg_finish(uint32_t* keys, T* vals, uint32_t id, uint32_t k, T v) {
  uint32_t h = agg_slot(id);
  if (!agg_own(keys, h, id, k)) {
    h = (h + kAggLine) & (kAggSize - 1);
    if (!agg_own(keys, h, id, keys[h])) return false;
  }
  atomicAdd(vals + h, v);
  return true;
}

// The batched plan's unit-weight walk keeps a different per-tile table,
// keyed by the 64-byte accumulator line itself: an entry holds one line's 16
// counts (8 voxels along x, miss and hit) as 16-bit counters, two to an LDS
// word.  A voxel is visited at most once per ray, so no count in a 256-ray
// tile exceeds 256 and the halves never carry into each other.  A tile
// touches 430 lines on average (p99 about 1,500) against about 1,430 update
// ids, so 1,024 line entries hold every line of most tiles, where the id
// table's 16-entry line groups overflow on hash collisions of lines.
// Lookups probe up to kLineProbes consecutive entries; an update finding
// none of them is applied to the accumulator at once.  A lane that claims an
// entry appends it to a list, so the flush visits only the claimed entries,
// each by 16 consecutive lanes.  (Fewer entries and fallbacks also make the
// brick marks below cheaper; on the spinning-lidar groups the id table is
// faster.)
constexpr uint32_t kLineEntries = 1024;
constexpr uint32_t kLineWords = 8;  // 16 x u16 counts per entry
constexpr int kLineProbes = 4;

__device__ __forceinline__ uint32_t line_slot(uint32_t line) {
  return (line * 0x9E3779B1u) >> (32 - 10);
}
static_assert(kLineEntries == 1024u, "line_slot hashes to 10 bits");

// Add `len` unit updates of id to the line table (k: the key of the first
// probe, read earlier); false when no probed entry is, or could become, the
// line's.  A claimed entry is appended to list[*n_list].
__device__ __forceinline__ bool line_add(uint32_t* keys, uint32_t* cnt, uint32_t* list, uint32_t* n_list, uint32_t id,
                                         uint32_t k, uint32_t len) {
  const uint32_t line = id >> 4, pos = id & 15u;
  uint32_t h = line_slot(line);
  for (int p = 0; p < kLineProbes; ++p) {
    if (p > 0) {
      h = (h + 1u) & (kLineEntries - 1u);
      k = keys[h];
    }
    if (k == kAggEmpty) {
      const uint32_t old = atomicCAS(keys + h, kAggEmpty, line);
      if (old == kAggEmpty) list[atomicAdd(n_list, 1u)] = h;
      k = old == kAggEmpty ? line : old;
    }
    if (k == line) {
      atomicAdd(cnt + h * kLineWords + (pos >> 1), len << (16u * (pos & 1u)));
      return true;
    }
  }
  return false;
}

// Per-tile record of the bricks that received counts (the batched plan's
// walks, whose finalize reads only the slots a brick received): region slot
// -> 64-bit brick mask in LDS, flushed with one global OR per region the
// tile reached.  Linear probing over kBrickEntries; a region finding no
// entry ORs its bit into the global mask at once.
constexpr uint32_t kBrickEntries = 256;
constexpr int kBrickProbes = 8;

__device__ __forceinline__ void brick_mark(const DevMap& m, uint32_t* keys, unsigned long long* masks, uint32_t voxel) {
  const uint32_t slot = voxel >> 15;
  const unsigned long long bit = 1ull << brick_of(voxel & (uint32_t)(kRegionVoxels - 1));
  uint32_t h = (slot * 0x9E3779B1u) >> 24;
  for (int p = 0; p < kBrickProbes; ++p) {
    if (agg_own(keys, h, slot, keys[h])) {
      atomicOr(masks + h, bit);
      return;
    }
    h = (h + 1u) & (kBrickEntries - 1u);
  }
  atomicOr(m.brick_mask + slot, bit);
}

// Clamp-add a wave's queued (update id, summed weight) pairs, one per lane.
__device__ __forceinline__ void drain_cas(const DevMap& m, const uint32_t* qid, const float* qv, uint32_t n,
                                          uint32_t lane) {
  __threadfence_block();  // the queue was written by other lanes of this wave
  if (lane < n) {
    const uint32_t id = qid[lane];
    cas_clamp_add(m.occ + (id >> 1), qv[lane] * ((id & 1u) ? m.l_hit : m.l_miss), m.l_min, m.l_max);
  }
}

// Per-ray data a tile keeps in LDS.
struct TileRays {
  long long q0[3];  // the scan origin, quantised: every ray of a tile starts there
  long long q1[3][kTileRays];
  uint8_t nseg[kTileRays];
  uint8_t trunc[kTileRays];
  uint16_t level_base[kMaxLevels + 1];
  uint16_t wave_count[kMaxLevels][kTileRays / 64];
  uint8_t item_ray[kMaxItems];
  uint32_t src[kTileRays];  // the ray's index within its scan (the walk order may differ)
  uint32_t max_seg;
};

// Per-thread results of the tile prologue; threads >= kTileRays hold no ray.
struct TileRay {
  Ray r;
  int st;           // kRayOk / kRayInvalid / kRayOriginOob
  bool inrange;     // the thread's tile slot holds a ray of the scan
  bool ok;          // ... which prepared successfully
  bool clipped;     // its walk leaves the map (the end voxel is outside)
  uint32_t voxels;  // voxels its walk visits inside the map
};

// Region staging done by the prologue.
enum : int { kStageNone = 0, kStageResolve = 1, kStageTouch = 2 };

// Walk position i of a scan of n rays that arrives as a column-major range
// image of R rays per column (ray = column * R + beam, R a multiple of 8):
// every full chunk of 32 columns is walked as R / 8 tiles of 8 beams by 32
// columns, consecutive walk positions (lanes) taking consecutive columns of
// one beam; a partial last chunk keeps the given order.  A bijection on
// each chunk.  A tile of the sensor's own order is 4 columns by 64 beams, a
// sliver 0.7 by 45 degrees on a 64-beam spinning lidar; the 32-by-8 patch is
// about square in angle and its rays share about twice as many voxels, so
// the tile's table flushes half as many global atomics and adjacent lanes
// more often step through the same voxel.
__device__ __forceinline__ uint32_t column_patch_index(uint32_t i, uint32_t n, uint32_t R) {
  const uint32_t chunk = 32u * R;
  const uint32_t base = i - i % chunk;
  if (n - base < chunk) return i;
  const uint32_t j = i - base, u = j >> 8, p = j & 255u;
  return base + (p & 31u) * R + u * 8u + (p >> 5);
}

// Prologue of a tile walk (every thread of the block must call it): threads
// 0..255 prepare rays tile0.. of the scan in walk order (perm[i] is the scan
// index of walk position i; null: column_patch_index with col_rays = R when
// it is nonzero, else the scan's own order), reject rays whose
// weight (when weights is not null) is negative or not finite, and fill the LDS
// ray table, the block stages the tile's regions in LDS (kStage), and the
// level-major item list is built: level j lists, in ray order, the rays with
// more than j segments.  Returns the number of items; tr.max_seg holds the
// level count, rw how the staged regions are looked up.
template <int kStage>
__device__ __forceinline__ uint32_t tile_prologue(const DevMap& m, TileRays& tr, RegionCache& rc, RegionWindow& rw,
                                                  const float* __restrict__ origin, const float* __restrict__ samples,
                                                  const float* __restrict__ weights,
                                                  const uint32_t* __restrict__ perm, uint32_t r0, uint32_t n,
                                                  uint32_t tile0, int K, uint32_t tag, uint32_t parity, TileRay& t,
                                                  uint32_t col_rays = 0) {
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const bool holds_ray = tid < (uint32_t)kTileRays;
  t.st = kRayInvalid;
  t.inrange = holds_ray && tile0 + tid < n;
  t.ok = false;
  t.clipped = false;
  t.voxels = 0;
  if (tid == 0) tr.max_seg = 0;
  bool bad_weight = false;
  if (t.inrange) {
    uint32_t src = tile0 + tid;
    if (perm)
      src = perm[src];
    else if (col_rays)
      src = column_patch_index(src, n, col_rays);
    tr.src[tid] = src;
    const size_t ray = (size_t)r0 + src;
    const float o[3] = {origin[0], origin[1], origin[2]};
    const float e[3] = {samples[3 * ray + 0], samples[3 * ray + 1], samples[3 * ray + 2]};
    t.st = prepare_ray(m, o, e, t.r);
    if (weights) {
      const float w = weights[ray];
      bad_weight = !(w >= 0.f) || !__builtin_isfinite(w);
      if (bad_weight) t.st = kRayInvalid;
    }
    t.ok = t.st == kRayOk;
  }
  if (__ballot(bad_weight) != 0ull && lane == 0)
    atomicOr(reinterpret_cast<int32_t*>(m.hdr + kHdrSticky), kStickyBadWeight);
  __syncthreads();
  uint32_t nseg = 0;
  if (holds_ray) {
    if (t.ok) {
      Walk w;
      const int32_t hi[3] = {m.kmax[0] - 1, m.kmax[1] - 1, m.kmax[2] - 1};
      walk_init(w, t.r.q0, t.r.q1, t.r.k0, t.r.k1, m.kmin, hi, m.F);
      nseg = seg_count(w, t.r.q0, t.r.q1, K);
      // the end voxel lies outside the map exactly when some axis is clipped
      t.clipped = w.clip != 0;
      t.voxels = walk_voxels(w, t.r.q0, t.r.q1, m.F);
      for (int a = 0; a < 3; ++a) {
        tr.q0[a] = t.r.q0[a];  // the same value from every ray
        tr.q1[a][tid] = t.r.q1[a];
      }
      tr.trunc[tid] = t.r.truncated ? 1 : 0;
    }
    tr.nseg[tid] = (uint8_t)nseg;
    const int32_t wmax = wave_max_i32((int32_t)nseg);
    if (lane == 0 && wmax > 0) atomicMax(&tr.max_seg, (uint32_t)wmax);
  }
  rw = RegionWindow{};
  if (kStage == kStageTouch) rw = stage_regions<true>(m, rc, t.ok, t.r, tag, parity);
  else if (kStage == kStageResolve) rw = stage_regions<false>(m, rc, t.ok, t.r, tag, parity);
  else __syncthreads();
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
        tr.item_ray[tr.wave_count[j][wave] + __popcll(below)] = (uint8_t)tid;
      }
    }
  }
  __syncthreads();
  return tr.level_base[levels];
}

// A 64-bit value every lane of the wave holds (the tile's quantised
// origin), moved to scalar registers so that it costs no vector registers
// in the loops.
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Item `it` of the list: its tile-local ray, major axis and segment state
// (and, when asked, its segment level).  False when the segment is empty
// (its ray left the map before it starts).
__device__ __forceinline__ bool tile_item(const DevMap& m, const TileRays& tr, uint32_t it, int K, SegState& s,
                                          uint32_t& ray_t, int& M, uint32_t* level_out = nullptr) {
  ray_t = tr.item_ray[it];
  const uint32_t levels = tr.max_seg;
  uint32_t level = 0;
  while (level + 1 < levels && tr.level_base[level + 1] <= it) ++level;
  if (level_out) *level_out = level;
  const int64_t q0[3] = {wave_uniform(tr.q0[0]), wave_uniform(tr.q0[1]), wave_uniform(tr.q0[2])};
  const int64_t q1[3] = {tr.q1[0][ray_t], tr.q1[1][ray_t], tr.q1[2][ray_t]};
  seg_init(s, q0, q1, m, (int)level, K);
  M = ray_major_axis(q0, q1);
  return !s.empty;
}

// Move past the current voxel (requires s.w.total > 0).  False when the
// segment ends; otherwise s.k is the next voxel and lidx (and, with kSlots,
// the staged region slot) follow it.
template <bool kSlots>
__device__ __forceinline__ bool tile_advance(const DevMap& m, const RegionCache& rc, const RegionWindow& rw,
                                             SegState& s, int M, int32_t& slot, uint32_t& lidx) {
  const int a = seg_advance(s, M);
  const bool moved = a >= 0;
  const int32_t sg = pick3(a, s.w.sg[0], s.w.sg[1], s.w.sg[2]);
  const int32_t kn = pick3(a, s.k[0], s.k[1], s.k[2]);
  const bool cross = moved && (kn & kRegionMask) == (sg > 0 ? 0 : kRegionMask);
  // the local index moves by sg along axis a: strides 1, 32, 1024 (wrapping
  // adds; a crossing recomputes it)
  lidx += (uint32_t)sg << (kRegionLog2 * (a & 3));
  if (cross) {
    if (kSlots) slot = staged_slot(m, rc, rw, s.k[0], s.k[1], s.k[2]);
    lidx = local_index(s.k[0], s.k[1], s.k[2]);
  }
  return moved;
}

// Block statistics of a tile walk (every thread must call it).  The walks
// flush them before their voxel loops, while the prepared rays are at hand
// (so that nothing of them stays live through the loop), counting every
// visit as an update and every untruncated ray ending in the map as a hit;
// the loops then count, per wave, the updates and hits they drop (regions
// the pool could not hold) and take them off with drop_tile_stats.
__device__ __forceinline__ void flush_tile_stats(const DevMap& m, const TileRay& t) {
  uint32_t vals[kStatCount];
  vals[kStatRays] = t.inrange ? 1u : 0u;
  vals[kStatInvalid] = (t.inrange && t.st == kRayInvalid) ? 1u : 0u;
  vals[kStatOriginOob] = (t.inrange && t.st == kRayOriginOob) ? 1u : 0u;
  vals[kStatTruncated] = (t.ok && t.r.truncated) ? 1u : 0u;
  vals[kStatClipped] = (t.ok && t.clipped) ? 1u : 0u;
  vals[kStatHits] = (t.ok && !t.clipped && !t.r.truncated) ? 1u : 0u;
  vals[kStatUpdates] = t.ok ? t.voxels : 0u;
  vals[kStatDropped] = 0u;
  flush_stats(m, vals);
}

// Take one wave's dropped updates (of which `hits` were hits) off the
// statistics (modulo-2^64 sums); called by every lane, wave-uniform counts.
__device__ __forceinline__ void drop_tile_stats(const DevMap& m, uint32_t drops, uint32_t hits) {
  if (drops != 0u && lane_id() == 0u) {
    atomicAdd(m.stats + kStatUpdates, 0ull - (unsigned long long)drops);
    atomicAdd(m.stats + kStatHits, 0ull - (unsigned long long)hits);
    atomicAdd(m.stats + kStatDropped, (unsigned long long)drops);
  }
}

// Occupancy walk of the tile of rays [tile0, tile0 + kTileRays) of a scan
// (n rays from r0): count or per-update sinks, or the trace outputs.  With
// kLayers the voxel mean and decay-rate layers the map holds are updated
// too (ohm_layers.h); with kBricks (count sink) the bricks that received
// counts are marked in m.brick_mask, and with kLineTable (unit-weight count
// sink) updates aggregate in the line table instead of the id table.
// col_rays: the scan's column layout for the walk order (tile_prologue).
// Every thread of the block must call it.
template <int kSink, bool kWeighted, bool kLayers = false, bool kBricks = false, bool kLineTable = false>
__device__ void walk_tile(const DevMap& m, const float* __restrict__ origin, const float* __restrict__ samples,
                          const float* __restrict__ weights, const uint32_t* __restrict__ perm, uint32_t r0,
                          uint32_t n, uint32_t tile0, int K,
                          uint32_t tag, uint32_t parity, uint32_t* __restrict__ ray_counts,
                          int32_t* __restrict__ ray_flags, const int64_t* __restrict__ ray_offsets,
                          int32_t* __restrict__ updates, uint32_t col_rays = 0) {
  constexpr bool kAccum = kSink == kSinkCount || kSink == kSinkCas;
  constexpr int kStage = kSink == kSinkCount ? kStageTouch : (kSink == kSinkCas ? kStageResolve : kStageNone);
  constexpr bool kLine = kLineTable && kSink == kSinkCount && !kWeighted;
  constexpr bool kAgg = kAccum && !kLine;
  // weighted count mode sums Q32.32 integers (order-independent, exact up to
  // the 2^-33 rounding of each weight) into the wide accumulators
  constexpr bool kWide = kSink == kSinkCount && kWeighted;
  using AggT = std::conditional_t<kWide, unsigned long long, float>;
  __shared__ TileRays tr;
  __shared__ RegionCache rc;
  __shared__ uint32_t agg_key[kAgg ? kAggSize : (kLine ? kLineEntries : 1)];
  __shared__ AggT agg_val[kAgg ? kAggSize : 1];
  static_assert(!kBricks || kSink == kSinkCount, "brick marks are for count walks");
  __shared__ uint32_t line_cnt[kLine ? kLineEntries * kLineWords : 1];
  __shared__ uint32_t line_list[kLine ? kLineEntries : 1];  // claimed entries, in claim order
  __shared__ uint32_t line_n;
  __shared__ uint32_t bk_key[kBricks ? kBrickEntries : 1];
  __shared__ unsigned long long bk_mask[kBricks ? kBrickEntries : 1];
  // per-update mode: table misses queued per wave, clamp-added 64 at a time
  // (a compare-and-swap waits for its reply; one wave-wide batch shares it)
  constexpr bool kQueue = kSink == kSinkCas;
  __shared__ uint32_t cq_id[kQueue ? 16 : 1][64];
  __shared__ float cq_v[kQueue ? 16 : 1][64];
  uint32_t cq_n = 0;  // wave-uniform
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = lane_id();
  if (kAgg)
    for (uint32_t h = tid; h < kAggSize; h += blockDim.x) {
      agg_key[h] = kAggEmpty;
      agg_val[h] = AggT(0);
    }
  if (kLine) {
    if (tid == 0) line_n = 0u;
    for (uint32_t h = tid; h < kLineEntries; h += blockDim.x) agg_key[h] = kAggEmpty;
    for (uint32_t h = tid; h < kLineEntries * kLineWords; h += blockDim.x) line_cnt[h] = 0u;
  }
  if (kBricks)
    for (uint32_t h = tid; h < kBrickEntries; h += blockDim.x) {
      bk_key[h] = kAggEmpty;
      bk_mask[h] = 0ull;
    }
  TileRay t;
  RegionWindow rw;
  const uint32_t items =
      tile_prologue<kStage>(m, tr, rc, rw, origin, samples, kWeighted ? weights : nullptr, perm, r0, n, tile0, K,
                            tag, parity, t, col_rays);

  if (kSink == kSinkTraceCount && t.inrange) {
    int32_t flags = 0;
    if (t.st == kRayInvalid) flags |= 8;
    if (t.st == kRayOriginOob) flags |= 16;
    if (t.ok) {
      flags |= t.r.truncated ? 1 : 0;
      flags |= t.clipped ? 2 : 0;
      flags |= (!t.r.truncated && !t.clipped) ? 4 : 0;
    }
    const size_t ray = (size_t)r0 + tr.src[tid];
    ray_counts[ray] = t.ok ? t.voxels : 0u;
    ray_flags[ray] = flags;
  }
  flush_tile_stats(m, t);
  uint32_t w_drop = 0, w_hit_drop = 0;  // this wave's dropped updates and hits (wave-uniform)

  // segment walks, one item per thread per round, with lane-run merging
  const uint32_t rounds = (items + blockDim.x - 1) / blockDim.x;
  for (uint32_t round = 0; round < rounds; ++round) {
    const uint32_t it = round * blockDim.x + tid;
    bool alive = it < items;
    uint32_t ray_t = 0;
    int M = 0;
    SegState s = {};
    float wt = 1.f;
    long long wq = 0;  // Q32.32 weight (wide accumulators)
    bool trunc = false;
    int32_t slot = -1;
    uint32_t lidx = 0;
    int64_t out_base = 0;
    DecayState dec;
    if (alive) {
      uint32_t level = 0;
      alive = tile_item(m, tr, it, K, s, ray_t, M, &level);
      if (kLayers && m.decay_len && alive) {
        const int64_t q0[3] = {wave_uniform(tr.q0[0]), wave_uniform(tr.q0[1]), wave_uniform(tr.q0[2])};
        const int64_t q1[3] = {tr.q1[0][ray_t], tr.q1[1][ray_t], tr.q1[2][ray_t]};
        decay_init(dec, m, q0, q1, s, (int)level, M);
      }
      trunc = tr.trunc[ray_t] != 0;
      const size_t ray = (size_t)r0 + tr.src[ray_t];
      if (kWeighted) wt = weights[ray];
      if (kWide) wq = llrint((double)wt * kQ32);
      if (kSink == kSinkTraceWrite) out_base = ray_offsets[ray] + s.pos;
      if (kAccum && alive) slot = staged_slot(m, rc, rw, s.k[0], s.k[1], s.k[2]);
      lidx = local_index(s.k[0], s.k[1], s.k[2]);
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
        AggT v;
        bool emit_here;
        if constexpr (!kWeighted) {
          v = (float)run.len;
          emit_here = has && run.head;
        } else if constexpr (kWide) {
          v = (unsigned long long)segmented_sum<long long>(has ? wq : 0ll, run.head, lane);
          emit_here = has && run.tail;
        } else {
          v = segmented_sum(has ? wt : 0.f, run.head, lane);
          emit_here = has && run.tail;
        }
        // read the table entry now, step the walk on, then use it: the LDS
        // read's latency overlaps the step's arithmetic
        const uint32_t k = emit_here ? agg_key[kLine ? line_slot(id >> 4) : agg_slot(id)] : 0u;
        // updates and hits were counted per ray before the loop; only drops
        // (region pool exhausted) are counted here, per wave
        const unsigned long long dropped = __ballot(alive && !has);
        if (dropped) {
          w_drop += (uint32_t)__popcll(dropped);
          w_hit_drop += (uint32_t)__popcll(dropped & __ballot(is_hit));
        }
        if constexpr (kLayers) {
          if (m.decay_len) {
            // the distance through this voxel, summed over the lanes' run
            const long long dq = alive ? decay_visit(dec, m, s) : 0ll;
            const long long sum = segmented_sum<long long>(has ? dq : 0ll, run.head, lane);
            if (has && run.tail && sum) atomicAdd(m.decay_len + (id >> 1), (unsigned long long)sum);
            if (has && is_hit && run.head) atomicAdd(m.decay_hits + (id >> 1), run.len);
          }
          if (m.mean && has && is_hit) {
            const int64_t q1[3] = {tr.q1[0][ray_t], tr.q1[1][ray_t], tr.q1[2][ray_t]};
            mean_sample<kSink == kSinkCount>(m, id >> 1, pack_codes(q1, m.F));
          }
        }
        if (alive) alive = !last && tile_advance<kAccum>(m, rc, rw, s, M, slot, lidx);
        bool miss_table;
        if constexpr (kLine) {
          miss_table = emit_here && !line_add(agg_key, line_cnt, line_list, &line_n, id, k, run.len);
        } else {
          miss_table = emit_here && !agg_finish(agg_key, agg_val, id, k, v);
        }
        if (kBricks && miss_table) brick_mark(m, bk_key, bk_mask, id >> 1);
        if constexpr (kWide) {
          if (miss_table) atomicAdd(reinterpret_cast<unsigned long long*>(m.acc) + id, v);
        } else if constexpr (kSink == kSinkCount) {
          if (miss_table) unsafeAtomicAdd(m.acc + id, v);
        } else {
          const unsigned long long qm = __ballot(miss_table);
          if (qm) {
            const uint32_t nq = (uint32_t)__popcll(qm);
            const uint32_t w = tid >> 6;
            if (cq_n + nq > 64u) {
              drain_cas(m, cq_id[w], cq_v[w], cq_n, lane);
              cq_n = 0;
            }
            if (miss_table) {
              const uint32_t rank = (uint32_t)__popcll(qm & ((1ull << lane) - 1ull));
              cq_id[w][cq_n + rank] = id;
              cq_v[w][cq_n + rank] = v;
            }
            cq_n += nq;
          }
        }
      } else {
        if (alive && kSink == kSinkTraceWrite) {
          int32_t* out = updates + 4 * (out_base + local);
          out[0] = s.k[0];
          out[1] = s.k[1];
          out[2] = s.k[2];
          out[3] = is_hit ? 1 : 0;
        }
        local += alive ? 1u : 0u;
        if (alive) alive = !last && tile_advance<kAccum>(m, rc, rw, s, M, slot, lidx);
      }
    }
  }
  if (kSink == kSinkTraceCount || kSink == kSinkTraceWrite) return;
  if (kQueue && cq_n) drain_cas(m, cq_id[tid >> 6], cq_v[tid >> 6], cq_n, lane);
  if (kLine) {
    __syncthreads();
    // 16 lanes per claimed line: one wave instruction reaches four
    // accumulator lines
    const uint32_t pos = tid & 15u;
    const uint32_t n_lines = line_n;
    for (uint32_t e = tid >> 4; e < n_lines; e += blockDim.x >> 4) {
      const uint32_t h = line_list[e];
      const uint32_t line = agg_key[h];
      const uint32_t c = (line_cnt[h * kLineWords + (pos >> 1)] >> (16u * (pos & 1u))) & 0xFFFFu;
      if (c) unsafeAtomicAdd(m.acc + (line << 4) + pos, (float)c);
      if (kBricks && pos == 0u) brick_mark(m, bk_key, bk_mask, line << 3);
    }
  }
  if (kAgg) {
    __syncthreads();
    if constexpr (kSink == kSinkCount) {
      for (uint32_t h = tid; h < kAggSize; h += blockDim.x) {
        const uint32_t k = agg_key[h];
        if constexpr (kWide) {
          if (k != kAggEmpty) atomicAdd(reinterpret_cast<unsigned long long*>(m.acc) + k, agg_val[h]);
        } else {
          if (k != kAggEmpty) unsafeAtomicAdd(m.acc + k, agg_val[h]);
        }
        if (kBricks && k != kAggEmpty) brick_mark(m, bk_key, bk_mask, k >> 1);
      }
    } else {
      // clamp-adds by compare-and-swap, four entries in flight per thread:
      // each round trip to memory is shared by the four
      constexpr int kFly = 4;
      for (uint32_t h0 = tid; h0 < kAggSize; h0 += kFly * blockDim.x) {
        uint32_t* u[kFly];
        float d[kFly];
        uint32_t old[kFly];
        bool pending[kFly];
#pragma unroll
        for (int i = 0; i < kFly; ++i) {
          const uint32_t h = h0 + (uint32_t)i * blockDim.x;
          const uint32_t k = h < kAggSize ? agg_key[h] : kAggEmpty;
          pending[i] = k != kAggEmpty;
          u[i] = reinterpret_cast<uint32_t*>(m.occ + (pending[i] ? (k >> 1) : 0u));
          d[i] = pending[i] ? agg_val[h] * ((k & 1u) ? m.l_hit : m.l_miss) : 0.f;
          old[i] = pending[i] ? __hip_atomic_load(u[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        }
        for (;;) {
          bool any = false;
#pragma unroll
          for (int i = 0; i < kFly; ++i) {
            if (!pending[i]) continue;
            const float nv = fminf(fmaxf(__uint_as_float(old[i]) + d[i], m.l_min), m.l_max);
            const uint32_t prev = atomicCAS(u[i], old[i], __float_as_uint(nv));
            pending[i] = prev != old[i];
            old[i] = prev;
            any = any || pending[i];
          }
          if (!any) break;
        }
      }
    }
  }
  if (kBricks) {
    __syncthreads();
    for (uint32_t h = tid; h < kBrickEntries; h += blockDim.x) {
      const uint32_t slot = bk_key[h];
      if (slot != kAggEmpty) atomicOr(m.brick_mask + slot, bk_mask[h]);
    }
  }
  drop_tile_stats(m, w_drop, w_hit_drop);
}

}  // namespace ohm
