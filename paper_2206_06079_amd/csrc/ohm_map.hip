// Map storage, region allocation, the ray-walk kernels for occupancy
// integration and the host side of the C ABI declared in include/ohm.h.
//
// Layout (all inside the caller's workspace, see layout()):
//   header      64 u32 words + 8 u64 statistics
//   table       int32 per region of the map's bounding box: slot or <0
//   stamp       u32 per slot: tag of the last count-mode scan that touched it
//   touched     u32 [2][capacity]: slots touched by the current / previous scan
//   occ         f32 [capacity][32^3] log-odds
//   acc         f32 [capacity][32^3][2] per-scan miss / hit weight (count mode)
//   ndt, mom    NDT-OM voxel statistics and per-scan sample moments (optional)
//   clampscan   u32 [capacity][32^3] (optional, adjoint)
//
// Per scan the library runs (paper Sec. III-B):
//   walk      one block per tile of 256 rays.  Prologue: the block walks
//             its rays over 32^3 regions, allocates missing regions and
//             stages their slots in LDS (count mode also lists them for
//             finalize).  Then the exact voxel walk, cut into segments of K
//             major-axis crossings (ohm_walk_seg.h), one update per voxel;
//             equal updates of adjacent lanes are merged before they are
//             applied.
//   finalize  (count mode) one clamp per touched voxel: l = clamp(l + t + u)
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

#include "ohm.h"
#include "ohm_device.h"
#include "ohm_host.h"
#include "ohm_regions.h"
#include "ohm_wave.h"
#include "ohm_order.h"
#include "ohm_walk_seg.h"

namespace ohm {

// ---------------------------------------------------------------------------
// small wave helpers
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// initialisation
// ---------------------------------------------------------------------------

__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// Segmented walk: one block per tile of 256 rays (perm: walk order or null).
template <int kSink, bool kWeighted, bool kLayers = false>
__global__ __launch_bounds__(1024) void walk_seg_kernel(DevMap m, const float* __restrict__ origins, uint32_t scan,
                                                        const float* __restrict__ samples,
                                                        const float* __restrict__ weights,
                                                        const uint32_t* __restrict__ perm, uint32_t r0, uint32_t n,
                                                        int K, uint32_t tag, uint32_t parity,
                                                        uint32_t* __restrict__ ray_counts,
                                                        int32_t* __restrict__ ray_flags,
                                                        const int64_t* __restrict__ ray_offsets,
                                                        int32_t* __restrict__ updates) {
  // per-update mode keeps the round-robin deal: its compare-and-swaps on the
  // voxels near the sensor retry more when neighbouring tiles share an XCD
  // (18.3 against 20.6 ms per headline step)
  const uint32_t tile = kSink == kSinkCas ? blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
  walk_tile<kSink, kWeighted, kLayers>(m, origins + 3 * (size_t)scan, samples, weights, perm, r0, n,
                                       tile * kTileRays, K, tag, parity, ray_counts, ray_flags, ray_offsets,
                                       updates);
}

// Direction ordering of one scan (ohm_order.h): count, prefix, place.
__global__ __launch_bounds__(256) void scan_order_count_kernel(const float* __restrict__ origin,
                                                               const float* __restrict__ samples, uint32_t n,
                                                               uint32_t* __restrict__ hist) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) order_count(origin, samples, n, kOrderStripRaysScan, i, hist);
}

__global__ __launch_bounds__(kOrderElevationBins) void scan_order_strip_kernel(uint32_t* __restrict__ hist,
                                                                              uint32_t* __restrict__ sums) {
  order_strip_prefix(hist + (size_t)blockIdx.x * kOrderElevationBins, sums + blockIdx.x);
}

__global__ __launch_bounds__(kOrderMaxStrips) void scan_order_sums_kernel(uint32_t* __restrict__ sums,
                                                                          uint32_t strips) {
  order_scan_prefix(sums, strips);
}

__global__ __launch_bounds__(256) void scan_order_place_kernel(const float* __restrict__ origin,
                                                               const float* __restrict__ samples, uint32_t n,
                                                               uint32_t* __restrict__ hist,
                                                               const uint32_t* __restrict__ sums,
                                                               uint32_t* __restrict__ perm) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) order_place(origin, samples, n, kOrderStripRaysScan, i, hist, sums, perm);
}

// ---------------------------------------------------------------------------
// per-scan finalize (count mode)
// ---------------------------------------------------------------------------

constexpr int kFinalChunk = 1024;  // voxels per work unit
constexpr int kFinalUnits = kRegionVoxels / kFinalChunk;

// Count mode: the per-scan parts of the optional layers for one unit of
// kFinalChunk voxels from `base` (the voxel mean merges its scans' samples;
// the decay-rate layer needs nothing here).  Every thread of the block calls it.
__device__ __forceinline__ void finalize_layers(const DevMap& m, size_t base) {
  if (!m.mean) return;
  for (int v = threadIdx.x; v < kFinalChunk; v += blockDim.x) mean_finalize_voxel(m, base + v, mean_slot_words(m));
}

// Applies l <- clamp((l + H l_hit) + M l_miss) to every voxel of the touched
// regions (kWide: from Q32.32 weight sums, in fp64).  With `apply` = 0 only
// clears the accumulators.  Clears the accumulators when `clear`, and resets
// the other parity's touched counter for the next scan.
template <bool kWide>
__global__ __launch_bounds__(256) void finalize_kernel(DevMap m, uint32_t parity, int apply, int clear,
                                                       uint32_t scan_tag) {
  const uint32_t count = __hip_atomic_load(m.hdr + kHdrTouched0 + parity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t units = count * kFinalUnits;
  if constexpr (kWide) {
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
      const uint32_t slot = m.touched[(size_t)parity * m.capacity + u / kFinalUnits];
      const size_t base = (size_t)slot * kRegionVoxels + (size_t)(u % kFinalUnits) * kFinalChunk;
      if (apply) finalize_layers(m, base);
      for (int v = threadIdx.x; v < kFinalChunk; v += blockDim.x) {
        const size_t vi = base + v;
        longlong2* ap = reinterpret_cast<longlong2*>(m.acc) + vi;  // (miss, hit)
        const longlong2 a = *ap;
        if (a.x == 0 && a.y == 0) continue;
        if (apply) m.occ[vi] = apply_wide(m, m.occ[vi], a.x, a.y, vi, scan_tag);
        if (clear) *ap = make_longlong2(0, 0);
      }
    }
  } else {
  for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
    const uint32_t slot = m.touched[(size_t)parity * m.capacity + u / kFinalUnits];
    const size_t base = (size_t)slot * kRegionVoxels + (size_t)(u % kFinalUnits) * kFinalChunk;
    if (apply) finalize_layers(m, base);
    for (int v = threadIdx.x * 2; v < kFinalChunk; v += blockDim.x * 2) {
      float4* ap = reinterpret_cast<float4*>(m.acc + 2 * (base + v));
      float4 a = *ap;  // (miss0, hit0, miss1, hit1)
      if (a.x == 0.f && a.y == 0.f && a.z == 0.f && a.w == 0.f) continue;
      if (apply) {
        float2* lp = reinterpret_cast<float2*>(m.occ + base + v);
        float2 l = *lp;
        float lv[2] = {l.x, l.y};
        const float mw[2] = {a.x, a.z};
        const float hw[2] = {a.y, a.w};
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (mw[j] == 0.f && hw[j] == 0.f) continue;
          const float t = __fmul_rn(hw[j], m.l_hit);
          const float uu = __fmul_rn(mw[j], m.l_miss);
          float s = __fadd_rn(lv[j], t);
          s = __fadd_rn(s, uu);
          if (m.clampscan && (s < m.l_min || s > m.l_max)) m.clampscan[base + v + j] = scan_tag;
          lv[j] = fminf(fmaxf(s, m.l_min), m.l_max);
        }
        *lp = make_float2(lv[0], lv[1]);
      }
      if (clear) *ap = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(m.hdr + kHdrTouched0 + (parity ^ 1u), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grouped scans (OHM_LAYER_SCAN_GROUPS): up to G (the map's slots) consecutive scans
// of a call walk in one launch, scan j of the group into accumulator slot j
// under one tag, and group_finalize_kernel applies them per voxel in scan
// order.  More tiles per launch keep the whole device busy: one scan's
// tiles alone leave most compute units idle behind its longest tiles.
struct GroupArgs {
  uint32_t count;                  // scans in the group
  uint32_t col_rays;               // column layout of the scans (column_patch_index), 0: none
  uint32_t scan[kMaxGroupSlots];      // scan index within the call
  uint32_t r0[kMaxGroupSlots];        // first ray
  uint32_t n[kMaxGroupSlots];         // rays
  uint32_t tile_end[kMaxGroupSlots];  // exclusive end of the scan's blocks
};

// Tiles of up to 512 threads of the plain walk run three blocks per CU (six
// waves per SIMD: the kernel is held to 80 VGPRs, which it fits without
// spills since the tile statistics are flushed before the voxel loop, and
// its 52 KB of LDS fit three times); the extra waves hide more of the voxel
// loop's latency.  With the layers (kLayers) the loop holds too
// much for 80 VGPRs, and 1024-thread tiles (kWideTile) fit one block per
// CU: both keep the 128-VGPR budget.
template <bool kWeighted, bool kLayers = false, bool kWideTile = false>
__global__ __launch_bounds__((kWideTile || kLayers) ? 1024 : 512, (kWideTile || kLayers) ? 1 : 6) void walk_group_kernel(
    DevMap m, const float* __restrict__ origins,
                                                          const float* __restrict__ samples,
                                                          const float* __restrict__ weights, GroupArgs g, int K,
                                                          uint32_t tag, uint32_t parity) {
  const uint32_t lb = xcd_tile(blockIdx.x, gridDim.x);  // the launch's tile index
  uint32_t j = 0;  // the block's scan (uniform over the block)
  while (j + 1 < g.count && lb >= g.tile_end[j]) ++j;
  const uint32_t tile = lb - (j ? g.tile_end[j - 1] : 0u);
  DevMap mj = m;
  mj.acc += (size_t)j * acc_slot_floats(m, kWeighted);
  if (kLayers && mj.mean) {
    mj.mean_acc += (size_t)j * mean_slot_words(m);
    mj.mean_slot = j;
  }
  walk_tile<kSinkCount, kWeighted, kLayers>(mj, origins + 3 * (size_t)g.scan[j], samples, weights, nullptr, g.r0[j], g.n[j],
                                   tile * kTileRays, K, tag, parity, nullptr, nullptr, nullptr, nullptr, g.col_rays);
}

constexpr int kGroupBatch = 8;  // accumulator slots loaded together by a group finalize

// Apply the group's g scans in order to every voxel of the regions the group
// touched: l = clamp((l + H_j l_hit) + M_j l_miss) for j = 0..g-1, recording
// the clamp scan (scan_tag0 + j), and clear the slots except slot `keep`
// (the call's last scan, whose counts stay readable; keep >= g keeps none).
// kWide: the slots hold Q32.32 weight sums (weighted scans), applied in fp64.
template <bool kWide>
__global__ __launch_bounds__(256) void group_finalize_kernel(DevMap m, uint32_t parity, uint32_t g,
                                                             uint32_t scan_tag0, uint32_t keep) {
  const uint32_t count = __hip_atomic_load(m.hdr + kHdrTouched0 + parity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t units = count * kFinalUnits;
  const size_t stride = (size_t)m.capacity * kRegionVoxels;  // accumulator pairs per slot
  if constexpr (kWide) {
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
      const uint32_t slot = m.touched[(size_t)parity * m.capacity + u / kFinalUnits];
      const size_t base = (size_t)slot * kRegionVoxels + (size_t)(u % kFinalUnits) * kFinalChunk;
      finalize_layers(m, base);
      for (int v = threadIdx.x; v < kFinalChunk; v += blockDim.x) {
        const size_t vi = base + v;
        longlong2* const a0 = reinterpret_cast<longlong2*>(m.acc) + vi;
        float l = m.occ[vi];
        bool any = false;
        for (uint32_t j0 = 0; j0 < g; j0 += kGroupBatch) {
          longlong2 a[kGroupBatch];
#pragma unroll
          for (int q = 0; q < kGroupBatch; ++q) a[q] = j0 + q < g ? a0[(j0 + q) * stride] : make_longlong2(0, 0);
#pragma unroll
          for (int q = 0; q < kGroupBatch; ++q) {
            if (a[q].x == 0 && a[q].y == 0) continue;
            const uint32_t j = j0 + q;
            l = apply_wide(m, l, a[q].x, a[q].y, vi, scan_tag0 + j);
            if (j != keep) a0[j * stride] = make_longlong2(0, 0);
            any = true;
          }
        }
        if (any) m.occ[vi] = l;
      }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
      __hip_atomic_store(m.hdr + kHdrTouched0 + (parity ^ 1u), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
    const uint32_t slot = m.touched[(size_t)parity * m.capacity + u / kFinalUnits];
    const size_t base = (size_t)slot * kRegionVoxels + (size_t)(u % kFinalUnits) * kFinalChunk;
    finalize_layers(m, base);
    for (int v = threadIdx.x; v < kFinalChunk; v += blockDim.x) {
      const size_t vi = base + v;
      float2* const a0 = reinterpret_cast<float2*>(m.acc) + vi;
      float l = m.occ[vi];
      bool any = false;
      // slots are loaded kGroupBatch at a time, all before the batch's
      // clearing stores, so the loads overlap instead of waiting on each other
      for (uint32_t j0 = 0; j0 < g; j0 += kGroupBatch) {
        float2 a[kGroupBatch];
#pragma unroll
        for (int q = 0; q < kGroupBatch; ++q) a[q] = j0 + q < g ? a0[(j0 + q) * stride] : make_float2(0.f, 0.f);
#pragma unroll
        for (int q = 0; q < kGroupBatch; ++q) {
          if (a[q].x == 0.f && a[q].y == 0.f) continue;
          const uint32_t j = j0 + q;
          const float t = __fmul_rn(a[q].y, m.l_hit);
          const float uu = __fmul_rn(a[q].x, m.l_miss);
          float sum = __fadd_rn(l, t);
          sum = __fadd_rn(sum, uu);
          if (m.clampscan && (sum < m.l_min || sum > m.l_max)) m.clampscan[vi] = scan_tag0 + j;
          l = fminf(fmaxf(sum, m.l_min), m.l_max);
          if (j != keep) a0[j * stride] = make_float2(0.f, 0.f);
          any = true;
        }
      }
      if (any) m.occ[vi] = l;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(m.hdr + kHdrTouched0 + (parity ^ 1u), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// dense read-back
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void read_dense_kernel(DevMap m, int what, int wide, int32_t bx, int32_t by,
                                                         int32_t bz, int32_t dx, int32_t dy, int32_t dz, void* out) {
  const size_t nvox = (size_t)dx * dy * dz;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox) return;
  const int32_t x = bx + (int32_t)(i % dx);
  const int32_t y = by + (int32_t)((i / dx) % dy);
  const int32_t z = bz + (int32_t)(i / ((size_t)dx * dy));
  int32_t slot = -1;
  if (x >= m.kmin[0] && x < m.kmax[0] && y >= m.kmin[1] && y < m.kmax[1] && z >= m.kmin[2] && z < m.kmax[2])
    slot = lookup_slot(m, x, y, z);
  const size_t v = slot >= 0 ? (size_t)slot * kRegionVoxels + local_index(x, y, z) : 0;
  switch (what) {
    case OHM_READ_OCC:
      static_cast<float*>(out)[i] = slot >= 0 ? m.occ[v] : m.l_init;
      break;
    case OHM_READ_HITS:
    case OHM_READ_MISSES: {
      const int kind = what == OHM_READ_HITS ? 1 : 0;
      float c = 0.f;
      if (slot >= 0)
        c = wide ? (float)((double)reinterpret_cast<const long long*>(m.acc)[2 * v + kind] * kInvQ32)
                 : m.acc[2 * v + kind];
      static_cast<float*>(out)[i] = c;
      break;
    }
    case OHM_READ_NDT_COUNT:
      static_cast<uint32_t*>(out)[i] = slot >= 0 ? m.ndt[v].n : 0u;
      break;
    case OHM_READ_NDT_MEAN:
      for (int c = 0; c < 3; ++c) static_cast<float*>(out)[3 * i + c] = slot >= 0 ? m.ndt[v].mean[c] : 0.f;
      break;
    case OHM_READ_NDT_COV:
      for (int c = 0; c < 6; ++c) static_cast<float*>(out)[6 * i + c] = slot >= 0 ? m.ndt[v].cov[c] : 0.f;
      break;
    case OHM_READ_CLAMP_SCAN:
      static_cast<uint32_t*>(out)[i] = slot >= 0 ? m.clampscan[v] : 0u;
      break;
    case OHM_READ_MEAN_PACKED:
      static_cast<uint32_t*>(out)[i] = slot >= 0 ? (uint32_t)m.mean[v] : 0u;
      break;
    case OHM_READ_MEAN_COUNT:
      static_cast<uint32_t*>(out)[i] = slot >= 0 ? (uint32_t)(m.mean[v] >> 32) : 0u;
      break;
    case OHM_READ_MEAN: {
      // centre of the code cell, metres from the voxel centre (0 where empty)
      const unsigned long long w = slot >= 0 ? m.mean[v] : 0ull;
      for (int c = 0; c < 3; ++c) {
        const uint32_t code = ((uint32_t)w >> (10 * c)) & 1023u;
        static_cast<float*>(out)[3 * i + c] =
            (w >> 32) ? (float)((((double)code + 0.5) / 1024.0 - 0.5) * m.voxel_size) : 0.f;
      }
      break;
    }
    case OHM_READ_DECAY_LENGTH:
      static_cast<float*>(out)[i] = slot >= 0 ? (float)((double)m.decay_len[v] * kInvQ32) : 0.f;
      break;
    case OHM_READ_DECAY_HITS:
      static_cast<uint32_t*>(out)[i] = slot >= 0 ? m.decay_hits[v] : 0u;
      break;
    case OHM_READ_DECAY_RATE: {
      const double len = slot >= 0 ? (double)m.decay_len[v] * kInvQ32 : 0.0;
      static_cast<float*>(out)[i] = len > 0.0 ? (float)((double)m.decay_hits[v] / len) : 0.f;
      break;
    }
    case OHM_READ_TM_MISSES:
      static_cast<uint32_t*>(out)[i] = slot >= 0 ? m.tm[v].miss : 0u;
      break;
    case OHM_READ_TM_PERMEABILITY: {
      const double h = slot >= 0 ? (double)m.ndt[v].n : 0.0;
      const double hm = h + (slot >= 0 ? (double)m.tm[v].miss : 0.0);
      static_cast<float*>(out)[i] = hm > 0.0 ? (float)(h / hm) : 0.f;
      break;
    }
    case OHM_READ_INTENSITY_MEAN:
      static_cast<float*>(out)[i] = slot >= 0 ? m.tm[v].imean : 0.f;
      break;
    case OHM_READ_INTENSITY_VAR:
      static_cast<float*>(out)[i] = slot >= 0 ? m.tm[v].ivar : 0.f;
      break;
    case OHM_READ_TSDF_DISTANCE:
      static_cast<float*>(out)[i] = slot >= 0 ? __uint_as_float((uint32_t)m.tsdf[v]) : 0.f;
      break;
    case OHM_READ_TSDF_WEIGHT:
      static_cast<float*>(out)[i] = slot >= 0 ? __uint_as_float((uint32_t)(m.tsdf[v] >> 32)) : 0.f;
      break;
    default:
      break;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
  size_t hdr, stats, table, stamp, touched, occ, acc, ndt, nacc, mom, clampscan, mean, mean_acc, mean_mask,
      decay_len, decay_hits, tm, tm_mom, tsdf, tsdf_acc, ndt_ready, nsamp, total;
  int32_t rlo[3], rdim[3];
  size_t regions;
};

ohm_status validate_params(const ohm_params* p) {
  if (!p) return OHM_E_INVALID_ARG;
  if (!(p->voxel_size > 0.0) || !isfinite(p->voxel_size)) return OHM_E_INVALID_ARG;
  if (p->region_log2 != kRegionLog2) return OHM_E_UNSUPPORTED;
  if (p->fixed_bits < 8 || p->fixed_bits > 20) return OHM_E_INVALID_ARG;
  const int64_t kmax_abs = int64_t(1) << (45 - p->fixed_bits);
  for (int a = 0; a < 3; ++a) {
    if (!isfinite(p->map_origin[a])) return OHM_E_INVALID_ARG;
    if (p->key_min[a] >= p->key_max[a]) return OHM_E_INVALID_ARG;
    if (p->key_min[a] < -kmax_abs || p->key_max[a] > kmax_abs) return OHM_E_INVALID_ARG;
  }
  if (!(p->l_hit >= 0.f) || !(p->l_miss <= 0.f) || !isfinite(p->l_hit) || !isfinite(p->l_miss))
    return OHM_E_INVALID_ARG;
  if (!(p->l_min < p->l_max) || !isfinite(p->l_min) || !isfinite(p->l_max)) return OHM_E_INVALID_ARG;
  if (!(p->l_init >= p->l_min && p->l_init <= p->l_max)) return OHM_E_INVALID_ARG;
  if (isnan(p->max_range)) return OHM_E_INVALID_ARG;
  if (p->mode != OHM_MODE_PER_UPDATE && p->mode != OHM_MODE_COUNT_CLAMP) return OHM_E_INVALID_ARG;
  if (!(p->sensor_noise > 0.f) || !isfinite(p->sensor_noise)) return OHM_E_INVALID_ARG;
  if (!(p->adaptation_rate >= 0.f && p->adaptation_rate <= 1.f)) return OHM_E_INVALID_ARG;
  if (p->ndt_min_samples < 2) return OHM_E_INVALID_ARG;
  if (isnan(p->ndt_clear_below)) return OHM_E_INVALID_ARG;
  if (!(p->ndt_tm_gate > 0.0) || !isfinite(p->ndt_tm_gate)) return OHM_E_INVALID_ARG;
  if (!(p->tsdf_truncation > 0.0) || !isfinite(p->tsdf_truncation)) return OHM_E_INVALID_ARG;
  if (!(p->tsdf_max_weight >= 1.0) || !isfinite(p->tsdf_max_weight)) return OHM_E_INVALID_ARG;
  return OHM_OK;
}

ohm_status compute_layout(const ohm_params* p, uint32_t capacity, uint32_t layers, Layout* L) {
  ohm_status s = validate_params(p);
  if (s != OHM_OK) return s;
  if (capacity == 0 || capacity > kMaxCapacity) return OHM_E_INVALID_ARG;
  if (layers & ~(uint32_t)(OHM_LAYER_OCC | OHM_LAYER_NDT | OHM_LAYER_ADJOINT | OHM_LAYER_SCAN_GROUPS |
                           OHM_LAYER_MEAN | OHM_LAYER_DECAY | OHM_LAYER_NDT_TM | OHM_LAYER_TSDF |
                           OHM_SCAN_GROUP_SLOTS(0xff)))
    return OHM_E_INVALID_ARG;
  if ((layers & OHM_LAYER_NDT_TM) && !(layers & OHM_LAYER_NDT)) return OHM_E_INVALID_ARG;
  const uint32_t slots = group_slots_of(layers);
  if (slots == 0) return OHM_E_INVALID_ARG;
  // the NDT walk updates none of the occupancy walk's optional layers
  if ((layers & OHM_LAYER_NDT) && (layers & (OHM_LAYER_MEAN | OHM_LAYER_DECAY))) return OHM_E_UNSUPPORTED;
  size_t regions = 1;
  for (int a = 0; a < 3; ++a) {
    L->rlo[a] = p->key_min[a] >> kRegionLog2;
    int32_t rhi = (p->key_max[a] - 1) >> kRegionLog2;
    L->rdim[a] = rhi - L->rlo[a] + 1;
    regions *= (size_t)L->rdim[a];
  }
  if (regions > (size_t(1) << 28)) return OHM_E_UNSUPPORTED;
  L->regions = regions;
  const size_t V = kRegionVoxels;
  size_t off = 0;
  L->hdr = off;
  off = align_up(off + kHdrWords * sizeof(uint32_t));
  L->stats = off;
  off = align_up(off + 16 * sizeof(unsigned long long));
  L->table = off;
  off = align_up(off + regions * sizeof(int32_t));
  L->stamp = off;
  off = align_up(off + (size_t)capacity * sizeof(uint32_t));
  L->touched = off;
  off = align_up(off + 2 * (size_t)capacity * sizeof(uint32_t));
  L->occ = off;
  off = align_up(off + (size_t)capacity * V * sizeof(float));
  L->acc = off;
  // at least two f32 slots: a weighted scan's wide (int64) slot spans two
  off = align_up(off + (size_t)capacity * V * 2 * sizeof(float) * (slots < 2 ? 2 : slots));
  L->ndt = L->nacc = L->mom = L->clampscan = L->ndt_ready = L->nsamp = 0;
  if (layers & OHM_LAYER_NDT) {
    L->ndt = off;
    off = align_up(off + (size_t)capacity * V * sizeof(NdtVoxel));
    L->ndt_ready = off;
    off = align_up(off + (size_t)capacity * (V / 32) * sizeof(uint32_t));
    L->nacc = off;
    off = align_up(off + (size_t)capacity * V * kNaccWords * sizeof(long long));
    L->nsamp = off;
    off = align_up(off + (size_t)capacity * V * sizeof(uint32_t));
    L->mom = off;
    off = align_up(off + (size_t)capacity * V * kMomWords * sizeof(double));
  }
  if (layers & OHM_LAYER_ADJOINT) {
    L->clampscan = off;
    off = align_up(off + (size_t)capacity * V * sizeof(uint32_t));
  }
  L->mean = L->mean_acc = L->mean_mask = L->decay_len = L->decay_hits = 0;
  if (layers & OHM_LAYER_MEAN) {
    L->mean = off;
    off = align_up(off + (size_t)capacity * V * sizeof(unsigned long long));
    L->mean_acc = off;  // one slot of per-scan sums per accumulator slot
    off = align_up(off + (size_t)capacity * V * 2 * sizeof(unsigned long long) * slots);
    L->mean_mask = off;
    off = align_up(off + (size_t)capacity * V * sizeof(unsigned long long));
  }
  if (layers & OHM_LAYER_DECAY) {
    L->decay_len = off;
    off = align_up(off + (size_t)capacity * V * sizeof(unsigned long long));
    L->decay_hits = off;
    off = align_up(off + (size_t)capacity * V * sizeof(uint32_t));
  }
  L->tm = L->tm_mom = L->tsdf = L->tsdf_acc = 0;
  if (layers & OHM_LAYER_NDT_TM) {
    L->tm = off;
    off = align_up(off + (size_t)capacity * V * sizeof(TmVoxel));
    L->tm_mom = off;
    off = align_up(off + (size_t)capacity * V * 2 * sizeof(double));
  }
  if (layers & OHM_LAYER_TSDF) {
    L->tsdf = off;
    off = align_up(off + (size_t)capacity * V * sizeof(unsigned long long));
    L->tsdf_acc = off;
    off = align_up(off + (size_t)capacity * V * 2 * sizeof(long long));
  }
  L->total = off;
  return OHM_OK;
}

void fill_params(DevMap& dm, const ohm_params* p) {
  for (int a = 0; a < 3; ++a) {
    dm.origin[a] = p->map_origin[a];
    dm.kmin[a] = p->key_min[a];
    dm.kmax[a] = p->key_max[a];
  }
  dm.scale = ldexp(1.0, p->fixed_bits) / p->voxel_size;
  dm.voxel_size = p->voxel_size;
  dm.max_range = p->max_range;
  dm.max_range2 = p->max_range * p->max_range;
  dm.F = p->fixed_bits;
  dm.l_hit = p->l_hit;
  dm.l_miss = p->l_miss;
  dm.l_min = p->l_min;
  dm.l_max = p->l_max;
  dm.l_init = p->l_init;
  dm.sensor_noise = p->sensor_noise;
  dm.adaptation_rate = p->adaptation_rate;
  dm.ndt_min_samples = p->ndt_min_samples;
  dm.ndt_clear_below = p->ndt_clear_below;
  dm.tm_gate = p->ndt_tm_gate;
  dm.tsdf_tau = p->tsdf_truncation;
  dm.tsdf_wmax = p->tsdf_max_weight;
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

ohm_status last_hip_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? OHM_OK : OHM_E_HIP;
}

void launch_fill(void* p, size_t bytes, uint32_t v, hipStream_t st) {
  size_t n = bytes / sizeof(uint32_t);
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<uint32_t*>(p), n, v);
}

}  // namespace

size_t order_scratch_bytes(uint32_t max_rays) {
  return align_up((size_t)order_bins(max_rays, kOrderStripRaysScan) * sizeof(uint32_t)) +
         align_up((size_t)kOrderMaxStrips * sizeof(uint32_t)) + align_up((size_t)max_rays * sizeof(uint32_t));
}

OrderScratch order_scratch_at(void* base, uint32_t max_rays) {
  char* b = static_cast<char*>(base);
  const size_t hist_bytes = align_up((size_t)order_bins(max_rays, kOrderStripRaysScan) * sizeof(uint32_t));
  const size_t sums_bytes = align_up((size_t)kOrderMaxStrips * sizeof(uint32_t));
  return OrderScratch{reinterpret_cast<uint32_t*>(b), reinterpret_cast<uint32_t*>(b + hist_bytes),
                      reinterpret_cast<uint32_t*>(b + hist_bytes + sums_bytes), max_rays};
}

ohm_status map_initialise(ohm_map_s* map, hipStream_t st) {
  const DevMap& m = map->dm;
  const size_t V = kRegionVoxels;
  launch_fill(m.hdr, kHdrWords * sizeof(uint32_t), 0u, st);
  launch_fill(m.stats, 16 * sizeof(unsigned long long), 0u, st);
  launch_fill(m.table, map->regions * sizeof(int32_t), (uint32_t)kSlotEmpty, st);
  launch_fill(m.stamp, (size_t)m.capacity * sizeof(uint32_t), 0u, st);
  uint32_t init_bits;
  memcpy(&init_bits, &m.l_init, sizeof(init_bits));
  launch_fill(m.occ, (size_t)m.capacity * V * sizeof(float), init_bits, st);
  launch_fill(m.acc, (size_t)m.capacity * V * 2 * sizeof(float) * (map->group_slots < 2 ? 2 : map->group_slots),
              0u, st);
  if (m.ndt) {
    launch_fill(m.ndt, (size_t)m.capacity * V * sizeof(NdtVoxel), 0u, st);
    launch_fill(m.nacc, (size_t)m.capacity * V * kNaccWords * sizeof(long long), 0u, st);
    launch_fill(m.nsamp, (size_t)m.capacity * V * sizeof(uint32_t), 0u, st);
    launch_fill(m.mom, (size_t)m.capacity * V * kMomWords * sizeof(double), 0u, st);
    launch_fill(m.ndt_ready, (size_t)m.capacity * (V / 32) * sizeof(uint32_t), 0u, st);
  }
  if (m.clampscan) launch_fill(m.clampscan, (size_t)m.capacity * V * sizeof(uint32_t), 0u, st);
  if (m.mean) {
    launch_fill(m.mean, (size_t)m.capacity * V * sizeof(unsigned long long), 0u, st);
    launch_fill(m.mean_acc, (size_t)m.capacity * V * 2 * sizeof(unsigned long long) * map->group_slots, 0u, st);
    launch_fill(m.mean_mask, (size_t)m.capacity * V * sizeof(unsigned long long), 0u, st);
  }
  if (m.decay_len) {
    launch_fill(m.decay_len, (size_t)m.capacity * V * sizeof(unsigned long long), 0u, st);
    launch_fill(m.decay_hits, (size_t)m.capacity * V * sizeof(uint32_t), 0u, st);
  }
  if (m.tm) {
    launch_fill(m.tm, (size_t)m.capacity * V * sizeof(TmVoxel), 0u, st);
    launch_fill(m.tm_mom, (size_t)m.capacity * V * 2 * sizeof(double), 0u, st);
  }
  if (m.tsdf) {
    launch_fill(m.tsdf, (size_t)m.capacity * V * sizeof(unsigned long long), 0u, st);
    launch_fill(m.tsdf_acc, (size_t)m.capacity * V * 2 * sizeof(long long), 0u, st);
  }
  map->count_batches = 0;
  map->acc_dirty = false;
  map->ndt_ready_stale = false;
  map->kept_slot = 0;
  map->kept_wide = false;
  map->scans_done = 0;
  map->batched = false;
  return last_hip_status();
}

ohm_status check_scans(ohm_map map, const float* d_origins, const float* d_samples, const uint32_t* h_offsets,
                       uint32_t n_scans) {
  if (!map) return OHM_E_INVALID_ARG;
  if (n_scans == 0) return OHM_OK;
  if (!h_offsets || !d_origins) return OHM_E_INVALID_ARG;
  for (uint32_t s = 0; s < n_scans; ++s)
    if (h_offsets[s + 1] < h_offsets[s]) return OHM_E_INVALID_ARG;
  if (h_offsets[n_scans] > h_offsets[0] && !d_samples) return OHM_E_INVALID_ARG;
  return OHM_OK;
}

namespace {
hipEvent_t take_event(ohm_map_s* map) {
  if (map->events_used == map->event_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    map->event_pool.push_back(e);
  }
  return map->event_pool[map->events_used++];
}
}  // namespace

ProfScope::ProfScope(ohm_map_s* map, int kind, hipStream_t st, bool on)
    : map_(map), st_(st), kind_(kind), stop_(nullptr) {
  if (!on || !map->profiling) return;
  hipEvent_t start = take_event(map);
  stop_ = take_event(map);
  if (!start || !stop_) {
    stop_ = nullptr;
    return;
  }
  if (hipEventRecord(start, st) != hipSuccess) {
    stop_ = nullptr;
    return;
  }
  map->timed.push_back({kind, start, stop_});
}

ProfScope::~ProfScope() {
  if (stop_ && hipEventRecord(stop_, st_) != hipSuccess) map_->timed.back().stop = nullptr;
  (void)kind_;
}

// The map's device view with `acc` at the slot that holds the last
// count-mode scan's counts.
DevMap kept_counts(const ohm_map_s* map) {
  DevMap m = map->dm;
  m.acc += (size_t)map->kept_slot * acc_slot_floats(m, map->kept_wide);
  return m;
}

// Lazy clear of the previous count-mode scan's accumulators.
void clear_pending(ohm_map_s* map, hipStream_t st, bool prof) {
  if (!map->acc_dirty) return;
  ProfScope ps(map, OHM_KERNEL_FINALIZE, st, prof);
  if (map->kept_wide)
    hipLaunchKernelGGL(finalize_kernel<true>, dim3(kFinalizeBlocks), dim3(256), 0, st, kept_counts(map),
                       map->last_parity, 0, 1, 0u);
  else
    hipLaunchKernelGGL(finalize_kernel<false>, dim3(kFinalizeBlocks), dim3(256), 0, st, kept_counts(map),
                       map->last_parity, 0, 1, 0u);
  map->acc_dirty = false;
  map->kept_slot = 0;
  map->kept_wide = false;
}

// Walk launches with or without the optional-layer hooks (the hooks cost
// registers and instructions that maps without those layers do not pay).
template <int kSink, bool kWeighted>
void launch_walk_seg(const ohm_map_s* map, bool layers, dim3 grid, dim3 block, hipStream_t st, const float* origins,
                     uint32_t scan, const float* samples, const float* weights, const uint32_t* perm, uint32_t r0,
                     uint32_t n, int K, uint32_t tag, uint32_t parity) {
  if (layers)
    hipLaunchKernelGGL((walk_seg_kernel<kSink, kWeighted, true>), grid, block, 0, st, map->dm, origins, scan, samples,
                       weights, perm, r0, n, K, tag, parity, nullptr, nullptr, nullptr, nullptr);
  else
    hipLaunchKernelGGL((walk_seg_kernel<kSink, kWeighted, false>), grid, block, 0, st, map->dm, origins, scan,
                       samples, weights, perm, r0, n, K, tag, parity, nullptr, nullptr, nullptr, nullptr);
}

template <bool kWeighted>
void launch_walk_group(const ohm_map_s* map, bool layers, dim3 grid, dim3 block, hipStream_t st,
                       const float* origins, const float* samples, const float* weights, const GroupArgs& g, int K,
                       uint32_t tag, uint32_t parity) {
  const bool wide = block.x > 512;
  if (layers) {
    if (wide)
      hipLaunchKernelGGL((walk_group_kernel<kWeighted, true, true>), grid, block, 0, st, map->dm, origins, samples,
                         weights, g, K, tag, parity);
    else
      hipLaunchKernelGGL((walk_group_kernel<kWeighted, true, false>), grid, block, 0, st, map->dm, origins, samples,
                         weights, g, K, tag, parity);
  } else {
    if (wide)
      hipLaunchKernelGGL((walk_group_kernel<kWeighted, false, true>), grid, block, 0, st, map->dm, origins, samples,
                         weights, g, K, tag, parity);
    else
      hipLaunchKernelGGL((walk_group_kernel<kWeighted, false, false>), grid, block, 0, st, map->dm, origins, samples,
                         weights, g, K, tag, parity);
  }
}

}  // namespace ohm

using namespace ohm;

extern "C" {

#ifndef OHM_SOURCE_DIGEST
#define OHM_SOURCE_DIGEST "unknown"
#endif

const char* ohm_build_source_digest(void) { return OHM_SOURCE_DIGEST; }

const char* ohm_status_string(ohm_status s) {
  switch (s) {
    case OHM_OK: return "ok";
    case OHM_E_INVALID_ARG: return "invalid argument";
    case OHM_E_NO_DEVICE: return "no HIP device";
    case OHM_E_HIP: return "HIP runtime error";
    case OHM_E_WORKSPACE_TOO_SMALL: return "workspace too small";
    case OHM_E_UNSUPPORTED: return "unsupported parameter";
  }
  return "unknown status";
}

ohm_status ohm_map_workspace_size(const ohm_params* params, uint32_t region_capacity, uint32_t layers,
                                  size_t* bytes) {
  if (!bytes) return OHM_E_INVALID_ARG;
  Layout L;
  ohm_status s = compute_layout(params, region_capacity, layers, &L);
  if (s != OHM_OK) return s;
  *bytes = L.total;
  return OHM_OK;
}

ohm_status ohm_map_create(const ohm_params* params, uint32_t region_capacity, uint32_t layers, void* d_workspace,
                          size_t workspace_bytes, void* stream, ohm_map* out) {
  if (!out) return OHM_E_INVALID_ARG;
  *out = nullptr;
  Layout L;
  ohm_status s = compute_layout(params, region_capacity, layers, &L);
  if (s != OHM_OK) return s;
  if (!d_workspace || ((uintptr_t)d_workspace & (kAlign - 1))) return OHM_E_INVALID_ARG;
  if (workspace_bytes < L.total) return OHM_E_WORKSPACE_TOO_SMALL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return OHM_E_NO_DEVICE;
  }
  ohm_map_s* map = new (std::nothrow) ohm_map_s();
  if (!map) return OHM_E_INVALID_ARG;
  map->params = *params;
  map->layers = layers | OHM_LAYER_OCC;
  map->group_slots = group_slots_of(layers);
  map->seg_major_steps = kDefaultSegMajorSteps;
  map->walk_threads = kDefaultTileThreads;
  map->column_rays = 0;
  map->order_hist = map->order_sums = map->order_perm = nullptr;
  map->order_max_rays = 0;
  map->regions = L.regions;
  map->workspace = d_workspace;
  map->workspace_bytes = workspace_bytes;
  if (hipGetDevice(&map->device) != hipSuccess) map->device = 0;
  DevMap& dm = map->dm;
  memset(&dm, 0, sizeof(dm));
  fill_params(dm, params);
  for (int a = 0; a < 3; ++a) {
    dm.rlo[a] = L.rlo[a];
    dm.rdim[a] = L.rdim[a];
  }
  dm.capacity = region_capacity;
  char* base = static_cast<char*>(d_workspace);
  dm.hdr = reinterpret_cast<uint32_t*>(base + L.hdr);
  dm.stats = reinterpret_cast<unsigned long long*>(base + L.stats);
  dm.table = reinterpret_cast<int32_t*>(base + L.table);
  dm.stamp = reinterpret_cast<uint32_t*>(base + L.stamp);
  dm.touched = reinterpret_cast<uint32_t*>(base + L.touched);
  dm.occ = reinterpret_cast<float*>(base + L.occ);
  dm.acc = reinterpret_cast<float*>(base + L.acc);
  dm.ndt = (layers & OHM_LAYER_NDT) ? reinterpret_cast<NdtVoxel*>(base + L.ndt) : nullptr;
  dm.nacc = (layers & OHM_LAYER_NDT) ? reinterpret_cast<long long*>(base + L.nacc) : nullptr;
  dm.nsamp = (layers & OHM_LAYER_NDT) ? reinterpret_cast<uint32_t*>(base + L.nsamp) : nullptr;
  dm.mom = (layers & OHM_LAYER_NDT) ? reinterpret_cast<double*>(base + L.mom) : nullptr;
  dm.ndt_ready = (layers & OHM_LAYER_NDT) ? reinterpret_cast<uint32_t*>(base + L.ndt_ready) : nullptr;
  dm.clampscan = (layers & OHM_LAYER_ADJOINT) ? reinterpret_cast<uint32_t*>(base + L.clampscan) : nullptr;
  const bool has_mean = (layers & OHM_LAYER_MEAN) != 0, has_decay = (layers & OHM_LAYER_DECAY) != 0;
  dm.mean = has_mean ? reinterpret_cast<unsigned long long*>(base + L.mean) : nullptr;
  dm.mean_acc = has_mean ? reinterpret_cast<unsigned long long*>(base + L.mean_acc) : nullptr;
  dm.mean_mask = has_mean ? reinterpret_cast<unsigned long long*>(base + L.mean_mask) : nullptr;
  dm.mean_slot = 0;
  dm.decay_len = has_decay ? reinterpret_cast<unsigned long long*>(base + L.decay_len) : nullptr;
  dm.decay_hits = has_decay ? reinterpret_cast<uint32_t*>(base + L.decay_hits) : nullptr;
  const bool has_tm = (layers & OHM_LAYER_NDT_TM) != 0, has_tsdf = (layers & OHM_LAYER_TSDF) != 0;
  dm.tm = has_tm ? reinterpret_cast<TmVoxel*>(base + L.tm) : nullptr;
  dm.tm_mom = has_tm ? reinterpret_cast<double*>(base + L.tm_mom) : nullptr;
  dm.tsdf = has_tsdf ? reinterpret_cast<unsigned long long*>(base + L.tsdf) : nullptr;
  dm.tsdf_acc = has_tsdf ? reinterpret_cast<long long*>(base + L.tsdf_acc) : nullptr;
  s = map_initialise(map, as_stream(stream));
  if (s != OHM_OK) {
    delete map;
    return s;
  }
  *out = map;
  return OHM_OK;
}

ohm_status ohm_map_destroy(ohm_map map) {
  if (!map) return OHM_E_INVALID_ARG;
  for (hipEvent_t e : map->event_pool) (void)hipEventDestroy(e);
  delete map;
  return OHM_OK;
}

ohm_status ohm_map_reset(ohm_map map, void* stream) {
  if (!map) return OHM_E_INVALID_ARG;
  return map_initialise(map, as_stream(stream));
}

ohm_status ohm_map_set_params(ohm_map map, const ohm_params* params) {
  if (!map) return OHM_E_INVALID_ARG;
  ohm_status s = validate_params(params);
  if (s != OHM_OK) return s;
  const ohm_params& o = map->params;
  if (params->voxel_size != o.voxel_size || params->fixed_bits != o.fixed_bits ||
      params->region_log2 != o.region_log2)
    return OHM_E_INVALID_ARG;
  for (int a = 0; a < 3; ++a)
    if (params->map_origin[a] != o.map_origin[a] || params->key_min[a] != o.key_min[a] ||
        params->key_max[a] != o.key_max[a])
      return OHM_E_INVALID_ARG;
  if (map->dm.ndt && params->ndt_min_samples != map->params.ndt_min_samples) map->ndt_ready_stale = true;
  map->params = *params;
  fill_params(map->dm, params);
  return OHM_OK;
}

}  // extern "C"

namespace ohm {

// ohm_integrate_rays with the ordering scratch given explicitly; prof =
// false records no profiling events (the allocation-free entry point).
ohm_status integrate_rays_impl(ohm_map map, const float* d_origins, const float* d_samples,
                               const uint32_t* h_scan_offsets, uint32_t n_scans, const float* d_weights,
                               hipStream_t st, const OrderScratch& ord, bool prof) {
  const bool layers = map->dm.mean || map->dm.decay_len;  // walks that also update the optional layers
  const bool count_mode = map->params.mode == OHM_MODE_COUNT_CLAMP;
  const bool weighted = d_weights != nullptr;
  uint32_t last = n_scans;
  for (uint32_t sc = 0; sc < n_scans; ++sc)
    if (h_scan_offsets[sc + 1] > h_scan_offsets[sc]) last = sc;
  uint32_t first = 0;  // scans before `first` went through grouped launches
  if (count_mode && (map->layers & OHM_LAYER_SCAN_GROUPS) && ord.max_rays == 0 && last < n_scans) {
    // groups of up to G non-empty scans; the group holding the last one
    // keeps its counts readable in that scan's slot
    const uint32_t threads = map->walk_threads;
    const int K = map->seg_major_steps;
    // a weighted scan's wide slot takes two of the map's f32 slots
    const uint32_t group_max = weighted ? map->group_slots / 2 : map->group_slots;
    uint32_t sc = 0;
    while (sc <= last && group_max > 0) {
      GroupArgs g = {};
      g.col_rays = map->column_rays;
      uint32_t tiles = 0;
      for (; sc <= last && g.count < group_max; ++sc) {
        const uint32_t r0 = h_scan_offsets[sc];
        const uint32_t n = h_scan_offsets[sc + 1] - r0;
        if (n == 0) continue;
        g.scan[g.count] = sc;
        g.r0[g.count] = r0;
        g.n[g.count] = n;
        tiles += (n + kTileRays - 1) / kTileRays;
        g.tile_end[g.count] = tiles;
        ++g.count;
      }
      if (g.count == 0) break;
      clear_pending(map, st, prof);
      const uint32_t tag = ++map->count_batches;
      const uint32_t parity = tag & 1u;
      {
        ProfScope ps(map, OHM_KERNEL_WALK_GROUP, st, prof);
        if (weighted)
          launch_walk_group<true>(map, layers, dim3(tiles), dim3(threads), st, d_origins, d_samples, d_weights, g, K,
                                  tag, parity);
        else
          launch_walk_group<false>(map, layers, dim3(tiles), dim3(threads), st, d_origins, d_samples, d_weights, g,
                                   K, tag, parity);
      }
      const bool has_last = g.scan[g.count - 1] == last;
      const uint32_t keep = has_last ? g.count - 1 : kMaxGroupSlots;
      {
        ProfScope ps(map, OHM_KERNEL_FINALIZE_GROUP, st, prof);
        if (weighted)
          hipLaunchKernelGGL(group_finalize_kernel<true>, dim3(kFinalizeBlocks), dim3(256), 0, st, map->dm, parity,
                             g.count, map->scans_done + 1, keep);
        else
          hipLaunchKernelGGL(group_finalize_kernel<false>, dim3(kFinalizeBlocks), dim3(256), 0, st, map->dm, parity,
                             g.count, map->scans_done + 1, keep);
      }
      map->scans_done += g.count;
      if (has_last) {
        map->acc_dirty = true;
        map->last_parity = parity;
        map->kept_slot = keep;
        map->kept_wide = weighted;
      }
    }
    if (group_max > 0) first = n_scans;
  }
  for (uint32_t sc = first; sc < n_scans; ++sc) {
    const uint32_t r0 = h_scan_offsets[sc];
    const uint32_t n = h_scan_offsets[sc + 1] - r0;
    if (n == 0) continue;
    uint32_t tag = 0, parity = 0;
    if (count_mode) {
      clear_pending(map, st, prof);
      tag = ++map->count_batches;
      parity = tag & 1u;
    }
    const dim3 tiles((n + kTileRays - 1) / kTileRays);
    const dim3 threads(map->walk_threads);
    const int K = map->seg_major_steps;
    const uint32_t* perm = nullptr;
    if (n <= ord.max_rays) {
      // walk the scan in direction order
      ProfScope ps(map, OHM_KERNEL_OTHER, st, prof);
      const float* o = d_origins + 3 * (size_t)sc;
      const float* smp = d_samples + 3 * (size_t)r0;
      const uint32_t bins = order_bins(n, kOrderStripRaysScan), strips = order_strips(n, kOrderStripRaysScan);
      hipLaunchKernelGGL(fill_u32_kernel, dim3((bins + 255) / 256 < 8192 ? (bins + 255) / 256 : 8192), dim3(256), 0,
                         st, ord.hist, (size_t)bins, 0u);
      hipLaunchKernelGGL(scan_order_count_kernel, dim3((n + 255) / 256), dim3(256), 0, st, o, smp, n,
                         ord.hist);
      hipLaunchKernelGGL(scan_order_strip_kernel, dim3(strips), dim3(kOrderElevationBins), 0, st, ord.hist,
                         ord.sums);
      hipLaunchKernelGGL(scan_order_sums_kernel, dim3(1), dim3(kOrderMaxStrips), 0, st, ord.sums, strips);
      hipLaunchKernelGGL(scan_order_place_kernel, dim3((n + 255) / 256), dim3(256), 0, st, o, smp, n,
                         ord.hist, ord.sums, ord.perm);
      perm = ord.perm;
    }
    if (count_mode) {
      {
        ProfScope ps(map, OHM_KERNEL_WALK, st, prof);
        if (weighted)
          launch_walk_seg<kSinkCount, true>(map, layers, tiles, threads, st, d_origins, sc, d_samples, d_weights,
                                            perm, r0, n, K, tag, parity);
        else
          launch_walk_seg<kSinkCount, false>(map, layers, tiles, threads, st, d_origins, sc, d_samples, d_weights,
                                             perm, r0, n, K, tag, parity);
      }
      const bool keep = sc == last;
      {
        ProfScope ps(map, OHM_KERNEL_FINALIZE, st, prof);
        if (weighted)
          hipLaunchKernelGGL(finalize_kernel<true>, dim3(kFinalizeBlocks), dim3(256), 0, st, map->dm, parity, 1,
                             keep ? 0 : 1, map->scans_done + 1);
        else
          hipLaunchKernelGGL(finalize_kernel<false>, dim3(kFinalizeBlocks), dim3(256), 0, st, map->dm, parity, 1,
                             keep ? 0 : 1, map->scans_done + 1);
      }
      if (keep) {
        map->acc_dirty = true;
        map->last_parity = parity;
        map->kept_wide = weighted;
      }
    } else {
      ProfScope ps(map, OHM_KERNEL_WALK, st, prof);
      if (weighted)
        launch_walk_seg<kSinkCas, true>(map, layers, tiles, threads, st, d_origins, sc, d_samples, d_weights, perm,
                                        r0, n, K, tag, parity);
      else
        launch_walk_seg<kSinkCas, false>(map, layers, tiles, threads, st, d_origins, sc, d_samples, d_weights, perm,
                                         r0, n, K, tag, parity);
    }
    map->scans_done += 1;
  }
  return last_hip_status();
}

}  // namespace ohm

extern "C" {

ohm_status ohm_integrate_rays(ohm_map map, const float* d_origins, const float* d_samples,
                              const uint32_t* h_scan_offsets, uint32_t n_scans, const float* d_weights,
                              void* stream) {
  ohm_status s = check_scans(map, d_origins, d_samples, h_scan_offsets, n_scans);
  if (s != OHM_OK || n_scans == 0) return s;
  const OrderScratch ord{map->order_hist, map->order_sums, map->order_perm, map->order_max_rays};
  return integrate_rays_impl(map, d_origins, d_samples, h_scan_offsets, n_scans, d_weights, as_stream(stream), ord,
                             true);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free entry point
// ---------------------------------------------------------------------------

namespace {

// Direction-ordering scratch of ohm_integrate_rays_no_alloc: the bin
// histogram, the strip sums and the permutation for one scan of up to
// OHM_NO_ALLOC_MAX_RAYS rays.  Each GPU the library runs on holds its own
// copy until the process ends; every call on that GPU shares it.
constexpr uint32_t kNoAllocMaxRays = OHM_NO_ALLOC_MAX_RAYS;
constexpr size_t kNoAllocScratchBytes = (size_t)kOrderMaxStrips * kOrderElevationBins * sizeof(uint32_t) +
                                        (size_t)kOrderMaxStrips * sizeof(uint32_t) +
                                        (size_t)kNoAllocMaxRays * sizeof(uint32_t);
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device (null until looked up)

// The device address of the current device's `scratch` (looked up once per
// device); null on failure.
void* scratch_of_device(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

ohm_status ohm_integrate_rays_no_alloc(ohm_map map, const float* d_origins, const float* d_samples,
                                       const uint32_t* h_scan_offsets, uint32_t n_scans, const float* d_weights,
                                       void* stream) {
  ohm_status s = check_scans(map, d_origins, d_samples, h_scan_offsets, n_scans);
  if (s != OHM_OK || n_scans == 0) return s;
  for (uint32_t sc = 0; sc < n_scans; ++sc)
    if (h_scan_offsets[sc + 1] - h_scan_offsets[sc] > kNoAllocMaxRays) return OHM_E_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != map->device) return OHM_E_INVALID_ARG;
  if (order_scratch_bytes(kNoAllocMaxRays) > kNoAllocScratchBytes) return OHM_E_UNSUPPORTED;
  void* base = scratch_of_device(dev);
  if (!base) return OHM_E_HIP;
  const OrderScratch ord = order_scratch_at(base, kNoAllocMaxRays);
  return integrate_rays_impl(map, d_origins, d_samples, h_scan_offsets, n_scans, d_weights, as_stream(stream), ord,
                             false);
}

ohm_status ohm_map_read_dense(ohm_map map, int32_t what, const int32_t h_box_min[3], const int32_t h_box_dim[3],
                              void* d_out, void* stream) {
  if (!map || !h_box_min || !h_box_dim || !d_out) return OHM_E_INVALID_ARG;
  if (what < OHM_READ_OCC || what > OHM_READ_TSDF_WEIGHT) return OHM_E_INVALID_ARG;
  if (what >= OHM_READ_TM_MISSES && what <= OHM_READ_INTENSITY_VAR && !map->dm.tm) return OHM_E_INVALID_ARG;
  if ((what == OHM_READ_TSDF_DISTANCE || what == OHM_READ_TSDF_WEIGHT) && !map->dm.tsdf) return OHM_E_INVALID_ARG;
  if ((what == OHM_READ_MEAN_PACKED || what == OHM_READ_MEAN_COUNT || what == OHM_READ_MEAN) && !map->dm.mean)
    return OHM_E_INVALID_ARG;
  if ((what == OHM_READ_DECAY_LENGTH || what == OHM_READ_DECAY_HITS || what == OHM_READ_DECAY_RATE) &&
      !map->dm.decay_len)
    return OHM_E_INVALID_ARG;
  if ((what == OHM_READ_NDT_COUNT || what == OHM_READ_NDT_MEAN || what == OHM_READ_NDT_COV) && !map->dm.ndt)
    return OHM_E_INVALID_ARG;
  if (what == OHM_READ_CLAMP_SCAN && !map->dm.clampscan) return OHM_E_INVALID_ARG;
  for (int a = 0; a < 3; ++a)
    if (h_box_dim[a] <= 0) return OHM_E_INVALID_ARG;
  const size_t n = (size_t)h_box_dim[0] * h_box_dim[1] * h_box_dim[2];
  const size_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffff) return OHM_E_INVALID_ARG;
  hipLaunchKernelGGL(read_dense_kernel, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), kept_counts(map), what,
                     map->kept_wide ? 1 : 0, h_box_min[0], h_box_min[1], h_box_min[2], h_box_dim[0], h_box_dim[1], h_box_dim[2], d_out);
  return last_hip_status();
}

ohm_status ohm_debug_trace_rays(ohm_map map, const float* d_origins, const float* d_samples,
                                const uint32_t* h_scan_offsets, uint32_t n_scans, uint32_t* d_ray_counts,
                                int32_t* d_ray_flags, const int64_t* d_ray_offsets, int32_t* d_updates,
                                void* stream) {
  ohm_status s = check_scans(map, d_origins, d_samples, h_scan_offsets, n_scans);
  if (s != OHM_OK || n_scans == 0) return s;
  if (!d_updates && (!d_ray_counts || !d_ray_flags)) return OHM_E_INVALID_ARG;
  if (d_updates && !d_ray_offsets) return OHM_E_INVALID_ARG;
  hipStream_t st = as_stream(stream);
  for (uint32_t sc = 0; sc < n_scans; ++sc) {
    const uint32_t r0 = h_scan_offsets[sc];
    const uint32_t n = h_scan_offsets[sc + 1] - r0;
    if (n == 0) continue;
    const dim3 tiles((n + kTileRays - 1) / kTileRays);
    const dim3 threads(map->walk_threads);
    if (!d_updates)
      hipLaunchKernelGGL((walk_seg_kernel<kSinkTraceCount, false>), tiles, threads, 0, st, map->dm, d_origins, sc,
                         d_samples, nullptr, nullptr, r0, n, map->seg_major_steps, 0u, 0u, d_ray_counts, d_ray_flags, nullptr,
                         nullptr);
    else
      hipLaunchKernelGGL((walk_seg_kernel<kSinkTraceWrite, false>), tiles, threads, 0, st, map->dm, d_origins, sc,
                         d_samples, nullptr, nullptr, r0, n, map->seg_major_steps, 0u, 0u, nullptr, nullptr, d_ray_offsets,
                         d_updates);
  }
  return last_hip_status();
}

ohm_status ohm_ray_order_scratch_size(uint32_t max_rays, size_t* bytes) {
  if (!bytes || max_rays == 0) return OHM_E_INVALID_ARG;
  *bytes = order_scratch_bytes(max_rays);
  return OHM_OK;
}

ohm_status ohm_map_set_ray_order(ohm_map map, void* d_scratch, size_t bytes, uint32_t max_rays) {
  if (!map) return OHM_E_INVALID_ARG;
  if (!d_scratch) {
    map->order_hist = map->order_sums = map->order_perm = nullptr;
    map->order_max_rays = 0;
    return OHM_OK;
  }
  size_t need = 0;
  if (ohm_ray_order_scratch_size(max_rays, &need) != OHM_OK) return OHM_E_INVALID_ARG;
  if ((uintptr_t)d_scratch & (kAlign - 1)) return OHM_E_INVALID_ARG;
  if (bytes < need) return OHM_E_WORKSPACE_TOO_SMALL;
  const OrderScratch o = order_scratch_at(d_scratch, max_rays);
  map->order_hist = o.hist;
  map->order_sums = o.sums;
  map->order_perm = o.perm;
  map->order_max_rays = max_rays;
  return OHM_OK;
}

ohm_status ohm_map_set_tuning(ohm_map map, const ohm_walk_tuning* t) {
  if (!map || !t) return OHM_E_INVALID_ARG;
  if (t->seg_major_steps < 1 || t->seg_major_steps > 4096) return OHM_E_INVALID_ARG;
  if (t->tile_threads != 256 && t->tile_threads != 512 && t->tile_threads != 1024) return OHM_E_INVALID_ARG;
  map->seg_major_steps = (int)t->seg_major_steps;
  map->walk_threads = t->tile_threads;
  return OHM_OK;
}

ohm_status ohm_map_set_scan_layout(ohm_map map, uint32_t column_rays) {
  if (!map) return OHM_E_INVALID_ARG;
  if (column_rays % 8u != 0u || column_rays > kMaxColumnRays) return OHM_E_INVALID_ARG;
  map->column_rays = column_rays;
  return OHM_OK;
}

ohm_status ohm_map_set_profiling(ohm_map map, int enable) {
  if (!map) return OHM_E_INVALID_ARG;
  map->profiling = enable != 0;
  return OHM_OK;
}

ohm_status ohm_map_kernel_times(ohm_map map, uint32_t* h_launches, double* h_ms) {
  if (!map || !h_launches || !h_ms) return OHM_E_INVALID_ARG;
  for (int k = 0; k < OHM_KERNEL_KINDS; ++k) {
    h_launches[k] = 0;
    h_ms[k] = 0.0;
  }
  ohm_status st = OHM_OK;
  for (const auto& t : map->timed) {
    if (!t.stop || hipEventSynchronize(t.stop) != hipSuccess) {
      st = OHM_E_HIP;
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.start, t.stop) != hipSuccess) {
      st = OHM_E_HIP;
      continue;
    }
    h_launches[t.kind] += 1;
    h_ms[t.kind] += (double)ms;
  }
  map->timed.clear();
  map->events_used = 0;
  return st;
}

ohm_status ohm_map_sync_status(ohm_map map, void* stream, ohm_map_stats* out) {
  if (!map || !out) return OHM_E_INVALID_ARG;
  hipStream_t st = as_stream(stream);
  uint32_t hdr[kHdrWords];
  unsigned long long stats[16];
  if (hipMemcpyAsync(hdr, map->dm.hdr, sizeof(hdr), hipMemcpyDeviceToHost, st) != hipSuccess) return OHM_E_HIP;
  if (hipMemcpyAsync(stats, map->dm.stats, sizeof(stats), hipMemcpyDeviceToHost, st) != hipSuccess)
    return OHM_E_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return OHM_E_HIP;
  memset(out, 0, sizeof(*out));
  out->rays_in = stats[kStatRays];
  out->rays_invalid = stats[kStatInvalid];
  out->rays_origin_oob = stats[kStatOriginOob];
  out->rays_truncated = stats[kStatTruncated];
  out->rays_clipped = stats[kStatClipped];
  out->rays_hit = stats[kStatHits];
  out->voxel_updates = stats[kStatUpdates];
  out->updates_dropped_pool = stats[kStatDropped];
  out->regions_used = hdr[kHdrPoolCount] < map->dm.capacity ? hdr[kHdrPoolCount] : map->dm.capacity;
  out->region_capacity = map->dm.capacity;
  out->sticky_error = (int32_t)hdr[kHdrSticky];
  return OHM_OK;
}

}  // extern "C"
