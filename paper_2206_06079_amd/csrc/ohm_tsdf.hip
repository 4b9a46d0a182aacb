// TSDF integration (paper Sec. II-F: voxels up to a truncation distance in
// front of and behind the measured point, along the ray from the sensor,
// take a projective distance; Sec. III-B: such 64-bit voxels are updated by
// compare-and-swap like the other layers).
//
// Only a ray with a surface takes part: valid, origin in the map, not
// truncated by max range, sample voxel in the map, non-zero length.  With
// r = |e - o| and u = (e - o) / r, its band is the segment from
// o + max(r - tau, 0) u to o + (r + tau) u.  The band's ends are quantised
// like ray ends and the band is walked with the same exact line walk as the
// occupancy rays, so its voxel set is exact.  Each band voxel with centre c
// takes sd = clamp(r - (c - o).u, -tau, tau).  A voxel keeps a distance D and
// a weight W; n updates of summed distance S give
//   D <- (W D + S) / (W + n),  W <- min(W + n, W_max)   (fp64, stored as float).
//
// One thread per ray, 256 rays per block: a band is a few voxels long, so
// segmenting it (as the occupancy walk does its rays) would cost more than
// it balances.  The block stages the regions of its bands in LDS first.
//   count mode: each update's Q32.32 distance and count go to the voxel's
//     per-scan sums (exact integers: the result does not depend on the order
//     of the adds); tsdf_finalize_kernel applies them per voxel of the
//     scan's regions.  Adjacent rays of a scan reach nearby points of one
//     surface, so their bands share voxels: the lanes step in lockstep, runs
//     of adjacent lanes in one voxel are summed in registers, and a per-block
//     LDS table (voxel -> sums) takes the runs, so the global sums see about
//     one update per voxel and block.
//   per-update mode: each update is applied at once by one 64-bit
//     compare-and-swap on the packed (D, W) word, retried until it lands.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ohm.h"
#include "ohm_device.h"
#include "ohm_host.h"
#include "ohm_regions.h"
#include "ohm_seg_math.h"
#include "ohm_wave.h"

namespace ohm {

namespace {

constexpr uint32_t kTsdfThreads = kTileRays;  // one ray per thread

__device__ __forceinline__ bool key_in_map(const DevMap& m, const int32_t k[3]) {
  return k[0] >= m.kmin[0] && k[0] < m.kmax[0] && k[1] >= m.kmin[1] && k[1] < m.kmax[1] && k[2] >= m.kmin[2] &&
         k[2] < m.kmax[2];
}

// The band of a prepared ray (r: prepare_ray's result, status ok); false
// when the ray has no surface or its band starts outside the map.
__device__ __forceinline__ bool tsdf_band(const DevMap& m, const float o[3], const float e[3], const Ray& r,
                                          Ray& band, double& range, double u[3]) {
#pragma clang fp contract(off)
  if (r.truncated || !key_in_map(m, r.k1)) return false;
  double d[3];
  for (int a = 0; a < 3; ++a) d[a] = (double)e[a] - (double)o[a];
  double r2 = d[0] * d[0];
  r2 = r2 + d[1] * d[1];
  r2 = r2 + d[2] * d[2];
  if (!(r2 > 0.0)) return false;
  const double len = __dsqrt_rn(r2);
  const double tau = m.tsdf_tau;
  double s0 = len - tau;
  s0 = s0 < 0.0 ? 0.0 : s0;
  const double s1 = len + tau;
  for (int a = 0; a < 3; ++a) {
    u[a] = d[a] / len;
    const double b0 = (double)o[a] + s0 * u[a];
    const double b1 = (double)o[a] + s1 * u[a];
    if (!quantise(b0, m.origin[a], m.scale, band.q0[a]) || !quantise(b1, m.origin[a], m.scale, band.q1[a]))
      return false;
    band.k0[a] = (int32_t)(band.q0[a] >> m.F);
    band.k1[a] = (int32_t)(band.q1[a] >> m.F);
    band.end[a] = b1;
  }
  band.truncated = false;
  if (!key_in_map(m, band.k0)) return false;
  range = len;
  return true;
}

// Projective distance of voxel k for a ray from o of length range along u.
__device__ __forceinline__ double tsdf_distance(const DevMap& m, const float o[3], double range, const double u[3],
                                                const int32_t k[3]) {
#pragma clang fp contract(off)
  double c[3];
  for (int a = 0; a < 3; ++a) c[a] = m.origin[a] + ((double)k[a] + 0.5) * m.voxel_size;
  double proj = (c[0] - (double)o[0]) * u[0];
  proj = proj + (c[1] - (double)o[1]) * u[1];
  proj = proj + (c[2] - (double)o[2]) * u[2];
  const double v = range - proj;
  const double tau = m.tsdf_tau;
  return v < -tau ? -tau : (v > tau ? tau : v);
}

// (D, W) after n updates of summed distance s, packed (D low, W high).
__device__ __forceinline__ unsigned long long tsdf_merge(const DevMap& m, unsigned long long word, double s,
                                                         double n) {
#pragma clang fp contract(off)
  const double D = (double)__uint_as_float((uint32_t)word);
  const double W = (double)__uint_as_float((uint32_t)(word >> 32));
  const double Dn = (D * W + s) / (W + n);
  double Wn = W + n;
  Wn = Wn > m.tsdf_wmax ? m.tsdf_wmax : Wn;
  return ((unsigned long long)__float_as_uint((float)Wn) << 32) | (unsigned long long)__float_as_uint((float)Dn);
}

// Per-block LDS table of count-mode updates: voxel index -> (summed Q32.32
// distance, update count), two probes; a run whose two entries belong to
// other voxels goes to the global sums at once.
constexpr int kTsdfAggLog2 = 11;
constexpr uint32_t kTsdfAggSize = 1u << kTsdfAggLog2;
constexpr uint32_t kTsdfEmpty = 0xFFFFFFFFu;  // above every voxel index (capacity <= kMaxCapacity)

__device__ __forceinline__ bool tsdf_agg_add(uint32_t* keys, unsigned long long* sums, uint32_t* counts, uint32_t v,
                                             long long q, uint32_t c) {
  uint32_t h = (v * 0x9E3779B1u) >> (32 - kTsdfAggLog2);
  for (int p = 0; p < 2; ++p) {
    uint32_t k = keys[h];
    if (k == kTsdfEmpty) {
      const uint32_t old = atomicCAS(keys + h, kTsdfEmpty, v);
      k = old == kTsdfEmpty ? v : old;
    }
    if (k == v) {
      atomicAdd(sums + h, (unsigned long long)q);
      atomicAdd(counts + h, c);
      return true;
    }
    h = (h + 1) & (kTsdfAggSize - 1);
  }
  return false;
}

__device__ __forceinline__ void tsdf_global_add(const DevMap& m, uint32_t v, long long q, uint32_t c) {
  unsigned long long* a = reinterpret_cast<unsigned long long*>(m.tsdf_acc + 2 * (size_t)v);
  atomicAdd(a, (unsigned long long)q);
  atomicAdd(a + 1, (unsigned long long)c);
}

template <bool kCount>
__global__ __launch_bounds__(kTsdfThreads) void tsdf_kernel(DevMap m, const float* __restrict__ origins, uint32_t scan,
                                                           const float* __restrict__ samples, uint32_t r0, uint32_t n,
                                                           uint32_t tag, uint32_t parity) {
  __shared__ RegionCache rc;
  __shared__ uint32_t agg_key[kCount ? kTsdfAggSize : 1];
  __shared__ unsigned long long agg_sum[kCount ? kTsdfAggSize : 1];
  __shared__ uint32_t agg_cnt[kCount ? kTsdfAggSize : 1];
  if (kCount)
    for (uint32_t h = threadIdx.x; h < kTsdfAggSize; h += blockDim.x) {
      agg_key[h] = kTsdfEmpty;
      agg_sum[h] = 0ull;
      agg_cnt[h] = 0u;
    }
  const uint32_t lane = lane_id();
  const uint32_t i = blockIdx.x * kTsdfThreads + threadIdx.x;
  const bool inrange = i < n;
  const float o[3] = {origins[3 * (size_t)scan], origins[3 * (size_t)scan + 1], origins[3 * (size_t)scan + 2]};
  int st = kRayInvalid;
  Ray r, band;
  bool has = false, clipped = false;
  double range = 0.0, u[3] = {0.0, 0.0, 0.0};
  if (inrange) {
    const size_t ray = (size_t)r0 + i;
    const float e[3] = {samples[3 * ray], samples[3 * ray + 1], samples[3 * ray + 2]};
    st = prepare_ray(m, o, e, r);
    if (st == kRayOk) {
      clipped = !r.truncated && !key_in_map(m, r.k1);
      has = tsdf_band(m, o, e, r, band, range, u);
    }
  }
  const RegionWindow rw = stage_regions<kCount>(m, rc, has, band, tag, parity);
  uint32_t n_upd = 0, n_drop = 0;
  Walk w;
  int32_t k[3] = {0, 0, 0};
  bool alive = has;
  if (has) {
    const int32_t hi[3] = {m.kmax[0] - 1, m.kmax[1] - 1, m.kmax[2] - 1};
    walk_init(w, band.q0, band.q1, band.k0, band.k1, m.kmin, hi, m.F);
    for (int a = 0; a < 3; ++a) k[a] = band.k0[a];
  }
  // lockstep band walks: at every step each live lane visits one voxel
  while (__ballot(alive)) {
    int32_t slot = -1;
    uint32_t v = kTsdfEmpty - lane;  // distinct per lane where there is no update
    long long q = 0;
    if (alive) {
      slot = staged_slot(m, rc, rw, k[0], k[1], k[2]);
      if (slot >= 0) {
        v = (uint32_t)slot * (uint32_t)kRegionVoxels + local_index(k[0], k[1], k[2]);
        if (kCount) q = llrint(tsdf_distance(m, o, range, u, k) * kQ32);
        ++n_upd;
      } else {
        ++n_drop;
      }
    }
    const bool upd = alive && slot >= 0;
    if (kCount) {
      // runs of adjacent lanes in one voxel: the run's tail holds its summed
      // distance and counts its lanes back to the head
      const LaneRuns run = lane_runs(v, lane);
      const long long qs = segmented_sum<long long>(q, run.head, lane);
      const unsigned long long heads = __ballot(run.head);
      const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
      const uint32_t head_lane = 63u - (uint32_t)__builtin_clzll(heads & upto);
      if (upd && run.tail) {
        const uint32_t c = lane - head_lane + 1u;
        if (!tsdf_agg_add(agg_key, agg_sum, agg_cnt, v, qs, c)) tsdf_global_add(m, v, qs, c);
      }
    } else if (upd) {
      const double sd = tsdf_distance(m, o, range, u, k);
      unsigned long long old = __hip_atomic_load(m.tsdf + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (;;) {
        const unsigned long long prev = atomicCAS(m.tsdf + v, old, tsdf_merge(m, old, sd, 1.0));
        if (prev == old) break;
        old = prev;
      }
    }
    if (alive) {
      if (w.total == 0) {
        alive = false;
      } else {
        const int a = walk_step(w);
        const int32_t ra = a == 0 ? w.rem[0] : (a == 1 ? w.rem[1] : w.rem[2]);
        if (ra == 0 && ((w.clip >> a) & 1u)) {
          alive = false;  // the band leaves the map
        } else {
          k[a] += w.sg[a];
        }
      }
    }
  }
  if (kCount) {
    __syncthreads();
    for (uint32_t h = threadIdx.x; h < kTsdfAggSize; h += blockDim.x) {
      const uint32_t key = agg_key[h];
      if (key != kTsdfEmpty) tsdf_global_add(m, key, (long long)agg_sum[h], agg_cnt[h]);
    }
  }
  uint32_t vals[kStatCount];
  vals[kStatRays] = inrange ? 1u : 0u;
  vals[kStatInvalid] = (inrange && st == kRayInvalid) ? 1u : 0u;
  vals[kStatOriginOob] = (inrange && st == kRayOriginOob) ? 1u : 0u;
  vals[kStatTruncated] = (st == kRayOk && r.truncated) ? 1u : 0u;
  vals[kStatClipped] = clipped ? 1u : 0u;
  vals[kStatHits] = has ? 1u : 0u;
  vals[kStatUpdates] = n_upd;
  vals[kStatDropped] = n_drop;
  flush_stats(m, vals);
}

constexpr int kTsdfChunk = 1024;  // voxels per work unit
constexpr int kTsdfUnits = kRegionVoxels / kTsdfChunk;

// Count mode: apply each voxel's summed distance and update count of the
// scan to (D, W), clear the sums, and reset the other parity's touched
// counter for the next scan.
__global__ __launch_bounds__(256) void tsdf_finalize_kernel(DevMap m, uint32_t parity) {
  const uint32_t count = __hip_atomic_load(m.hdr + kHdrTouched0 + parity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t units = count * kTsdfUnits;
  for (uint32_t unit = blockIdx.x; unit < units; unit += gridDim.x) {
    const uint32_t slot = m.touched[(size_t)parity * m.capacity + unit / kTsdfUnits];
    const size_t base = (size_t)slot * kRegionVoxels + (size_t)(unit % kTsdfUnits) * kTsdfChunk;
    for (int j = threadIdx.x; j < kTsdfChunk; j += blockDim.x) {
      const size_t v = base + j;
      longlong2* ap = reinterpret_cast<longlong2*>(m.tsdf_acc + 2 * v);
      const longlong2 a = *ap;
      if (a.y == 0) continue;
      m.tsdf[v] = tsdf_merge(m, m.tsdf[v], (double)a.x * kInvQ32, (double)a.y);
      *ap = make_longlong2(0, 0);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(m.hdr + kHdrTouched0 + (parity ^ 1u), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

}  // namespace ohm

using namespace ohm;

extern "C" ohm_status ohm_tsdf_integrate(ohm_map map, const float* d_origins, const float* d_samples,
                                         const uint32_t* h_scan_offsets, uint32_t n_scans, void* stream) {
  ohm_status s = check_scans(map, d_origins, d_samples, h_scan_offsets, n_scans);
  if (s != OHM_OK) return s;
  if (!map->dm.tsdf) return OHM_E_INVALID_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const bool count_mode = map->params.mode == OHM_MODE_COUNT_CLAMP;
  for (uint32_t sc = 0; sc < n_scans; ++sc) {
    const uint32_t r0 = h_scan_offsets[sc];
    const uint32_t n = h_scan_offsets[sc + 1] - r0;
    if (n == 0) continue;
    const dim3 blocks((n + kTsdfThreads - 1) / kTsdfThreads);
    if (count_mode) {
      clear_pending(map, st);
      const uint32_t tag = ++map->count_batches;
      const uint32_t parity = tag & 1u;
      {
        ProfScope ps(map, OHM_KERNEL_WALK, st);
        hipLaunchKernelGGL(tsdf_kernel<true>, blocks, dim3(kTsdfThreads), 0, st, map->dm, d_origins, sc, d_samples,
                           r0, n, tag, parity);
      }
      ProfScope ps(map, OHM_KERNEL_FINALIZE, st);
      hipLaunchKernelGGL(tsdf_finalize_kernel, dim3(kFinalizeBlocks), dim3(256), 0, st, map->dm, parity);
    } else {
      ProfScope ps(map, OHM_KERNEL_WALK, st);
      hipLaunchKernelGGL(tsdf_kernel<false>, blocks, dim3(kTsdfThreads), 0, st, map->dm, d_origins, sc, d_samples, r0,
                         n, 0u, 0u);
    }
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? OHM_OK : OHM_E_HIP;
}
