// NDT-OM integration (paper Sec. II-D and III-C).
//
// Each voxel of an NDT map keeps a sample count n, a mean mu and a population
// covariance Sigma (voxel-centred, metres).  Per scan:
//   phase 1 (ndt_seg_kernel): every ray is walked exactly as in the occupancy
//     path, segment by segment.  Each miss voxel whose statistics hold >= ndt_min_samples samples
//     weights its miss by the Gaussian agreement of the ray with the samples:
//       x* = closest point of the segment to mu,  D = x* - mu,
//       S = Sigma + sensor_noise^2 I,  g = exp(-D^T S^-1 D / 2),
//       p = 1/2 - lambda g (1/2 - sigmoid(l_miss)),  delta = logit(p),
//     (plain l_miss otherwise); statistics are only read in this phase.
//     Increments are summed per voxel as Q32.32 integers (exact, so the
//     result does not depend on the order the GPU adds them in); in
//     per-update mode the misses are instead applied at once by CAS.  A hit
//     adds its sample's offset x from the voxel centre to the voxel's
//     moments (sum x, sum x x^T, fp64) and counts one sample; extra blocks
//     of the same launch (ndt_hit_block) do this for the scan's hits.
//   phase 2 (ndt_finalize_kernel): one thread per voxel of the scan's
//     regions applies the occupancy update, clears the statistics of voxels
//     that fell below ndt_clear_below, and merges the scan's sample moments
//     into (n, mu, Sigma) (Chan et al.'s pairwise update), as the paper's
//     per-voxel second phase does.
//
// NDT-TM (paper Sec. II-D; OHM_LAYER_NDT_TM) rides on the same two phases:
// a miss the voxel's Gaussian weights is also checked against it, and
// counts toward the voxel's misses M when the squared Mahalanobis distance
// q of the ray's closest point is at most the gate; a hit adds its ray's
// intensity to the scan's intensity moments, which phase 2 merges into the
// voxel's intensity mean and variance alongside the position statistics.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ohm.h"
#include "ohm_device.h"
#include "ohm_host.h"
#include "ohm_regions.h"
#include "ohm_walk_seg.h"
#include "ohm_wave.h"

namespace ohm {


// The NDT-weighted miss increment (see the file comment).  o / d: ray start
// and direction (end - start), world, fp64; c: voxel centre; nv: statistics.
// q_out: the squared Mahalanobis distance D^T S^-1 D behind the weight.
__device__ __forceinline__ double ndt_delta(const DevMap& m, const double o[3], const double d[3], double dd,
                                            const double c[3], const NdtVoxel& nv, double sig_miss, double& q_out) {
#pragma clang fp contract(off)
  double mu[3], w[3];
  double wd = 0.0;
  for (int a = 0; a < 3; ++a) {
    mu[a] = c[a] + (double)nv.mean[a];
    w[a] = mu[a] - o[a];
    wd = wd + w[a] * d[a];
  }
  double t = dd > 0.0 ? wd / dd : 0.0;
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  double D[3];
  for (int a = 0; a < 3; ++a) D[a] = (o[a] + t * d[a]) - mu[a];
  const double s2 = (double)m.sensor_noise * (double)m.sensor_noise;
  // Cholesky of S = Sigma + s2 I; D^T S^-1 D = |L^-1 D|^2
  const double a00 = (double)nv.cov[0] + s2, a10 = nv.cov[1], a20 = nv.cov[2];
  const double a11 = (double)nv.cov[3] + s2, a21 = nv.cov[4], a22 = (double)nv.cov[5] + s2;
  const double l00 = sqrt(a00);
  const double l10 = a10 / l00, l20 = a20 / l00;
  const double l11 = sqrt(a11 - l10 * l10);
  const double l21 = (a21 - l20 * l10) / l11;
  const double l22 = sqrt(a22 - l20 * l20 - l21 * l21);
  const double z0 = D[0] / l00;
  const double z1 = (D[1] - l10 * z0) / l11;
  const double z2 = (D[2] - l20 * z0 - l21 * z1) / l22;
  const double q = z0 * z0 + z1 * z1 + z2 * z2;
  q_out = q;
  const double g = exp(-0.5 * q);
  const double p = 0.5 - (double)m.adaptation_rate * g * (0.5 - sig_miss);
  return log(p / (1.0 - p));
}

// Whether voxel v holds at least ndt_min_samples samples (its ready bit).
__device__ __forceinline__ bool ndt_is_ready(const DevMap& m, size_t v) {
  return ((m.ndt_ready[v >> 5] >> (v & 31u)) & 1u) != 0u;
}

// Phase 1 over a tile of 256 rays, walked segment by segment (see
// ohm_walk_seg.h): the same per-voxel work as the occupancy walk, with the
// NDT-weighted miss increment (the hit samples' moments: ndt_hit_block).
// Two 512-thread blocks per CU (four waves per SIMD): the kernel is held to
// 128 VGPRs (the cold fp64 path of the queued misses spills) and the LDS
// table below to 2048 entries, so two blocks' LDS fit in a CU.
constexpr uint32_t kNdtMaxThreads = 512;

// Per-tile LDS table of the NDT walk's increments (see the occupancy walk's
// table): update id -> summed Q32.32 increment, two probes, laid out by
// 64-byte accumulator line (four voxels' miss and hit words: 8 ids per
// group).  The sums are exact integers, so the result does not depend on how
// updates reach the table.
constexpr int kNdtAggLog2 = 11;
constexpr uint32_t kNdtAggSize = 1u << kNdtAggLog2;
constexpr int kNdtAggLineLog2 = 3;
constexpr uint32_t kNdtAggLine = 1u << kNdtAggLineLog2;

__device__ __forceinline__ bool ndt_agg_add(uint32_t* keys, unsigned long long* vals, uint32_t id, long long q) {
  const uint32_t group = ((id >> kNdtAggLineLog2) * 0x9E3779B1u) >> (32 - (kNdtAggLog2 - kNdtAggLineLog2));
  uint32_t h = group * kNdtAggLine + id % kNdtAggLine;
  for (int p = 0; p < 2; ++p) {
    uint32_t k = keys[h];
    if (k == kAggEmpty) {
      const uint32_t old = atomicCAS(keys + h, kAggEmpty, id);
      k = old == kAggEmpty ? id : old;
    }
    if (k == id) {
      atomicAdd(vals + h, (unsigned long long)q);
      return true;
    }
    h = (h + kNdtAggLine) & (kNdtAggSize - 1);
  }
  return false;
}

// Apply a summed increment of one (voxel, kind): Q32.32 accumulators, or in
// per-update mode a miss lands at once by CAS.
template <bool kCount>
__device__ __forceinline__ void ndt_apply(const DevMap& m, uint32_t id, long long qs) {
  const size_t v = (size_t)(id >> 1);
  const bool is_hit = (id & 1u) != 0;
  if (kCount || is_hit) {
    atomicAdd(reinterpret_cast<unsigned long long*>(m.nacc + v * kNaccWords + (is_hit ? kNaccHit : kNaccMiss)),
              (unsigned long long)qs);
  } else {
    uint32_t* u = reinterpret_cast<uint32_t*>(m.occ + v);
    const float delta = (float)((double)qs * kInvQ32);
    uint32_t old = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
      const float nvv = fminf(fmaxf(__uint_as_float(old) + delta, m.l_min), m.l_max);
      const uint32_t prev = atomicCAS(u, old, __float_as_uint(nvv));
      if (prev == old) break;
      old = prev;
    }
  }
}

// A sample-weighted miss deferred to a full-wave batch: the fp64 Gaussian
// weight costs hundreds of instructions, and a wave that evaluated it for
// the few lanes needing it at each step would run it at a few percent lane
// occupancy.  Each wave queues such misses in LDS and evaluates 64 at once.
struct NdtPending {
  uint32_t id;     // update id (voxel << 1, a miss)
  int32_t k[3];    // voxel key
  uint32_t ray_t;  // tile-local ray
};

template <bool kCount, bool kWeighted, bool kTm>
__device__ __forceinline__ void ndt_drain(const DevMap& m, const NdtPending* pend, uint32_t n, uint32_t lane,
                                          const double od[3], const double (*ray_end)[kTileRays], const TileRays& tr,
                                          const float* __restrict__ weights, uint32_t r0, double sig_miss,
                                          uint32_t* agg_key, unsigned long long* agg_val) {
#pragma clang fp contract(off)
  __threadfence_block();  // the queue was written by other lanes of this wave
  if (lane < n) {
    const NdtPending e = pend[lane];
    double dv[3];
    double dd = 0.0;
    for (int a = 0; a < 3; ++a) {
      dv[a] = ray_end[a][e.ray_t] - od[a];
      dd = dd + dv[a] * dv[a];
    }
    const double wt = kWeighted ? (double)weights[(size_t)r0 + tr.src[e.ray_t]] : 1.0;
    const NdtVoxel nv = m.ndt[e.id >> 1];
    const double c[3] = {m.origin[0] + ((double)e.k[0] + 0.5) * m.voxel_size,
                         m.origin[1] + ((double)e.k[1] + 0.5) * m.voxel_size,
                         m.origin[2] + ((double)e.k[2] + 0.5) * m.voxel_size};
    double maha;
    const long long q = llrint(ndt_delta(m, od, dv, dd, c, nv, sig_miss, maha) * wt * kQ32);
    if (!ndt_agg_add(agg_key, agg_val, e.id, q)) ndt_apply<kCount>(m, e.id, q);
    // NDT-TM: the ray came close enough to the voxel's data to count as a miss
    if (kTm && maha <= m.tm_gate) atomicAdd(&m.tm[e.id >> 1].miss, 1u);
  }
}

// Sample moments of a scan's hits (each hit's occupancy increment is the
// walk's): each hit sample whose voxel lies in the key box [lo, hi) joins
// the voxel's per-scan moments and sample count, and for NDT-TM its
// intensity sums.  A hit block takes kHitBlockRays consecutive rays of the
// scan.  Neighbouring beams often end in one voxel (a block of 512 rays of
// a spinning lidar holds about a quarter as many distinct hit voxels as
// hits), so a block sums its hits per voxel in LDS and sends each voxel's
// totals to memory once: about a quarter of the fp64 atomics of adding
// every sample on its own, which otherwise bound the NDT pass.  The sums are
// fp64 in any order.  The NDT integration runs these blocks as extra blocks
// of the walk's launch, after its tiles, so that they fill the walk's tail;
// with kAllocate they claim the hit voxels' regions as the walk does
// (whichever comes first allocates).  The adjoint's statistics replay runs
// them in a launch of their own after its walk (ndt_hit_kernel).
constexpr uint32_t kHitBlockRays = 512;
constexpr uint32_t kHitThreads = 512;
constexpr int kHitTableLog2 = 9;
constexpr uint32_t kHitTableSize = 1u << kHitTableLog2;  // >= the block's rays: every hit voxel finds an entry
static_assert(kHitTableSize >= kHitBlockRays, "a block's hit voxels must all fit the table");

struct NdtHitSmem {
  uint32_t key[kHitTableSize];
  uint32_t cnt[kHitTableSize];
  double sum[11][kHitTableSize];  // x (3), x x^T (6), then intensity and its square (NDT-TM)
};

template <bool kWeighted, bool kTm, bool kAllocate>
__device__ void ndt_hit_block(const DevMap& m, NdtHitSmem& sh, const float* __restrict__ origins, uint32_t scan,
                              const float* __restrict__ samples, const float* __restrict__ weights,
                              const float* __restrict__ intensities, uint32_t r0, uint32_t n, const HitBox& box,
                              uint32_t blk) {
#pragma clang fp contract(off)
  constexpr int kSums = kTm ? 11 : 9;
  const uint32_t tid = threadIdx.x;
  for (uint32_t h = tid; h < kHitTableSize; h += blockDim.x) {
    sh.key[h] = kAggEmpty;
    sh.cnt[h] = 0u;
    for (int c = 0; c < kSums; ++c) sh.sum[c][h] = 0.0;
  }
  __syncthreads();
  const float o[3] = {origins[3 * (size_t)scan], origins[3 * (size_t)scan + 1], origins[3 * (size_t)scan + 2]};
  const uint32_t first = blk * kHitBlockRays;
  const uint32_t end = n - first < kHitBlockRays ? n : first + kHitBlockRays;
  for (uint32_t i = first + tid; i < end; i += blockDim.x) {
    const size_t ray = (size_t)r0 + i;
    const float e[3] = {samples[3 * ray], samples[3 * ray + 1], samples[3 * ray + 2]};
    // the same ray preparation and checks as the walk: a hit is a valid,
    // untruncated ray whose end voxel lies in the map, in an allocated region
    Ray r;
    int st = prepare_ray(m, o, e, r);
    if (kWeighted) {
      const float w = weights[ray];
      if (!(w >= 0.f) || !__builtin_isfinite(w)) st = kRayInvalid;
    }
    if (st != kRayOk || r.truncated) continue;
    bool inside = true;
    for (int a = 0; a < 3; ++a) inside = inside && r.k1[a] >= m.kmin[a] && r.k1[a] < m.kmax[a];
    for (int a = 0; a < 3; ++a) inside = inside && r.k1[a] >= box.lo[a] && r.k1[a] < box.hi[a];
    if (!inside) continue;
    // the hit voxel lies on the ray's path, so the walk claims its region too
    const int32_t ri = region_index(m, r.k1[0] >> kRegionLog2, r.k1[1] >> kRegionLog2, r.k1[2] >> kRegionLog2);
    const int32_t slot = kAllocate ? resolve_region<false>(m, ri, 0u, 0u)
                                   : __hip_atomic_load(m.table + ri, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (slot < 0) continue;  // the walk drops the hit too (pool exhausted)
    const uint32_t v = (uint32_t)slot * (uint32_t)kRegionVoxels + local_index(r.k1[0], r.k1[1], r.k1[2]);
    // voxel-centred sample: x = sample - centre
    double x[3];
    for (int a = 0; a < 3; ++a) x[a] = (double)e[a] - (m.origin[a] + ((double)r.k1[a] + 0.5) * m.voxel_size);
    double terms[kSums];
    terms[0] = x[0];
    terms[1] = x[1];
    terms[2] = x[2];
    terms[3] = x[0] * x[0];
    terms[4] = x[0] * x[1];
    terms[5] = x[0] * x[2];
    terms[6] = x[1] * x[1];
    terms[7] = x[1] * x[2];
    terms[8] = x[2] * x[2];
    if (kTm) {
      const double in = (double)intensities[ray];
      terms[kSums - 2] = in;
      terms[kSums - 1] = in * in;
    }
    // linear probing over the whole table: at most kHitTableSize distinct
    // voxels, so the probe always ends at the voxel's entry
    uint32_t h = (v * 0x9E3779B1u) >> (32 - kHitTableLog2);
    for (uint32_t p = 0; p < kHitTableSize; ++p) {
      uint32_t k = sh.key[h];
      if (k == kAggEmpty) {
        const uint32_t old = atomicCAS(sh.key + h, kAggEmpty, v);
        k = old == kAggEmpty ? v : old;
      }
      if (k == v) break;
      h = (h + 1u) & (kHitTableSize - 1u);
    }
    atomicAdd(sh.cnt + h, 1u);
    for (int c = 0; c < kSums; ++c) atomicAdd(&sh.sum[c][h], terms[c]);
  }
  __syncthreads();
  for (uint32_t h = tid; h < kHitTableSize; h += blockDim.x) {
    const uint32_t v = sh.key[h];
    if (v == kAggEmpty) continue;
    double* mo = m.mom + (size_t)v * kMomWords;
    for (int c = 0; c < 9; ++c) unsafeAtomicAdd(mo + c, sh.sum[c][h]);
    atomicAdd(m.nsamp + v, sh.cnt[h]);
    if (kTm) {
      unsafeAtomicAdd(m.tm_mom + 2 * (size_t)v, sh.sum[kSums - 2][h]);
      unsafeAtomicAdd(m.tm_mom + 2 * (size_t)v + 1, sh.sum[kSums - 1][h]);
    }
  }
}

// LDS of a walk tile; the launch's hit blocks use the same memory.
struct NdtWalkSmem {
  TileRays tr;
  RegionCache rc;
  double ray_end[3][kTileRays];  // world end point after truncation
  uint32_t agg_key[kNdtAggSize];
  unsigned long long agg_val[kNdtAggSize];
  NdtPending pend[kNdtMaxThreads / 64][64];
};
union NdtSmem {
  NdtWalkSmem w;
  NdtHitSmem h;
};

template <bool kCount, bool kWeighted, bool kTm>
__global__ __launch_bounds__(kNdtMaxThreads, 4) void ndt_seg_kernel(DevMap m, const float* __restrict__ origins, uint32_t scan,
                                                       const float* __restrict__ samples,
                                                       const float* __restrict__ weights,
                                                       const float* __restrict__ intensities, uint32_t r0, uint32_t n,
                                                       uint32_t n_tiles, int K, uint32_t tag, uint32_t parity,
                                                       double sig_miss) {
#pragma clang fp contract(off)
  __shared__ NdtSmem sm;
  if (blockIdx.x >= n_tiles) {
    // a hit block (after the tiles): the scan's hit samples
    const HitBox all = {{m.kmin[0], m.kmin[1], m.kmin[2]}, {m.kmax[0], m.kmax[1], m.kmax[2]}};
    ndt_hit_block<kWeighted, kTm, true>(m, sm.h, origins, scan, samples, weights, intensities, r0, n, all,
                                        blockIdx.x - n_tiles);
    return;
  }
  TileRays& tr = sm.w.tr;
  RegionCache& rc = sm.w.rc;
  double(*ray_end)[kTileRays] = sm.w.ray_end;
  uint32_t* agg_key = sm.w.agg_key;
  unsigned long long* agg_val = sm.w.agg_val;
  NdtPending(*pend)[64] = sm.w.pend;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = lane_id();
  // blocks < n_tiles are tiles; per-update mode (compare-and-swap) keeps the
  // round-robin deal over the XCDs, as the occupancy walk does
  const uint32_t tile0 = (kCount ? xcd_tile(blockIdx.x, n_tiles) : blockIdx.x) * kTileRays;
  const float* origin = origins + 3 * (size_t)scan;
  for (uint32_t h = tid; h < kNdtAggSize; h += blockDim.x) {
    agg_key[h] = kAggEmpty;
    agg_val[h] = 0ull;
  }
  TileRay t;
  RegionWindow rw;
  const uint32_t items =
      tile_prologue<kStageTouch>(m, tr, rc, rw, origin, samples, kWeighted ? weights : nullptr, nullptr, r0, n,
                                 tile0, K, tag, parity, t);
  if (t.ok)
    for (int a = 0; a < 3; ++a) ray_end[a][tid] = t.r.end[a];
  __syncthreads();
  const double od[3] = {(double)origin[0], (double)origin[1], (double)origin[2]};
  flush_tile_stats(m, t);
  uint32_t w_drop = 0, w_hit_drop = 0;  // this wave's dropped updates and hits (wave-uniform)
  uint32_t pend_n = 0;  // this wave's queued sample-weighted misses (wave-uniform)
  NdtPending* wpend = pend[tid >> 6];

  const uint32_t rounds = (items + blockDim.x - 1) / blockDim.x;
  for (uint32_t round = 0; round < rounds; ++round) {
    const uint32_t it = round * blockDim.x + tid;
    bool alive = it < items;
    uint32_t ray_t = 0;
    int M = 0;
    SegState s = {};
    double wt = 1.0;
    bool trunc = false;
    int32_t slot = -1;
    uint32_t lidx = 0;
    size_t ray = 0;
    double dv[3] = {0.0, 0.0, 0.0};
    double dd = 0.0;
    if (alive) {
      alive = tile_item(m, tr, it, K, s, ray_t, M);
      trunc = tr.trunc[ray_t] != 0;
      ray = (size_t)r0 + tr.src[ray_t];
      if (kWeighted) wt = (double)weights[ray];
      for (int a = 0; a < 3; ++a) {
        dv[a] = ray_end[a][ray_t] - od[a];
        dd = dd + dv[a] * dv[a];
      }
      if (alive) slot = staged_slot(m, rc, rw, s.k[0], s.k[1], s.k[2]);
      lidx = local_index(s.k[0], s.k[1], s.k[2]);
    }
    const long long q_plain = llrint((double)m.l_miss * wt * kQ32);
    // whether the voxel being visited holds enough samples for its Gaussian,
    // from the per-region bit mask (4 KB per region, cache-resident, where
    // the 40-byte statistics are not), loaded one step ahead so the load's
    // latency overlaps the previous voxel's update work.  (A second level of
    // 64 brick bits per region, kept in registers to skip the load in free
    // space, cost more in spilled registers than it saved: 16.4 against
    // 17.5 ms per NDT-OM pass without it.)
    bool ready = alive && slot >= 0 && ndt_is_ready(m, (size_t)slot * kRegionVoxels + lidx);
    while (__ballot(alive)) {
      const bool last = alive && s.w.total == 0;
      const bool is_hit = last && !trunc;
      const bool has = alive && slot >= 0;
      const int32_t k0 = s.k[0], k1 = s.k[1], k2 = s.k[2];  // this voxel (the walk steps on below)
      long long q = 0;
      // a miss whose increment the voxel's samples weight: queued, see NdtPending
      bool deferred = false;
      if (has) {
        if (is_hit) {
          q = llrint(wt * kQ32);
        } else if (ready) {
          deferred = true;
        } else {
          q = q_plain;
        }
      }
      const uint32_t id = has ? (((uint32_t)slot * (uint32_t)kRegionVoxels + lidx) << 1) | (is_hit ? 1u : 0u)
                              : (0xFFFFFFFFu - lane);
      const unsigned long long dropped = __ballot(alive && slot < 0);
      if (dropped) {
        w_drop += (uint32_t)__popcll(dropped);
        w_hit_drop += (uint32_t)__popcll(dropped & __ballot(is_hit));
      }
      if (alive) alive = !last && tile_advance<true>(m, rc, rw, s, M, slot, lidx);
      const bool ready_next = alive && slot >= 0 && ndt_is_ready(m, (size_t)slot * kRegionVoxels + lidx);
      const unsigned long long dmask = __ballot(deferred);
      if (dmask) {
        const uint32_t nd = (uint32_t)__popcll(dmask);
        if (pend_n + nd > 64u) {
          ndt_drain<kCount, kWeighted, kTm>(m, wpend, pend_n, lane, od, ray_end, tr, weights, r0, sig_miss, agg_key,
                                            agg_val);
          pend_n = 0;
        }
        if (deferred) {
          const uint32_t rank = (uint32_t)__popcll(dmask & ((1ull << lane) - 1ull));
          NdtPending e;
          e.id = id;
          e.k[0] = k0;
          e.k[1] = k1;
          e.k[2] = k2;
          e.ray_t = ray_t;
          wpend[pend_n + rank] = e;
        }
        pend_n += nd;
      }
      // runs are homogeneous (one voxel and kind: all deferred or none), so
      // the deferred lanes' runs just emit nothing here
      const LaneRuns run = lane_runs(id, lane);
      long long qs;
      bool emit;
      if (!kWeighted) {
        // every increment of a run is the same (unit weight, plain miss or hit)
        qs = (long long)run.len * q;
        emit = has && run.head && !deferred;
      } else {
        qs = segmented_sum(q, run.head, lane);
        emit = has && run.tail && !deferred;
      }
      if (emit && !ndt_agg_add(agg_key, agg_val, id, qs)) ndt_apply<kCount>(m, id, qs);
      // (the hit sample's moments are added by the launch's hit blocks)
      ready = ready_next;
    }
  }
  if (pend_n)
    ndt_drain<kCount, kWeighted, kTm>(m, wpend, pend_n, lane, od, ray_end, tr, weights, r0, sig_miss, agg_key,
                                      agg_val);
  __syncthreads();
  for (uint32_t h = tid; h < kNdtAggSize; h += blockDim.x) {
    const uint32_t k = agg_key[h];
    if (k != kAggEmpty) ndt_apply<kCount>(m, k, (long long)agg_val[h]);
  }
  drop_tile_stats(m, w_drop, w_hit_drop);
}

template <bool kWeighted, bool kTm>
__global__ __launch_bounds__(kHitThreads) void ndt_hit_kernel(DevMap m, const float* __restrict__ origins,
                                                              uint32_t scan, const float* __restrict__ samples,
                                                              const float* __restrict__ weights, uint32_t r0,
                                                              uint32_t n, HitBox box) {
  __shared__ NdtHitSmem sh;
  ndt_hit_block<kWeighted, kTm, false>(m, sh, origins, scan, samples, weights, nullptr, r0, n, box, blockIdx.x);
}

void launch_ndt_hits(const DevMap& m, hipStream_t st, const float* origins, uint32_t scan, const float* samples,
                     const float* weights, uint32_t r0, uint32_t n, HitBox box) {
  if (n == 0) return;
  const dim3 blocks((n + kHitBlockRays - 1) / kHitBlockRays);
  if (weights)
    hipLaunchKernelGGL((ndt_hit_kernel<true, false>), blocks, dim3(kHitThreads), 0, st, m, origins, scan, samples,
                       weights, r0, n, box);
  else
    hipLaunchKernelGGL((ndt_hit_kernel<false, false>), blocks, dim3(kHitThreads), 0, st, m, origins, scan, samples,
                       weights, r0, n, box);
}

// Recompute every ready bit from the sample counts (after ndt_min_samples
// changed).  Each wave covers 64 consecutive voxels, two mask words.
__global__ __launch_bounds__(256) void ndt_ready_rebuild_kernel(DevMap m) {
  const size_t nv = (size_t)m.capacity * kRegionVoxels;
  for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (size_t)gridDim.x * blockDim.x) {
    const bool ready = m.ndt[v].n >= m.ndt_min_samples;
    const unsigned long long bal = __ballot(ready);
    const uint32_t lane = lane_id();
    if ((lane & 31u) == 0u) m.ndt_ready[v >> 5] = (uint32_t)(bal >> lane);
  }
}

constexpr int kNdtChunk = 1024;
constexpr int kNdtUnits = kRegionVoxels / kNdtChunk;

__global__ __launch_bounds__(256) void ndt_finalize_kernel(DevMap m, uint32_t parity, int count_mode,
                                                           uint32_t scan_tag) {
#pragma clang fp contract(off)
  const uint32_t count = __hip_atomic_load(m.hdr + kHdrTouched0 + parity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t units = count * kNdtUnits;
  const double lmin = m.l_min, lmax = m.l_max;
  for (uint32_t unit = blockIdx.x; unit < units; unit += gridDim.x) {
    const uint32_t slot = m.touched[(size_t)parity * m.capacity + unit / kNdtUnits];
    const size_t base = (size_t)slot * kRegionVoxels + (size_t)(unit % kNdtUnits) * kNdtChunk;
    for (int j = threadIdx.x; j < kNdtChunk; j += blockDim.x) {
      const size_t v = base + j;
      longlong2* ap = reinterpret_cast<longlong2*>(m.nacc + v * kNaccWords);
      const longlong2 a01 = *ap;
      const uint32_t nb32 = m.nsamp[v];
      if (a01.x == 0 && a01.y == 0 && nb32 == 0) continue;
      const double miss = (double)a01.x * kInvQ32;
      const double hitw = (double)a01.y * kInvQ32;
      double l = (double)m.occ[v];
      double s = count_mode ? (l + hitw * (double)m.l_hit) + miss : l + hitw * (double)m.l_hit;
      if (m.clampscan && (s < lmin || s > lmax)) m.clampscan[v] = scan_tag;
      s = s < lmin ? lmin : (s > lmax ? lmax : s);
      const float lf = (float)s;
      m.occ[v] = lf;
      NdtVoxel nv = m.ndt[v];
      const bool was_ready = nv.n >= m.ndt_min_samples;
      bool dirty = false;
      if (lf < m.ndt_clear_below && nv.n != 0) {
        nv.n = 0;
        for (int c = 0; c < 3; ++c) nv.mean[c] = 0.f;
        for (int c = 0; c < 6; ++c) nv.cov[c] = 0.f;
        dirty = true;
        if (m.tm) m.tm[v] = TmVoxel{0u, 0.f, 0.f};
      }
      const long long nb = nb32;
      if (nb > 0 && m.tm) {
        // NDT-TM intensity Gaussian: pairwise merge of the scan's moments
        // with the stored mean and variance (count: the NDT sample count)
        double* im = m.tm_mom + 2 * v;
        TmVoxel tv = m.tm[v];
        const double na = (double)nv.n, nbd = (double)nb, nt = na + nbd;
        const double mb = im[0] / nbd;
        double vb = im[1] / nbd - mb * mb;
        vb = vb < 0.0 ? 0.0 : vb;
        const double d = mb - (double)tv.imean;
        tv.ivar = (float)((na * (double)tv.ivar + nbd * vb) / nt + d * d * (na * nbd / (nt * nt)));
        tv.imean = (float)((double)tv.imean + d * (nbd / nt));
        m.tm[v] = tv;
        im[0] = 0.0;
        im[1] = 0.0;
      }
      if (nb > 0) {
        double* mo = m.mom + v * kMomWords;
        const double inv = 1.0 / (double)nb;
        // scan statistics (metres): mean and population covariance
        double mub[3], cb[6];
        for (int c = 0; c < 3; ++c) mub[c] = mo[c] * inv;
        cb[0] = mo[3] * inv - mub[0] * mub[0];
        cb[1] = mo[4] * inv - mub[0] * mub[1];
        cb[2] = mo[5] * inv - mub[0] * mub[2];
        cb[3] = mo[6] * inv - mub[1] * mub[1];
        cb[4] = mo[7] * inv - mub[1] * mub[2];
        cb[5] = mo[8] * inv - mub[2] * mub[2];
        // pairwise merge with the stored statistics
        const double na = (double)nv.n, nbd = (double)nb, nt = na + nbd;
        double d[3];
        for (int c = 0; c < 3; ++c) d[c] = mub[c] - (double)nv.mean[c];
        const double f = na * nbd / (nt * nt);
        const int ii[6] = {0, 0, 0, 1, 1, 2};
        const int jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int c = 0; c < 6; ++c)
          nv.cov[c] = (float)((na * (double)nv.cov[c] + nbd * cb[c]) / nt + d[ii[c]] * d[jj[c]] * f);
        for (int c = 0; c < 3; ++c) nv.mean[c] = (float)((double)nv.mean[c] + d[c] * (nbd / nt));
        nv.n = nv.n + (uint32_t)nb;
        for (int c = 0; c < kMomWords; ++c) mo[c] = 0.0;
        dirty = true;
      }
      if (dirty) {
        m.ndt[v] = nv;
        const bool now_ready = nv.n >= m.ndt_min_samples;
        if (now_ready != was_ready) {
          uint32_t* w = m.ndt_ready + (v >> 5);
          if (now_ready) {
            atomicOr(w, 1u << (v & 31u));
          } else {
            atomicAnd(w, ~(1u << (v & 31u)));
          }
        }
      }
      *ap = make_longlong2(0, 0);
      if (nb32 != 0) m.nsamp[v] = 0u;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(m.hdr + kHdrTouched0 + (parity ^ 1u), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace ohm

using namespace ohm;

namespace {

template <bool kCount, bool kWeighted>
void launch_ndt_seg(const ohm_map_s* map, bool tm, dim3 tiles, dim3 threads, hipStream_t st, const float* origins,
                    uint32_t sc, const float* samples, const float* weights, const float* intensities, uint32_t r0,
                    uint32_t n, int K, uint32_t tag, uint32_t parity, double sig_miss) {
  // the walk's tiles, then the hit blocks
  const dim3 grid(tiles.x + (n + kHitBlockRays - 1) / kHitBlockRays);
  if (tm)
    hipLaunchKernelGGL((ndt_seg_kernel<kCount, kWeighted, true>), grid, threads, 0, st, map->dm, origins, sc, samples,
                       weights, intensities, r0, n, tiles.x, K, tag, parity, sig_miss);
  else
    hipLaunchKernelGGL((ndt_seg_kernel<kCount, kWeighted, false>), grid, threads, 0, st, map->dm, origins, sc,
                       samples, weights, intensities, r0, n, tiles.x, K, tag, parity, sig_miss);
}

// Both NDT entry points: intensities non-null exactly for NDT-TM maps.
ohm_status ndt_integrate_impl(ohm_map map, const float* d_origins, const float* d_samples, const float* d_intensities,
                              const uint32_t* h_scan_offsets, uint32_t n_scans, const float* d_weights,
                              void* stream) {
  const bool tm = d_intensities != nullptr;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const bool count_mode = map->params.mode == OHM_MODE_COUNT_CLAMP;
  const bool weighted = d_weights != nullptr;
  const double sig_miss = 1.0 / (1.0 + exp(-(double)map->params.l_miss));
  if (map->ndt_ready_stale) {
    hipLaunchKernelGGL(ndt_ready_rebuild_kernel, dim3(8192), dim3(256), 0, st, map->dm);
    map->ndt_ready_stale = false;
  }
  for (uint32_t sc = 0; sc < n_scans; ++sc) {
    const uint32_t r0 = h_scan_offsets[sc];
    const uint32_t n = h_scan_offsets[sc + 1] - r0;
    if (n == 0) continue;
    clear_pending(map, st);
    const uint32_t tag = ++map->count_batches;
    const uint32_t parity = tag & 1u;
    const dim3 tiles((n + kTileRays - 1) / kTileRays);
    const dim3 threads(map->walk_threads < kNdtMaxThreads ? map->walk_threads : kNdtMaxThreads);
    const int K = map->seg_major_steps;
    {
      ProfScope ps(map, OHM_KERNEL_WALK, st);
      if (count_mode) {
        if (weighted)
          launch_ndt_seg<true, true>(map, tm, tiles, threads, st, d_origins, sc, d_samples, d_weights, d_intensities,
                                     r0, n, K, tag, parity, sig_miss);
        else
          launch_ndt_seg<true, false>(map, tm, tiles, threads, st, d_origins, sc, d_samples, d_weights, d_intensities,
                                      r0, n, K, tag, parity, sig_miss);
      } else {
        if (weighted)
          launch_ndt_seg<false, true>(map, tm, tiles, threads, st, d_origins, sc, d_samples, d_weights, d_intensities,
                                      r0, n, K, tag, parity, sig_miss);
        else
          launch_ndt_seg<false, false>(map, tm, tiles, threads, st, d_origins, sc, d_samples, d_weights,
                                       d_intensities, r0, n, K, tag, parity, sig_miss);
      }
    }
    {
      ProfScope ps(map, OHM_KERNEL_NDT_HIT, st);
      hipLaunchKernelGGL(ndt_finalize_kernel, dim3(kFinalizeBlocks), dim3(256), 0, st, map->dm, parity,
                         count_mode ? 1 : 0, map->scans_done + 1);
    }
    map->scans_done += 1;
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? OHM_OK : OHM_E_HIP;
}

}  // namespace

extern "C" ohm_status ohm_ndt_integrate(ohm_map map, const float* d_origins, const float* d_samples,
                                        const uint32_t* h_scan_offsets, uint32_t n_scans, const float* d_weights,
                                        void* stream) {
  ohm_status s = check_scans(map, d_origins, d_samples, h_scan_offsets, n_scans);
  if (s != OHM_OK) return s;
  if (!map->dm.ndt || map->dm.tm) return OHM_E_INVALID_ARG;  // an NDT-TM map needs intensities
  if (n_scans == 0) return OHM_OK;
  return ndt_integrate_impl(map, d_origins, d_samples, nullptr, h_scan_offsets, n_scans, d_weights, stream);
}

extern "C" ohm_status ohm_ndt_tm_integrate(ohm_map map, const float* d_origins, const float* d_samples,
                                           const float* d_intensities, const uint32_t* h_scan_offsets,
                                           uint32_t n_scans, const float* d_weights, void* stream) {
  ohm_status s = check_scans(map, d_origins, d_samples, h_scan_offsets, n_scans);
  if (s != OHM_OK) return s;
  if (!map->dm.ndt || !map->dm.tm) return OHM_E_INVALID_ARG;
  if (n_scans == 0) return OHM_OK;
  if (!d_intensities && h_scan_offsets[n_scans] > h_scan_offsets[0]) return OHM_E_INVALID_ARG;
  return ndt_integrate_impl(map, d_origins, d_samples, d_intensities, h_scan_offsets, n_scans, d_weights, stream);
}
