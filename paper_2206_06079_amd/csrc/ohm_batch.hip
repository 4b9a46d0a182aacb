// Batched integration: many scans of uneven size from several sensors, into
// several maps, replayed as one hipGraph launch.
//
// The scans of every set (one map each) are cut into groups of G consecutive
// scans per map.  One walk launch per group covers every ray of every scan of
// the group -- short scans share the GPU instead of each under-filling it --
// and each scan accumulates its own exact hit / miss counts into its own
// accumulator slot.  The group's finalize then applies, voxel by voxel, the
// group's scans in order, each with its own clamp, so the result is exactly
// the sequential per-scan count-then-clamp result.  The whole sequence is
// captured once into a graph; scan tags live in device memory so that every
// replay stays correct.
//
// Each replay first orders every scan's rays by direction (ohm_order.h):
// a histogram of direction bins per scan, an exclusive prefix per scan and
// a scatter give a permutation that the walk reads its rays through.  Scans
// of unordered directions then walk in coherent tiles; the voxels each ray
// updates do not change.  tuning->keep_ray_order skips this for scans that
// arrive in sensor order.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <new>
#include <vector>

#include "ohm.h"
#include "ohm_device.h"
#include "ohm_host.h"
#include "ohm_regions.h"
#include "ohm_wave.h"

#include "ohm_order.h"
#include "ohm_walk_seg.h"

namespace ohm {

constexpr uint32_t kBatchTagBase = 0x80000000u;  // batched tags never meet per-scan tags

struct BlockDesc {
  uint32_t set;    // scan set (map) index
  uint32_t pos;    // the scan's position within its group
  uint32_t scan;   // scan index within the set
  uint32_t r0;     // first ray of the scan
  uint32_t n;      // rays in the scan
  uint32_t block;  // block index within the scan
  uint32_t hbase;  // the scan's first direction bin in the plan's histogram
  uint32_t sbase;  // the scan's first strip in the plan's strip sums
};

struct ScanDesc {
  uint32_t sbase;   // first strip of the scan
  uint32_t strips;  // strips of the scan
};

struct SetPtrs {
  const float* origins;
  const float* samples;
  const float* weights;
  uint32_t* perm;  // walk order: perm[r0 + i] = scan index of the scan's i-th ray walked (null: given order)
};

// --- direction ordering (one block of 256 threads per 256 rays) ---

__global__ __launch_bounds__(256) void order_hist_kernel(const SetPtrs* __restrict__ sets,
                                                         const BlockDesc* __restrict__ descs,
                                                         uint32_t* __restrict__ hist) {
  const BlockDesc d = descs[blockIdx.x];
  const uint32_t i = d.block * kTileRays + threadIdx.x;
  if (i >= d.n) return;
  const SetPtrs sp = sets[d.set];
  order_count(sp.origins + 3 * (size_t)d.scan, sp.samples + 3 * (size_t)d.r0, d.n, kOrderStripRaysPlan, i,
              hist + d.hbase);
}

// one block per strip of every scan (strip s of the plan: bins [256 s, 256 s + 256))
__global__ __launch_bounds__(kOrderElevationBins) void order_strip_kernel(uint32_t* __restrict__ hist,
                                                                         uint32_t* __restrict__ sums) {
  order_strip_prefix(hist + (size_t)blockIdx.x * kOrderElevationBins, sums + blockIdx.x);
}

// one block per scan
__global__ __launch_bounds__(kOrderMaxStrips) void order_sums_kernel(const ScanDesc* __restrict__ scans,
                                                                     uint32_t* __restrict__ sums) {
  const ScanDesc sd = scans[blockIdx.x];
  order_scan_prefix(sums + sd.sbase, sd.strips);
}

__global__ __launch_bounds__(256) void order_scatter_kernel(const SetPtrs* __restrict__ sets,
                                                            const BlockDesc* __restrict__ descs,
                                                            uint32_t* __restrict__ hist,
                                                            const uint32_t* __restrict__ sums) {
  const BlockDesc d = descs[blockIdx.x];
  const uint32_t i = d.block * kTileRays + threadIdx.x;
  if (i >= d.n) return;
  const SetPtrs sp = sets[d.set];
  order_place(sp.origins + 3 * (size_t)d.scan, sp.samples + 3 * (size_t)d.r0, d.n, kOrderStripRaysPlan, i,
              hist + d.hbase,
              sums + d.sbase, sp.perm + d.r0);
}

template <bool kWeighted>
__global__ __launch_bounds__(1024) void batch_walk_kernel(const DevMap* __restrict__ maps,
                                                          const SetPtrs* __restrict__ sets,
                                                          const BlockDesc* __restrict__ descs, int K) {
  // blocks stay dealt round-robin over the XCDs (no xcd_tile): a plan's
  // launch mixes maps of different voxel sizes and scans of very different
  // lengths, and a contiguous eighth of it per XCD leaves the XCD holding the
  // finer map's tiles as the launch's tail (17 % slower on the 16-stream
  // workload, where the single-map walks gain 6-15 %)
  const BlockDesc d = descs[blockIdx.x];
  DevMap m = maps[d.set];
  m.acc += (size_t)d.pos * acc_slot_floats(m, kWeighted);
  m.brick_mask += (size_t)d.pos * m.capacity;
  const uint32_t tag = __hip_atomic_load(m.hdr + kHdrBatchTag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const SetPtrs sp = sets[d.set];
  walk_tile<kSinkCount, kWeighted, false, true, true>(m, sp.origins + 3 * (size_t)d.scan, sp.samples, sp.weights,
                                   sp.perm ? sp.perm + d.r0 : nullptr, d.r0, d.n,
                                   d.block * kTileRays, K, tag, tag & 1u, nullptr, nullptr, nullptr, nullptr);
}

// Applies the group's scans in order to every voxel of the regions the group
// touched: for j = 0..G-1, l = clamp((l + H_j l_hit) + M_j l_miss) (kWide:
// Q32.32 weight sums applied in fp64, as the per-scan path does).  Work goes
// by 8^3 brick: the brick masks the walk left say which scans' slots hold
// counts in the brick, and only those slots are read (a group's scans
// leave most of their slots' words zero).
template <bool kWide>
__global__ __launch_bounds__(256) void batch_finalize_kernel(const DevMap* __restrict__ maps, uint32_t n_sets,
                                                             uint32_t group) {
  __shared__ unsigned long long active_slots;
  for (uint32_t si = 0; si < n_sets; ++si) {
    const DevMap& m = maps[si];
    const uint32_t tag = __hip_atomic_load(m.hdr + kHdrBatchTag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t parity = tag & 1u;
    const uint32_t count = __hip_atomic_load(m.hdr + kHdrTouched0 + parity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t units = count * 64u;  // bricks
    const size_t stride = acc_slot_floats(m, kWide);
    for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
      const uint32_t slot = m.touched[(size_t)parity * m.capacity + u / 64u];
      const uint32_t brick = u % 64u;
      // the slots with counts in this brick: one wave, one slot per lane
      if (threadIdx.x < 64) {
        const bool has = threadIdx.x < group &&
                         ((m.brick_mask[(size_t)threadIdx.x * m.capacity + slot] >> brick) & 1ull) != 0ull;
        const unsigned long long bal = __ballot(has);
        if (threadIdx.x == 0) active_slots = bal;
      }
      __syncthreads();
      const unsigned long long act = active_slots;
      // brick origin within the region: x, y, z in steps of 8 (x fastest)
      const uint32_t b0 = ((brick >> 4) << 13) | (((brick >> 2) & 3u) << 8) | ((brick & 3u) << 3);
      for (uint32_t i = threadIdx.x; act && i < 512u; i += blockDim.x) {
        const size_t vi = (size_t)slot * kRegionVoxels + (b0 | (i & 7u) | (((i >> 3) & 7u) << 5) | ((i >> 6) << 10));
        float l = m.occ[vi];
        bool any = false;
        // the active slots' words are loaded kBatch at a time, all before
        // any of their clearing stores, so the loads overlap
        constexpr int kBatch = 8;
        unsigned long long rest = act;
        while (rest) {
          uint32_t js[kBatch];
#pragma unroll
          for (int q = 0; q < kBatch; ++q) {
            js[q] = rest ? (uint32_t)__builtin_ctzll(rest) : 0xFFFFFFFFu;
            rest &= rest ? rest - 1ull : 0ull;
          }
          if constexpr (kWide) {
            longlong2 a[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q)
              a[q] = js[q] != 0xFFFFFFFFu ? reinterpret_cast<const longlong2*>(m.acc + (size_t)js[q] * stride)[vi]
                                          : make_longlong2(0, 0);
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
              if (a[q].x == 0 && a[q].y == 0) continue;
              l = apply_wide(m, l, a[q].x, a[q].y, vi, 0u);  // (the plan's maps keep no clamp record)
              reinterpret_cast<longlong2*>(m.acc + (size_t)js[q] * stride)[vi] = make_longlong2(0, 0);
              any = true;
            }
          } else {
            float2 a[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q)
              a[q] = js[q] != 0xFFFFFFFFu ? reinterpret_cast<const float2*>(m.acc + (size_t)js[q] * stride)[vi]
                                          : make_float2(0.f, 0.f);
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
              if (a[q].x == 0.f && a[q].y == 0.f) continue;
              float s = __fadd_rn(l, __fmul_rn(a[q].y, m.l_hit));
              s = __fadd_rn(s, __fmul_rn(a[q].x, m.l_miss));
              l = fminf(fmaxf(s, m.l_min), m.l_max);
              reinterpret_cast<float2*>(m.acc + (size_t)js[q] * stride)[vi] = make_float2(0.f, 0.f);
              any = true;
            }
          }
        }
        if (any) m.occ[vi] = l;
      }
      __syncthreads();  // active_slots is rewritten by the next unit
    }
  }
}

// After a group's finalize: clear the brick masks of the regions it touched
// (one thread per region and slot).
__global__ __launch_bounds__(256) void batch_clear_masks_kernel(const DevMap* __restrict__ maps, uint32_t n_sets,
                                                                uint32_t group) {
  for (uint32_t si = 0; si < n_sets; ++si) {
    const DevMap& m = maps[si];
    const uint32_t tag = __hip_atomic_load(m.hdr + kHdrBatchTag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t parity = tag & 1u;
    const uint32_t count = __hip_atomic_load(m.hdr + kHdrTouched0 + parity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count * group; i += gridDim.x * blockDim.x) {
      const uint32_t slot = m.touched[(size_t)parity * m.capacity + i / group];
      m.brick_mask[(size_t)(i % group) * m.capacity + slot] = 0ull;
    }
  }
}

// Between groups: advance every set's batch tag and empty the touched list
// the next group will use.
__global__ void batch_advance_kernel(const DevMap* __restrict__ maps, uint32_t n_sets) {
  const uint32_t si = threadIdx.x;
  if (si >= n_sets) return;
  const DevMap& m = maps[si];
  const uint32_t tag = m.hdr[kHdrBatchTag] + 1u;
  m.hdr[kHdrBatchTag] = tag;
  m.hdr[kHdrTouched0 + (tag & 1u)] = 0u;
}

// End of a replay: empty both touched lists, so that a later per-scan call
// on the map (which expects the list of its scan's parity to start empty)
// does not append after this replay's last group.
__global__ void batch_end_kernel(const DevMap* __restrict__ maps, uint32_t n_sets) {
  const uint32_t si = threadIdx.x;
  if (si >= n_sets) return;
  const DevMap& m = maps[si];
  m.hdr[kHdrTouched0] = 0u;
  m.hdr[kHdrTouched1] = 0u;
}

// Start of a replay: empty both touched lists; start the tag sequence once.
__global__ void batch_begin_kernel(const DevMap* __restrict__ maps, uint32_t n_sets) {
  const uint32_t si = threadIdx.x;
  if (si >= n_sets) return;
  const DevMap& m = maps[si];
  if (m.hdr[kHdrBatchTag] < kBatchTagBase) m.hdr[kHdrBatchTag] = kBatchTagBase;
  m.hdr[kHdrTouched0] = 0u;
  m.hdr[kHdrTouched1] = 0u;
}

}  // namespace ohm

using namespace ohm;

struct ohm_batch_s {
  std::vector<ohm_map> maps;
  std::vector<uint32_t> nonempty;  // non-empty scans per set
  uint32_t n_sets;
  uint32_t group;
  uint32_t n_groups;
  int seg_major_steps;
  uint32_t tile_threads;
  bool weighted;
  bool order;  // direction-order the rays each run
  DevMap* d_maps;
  SetPtrs* d_sets;
  BlockDesc* d_descs;
  ScanDesc* d_scans;
  uint32_t* d_hist;
  uint32_t* d_sums;
  size_t hist_bins;
  uint32_t n_blocks, n_scans, n_strips;
  std::vector<uint32_t> group_first, group_blocks;
  hipStream_t capture;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace {

constexpr size_t kAlignB = 256;
inline size_t align_b(size_t v) { return (v + kAlignB - 1) & ~(kAlignB - 1); }

struct BatchLayout {
  size_t maps, sets, descs, scans, hist, sums, acc_total, total;
  std::vector<size_t> mask;  // per-set brick-mask offsets
  size_t hist_bins, strips;
  std::vector<size_t> acc;   // per-set accumulator offsets
  std::vector<size_t> perm;  // per-set walk-order offsets
  std::vector<BlockDesc> host_descs;
  std::vector<ScanDesc> host_scans;
  std::vector<uint32_t> group_first, group_blocks;
  uint32_t n_groups;
};

ohm_status plan_layout(const ohm_scan_set* sets, uint32_t n_sets, const ohm_batch_tuning* t, BatchLayout* L) {
  if (!sets || n_sets == 0 || n_sets > 64 || !t || t->group_scans == 0 || t->group_scans > 64)
    return OHM_E_INVALID_ARG;
  if (t->seg_major_steps > 4096) return OHM_E_INVALID_ARG;
  const bool order = t->keep_ray_order == 0;
  if (t->tile_threads != 0 && t->tile_threads != 256 && t->tile_threads != 512 && t->tile_threads != 1024)
    return OHM_E_INVALID_ARG;
  const uint32_t G = t->group_scans;
  bool weighted = sets[0].d_weights != nullptr;
  uint32_t max_scans = 0;
  for (uint32_t si = 0; si < n_sets; ++si) {
    const ohm_scan_set& s = sets[si];
    ohm_status st = check_scans(s.map, s.d_origins, s.d_samples, s.h_scan_offsets, s.n_scans);
    if (st != OHM_OK) return st;
    if (s.map->params.mode != OHM_MODE_COUNT_CLAMP) return OHM_E_UNSUPPORTED;
    if (s.map->dm.mean || s.map->dm.decay_len) return OHM_E_UNSUPPORTED;  // optional layers: per-scan path only
    if ((s.d_weights != nullptr) != weighted) return OHM_E_INVALID_ARG;
    for (uint32_t sj = 0; sj < si; ++sj)
      if (sets[sj].map == s.map) return OHM_E_INVALID_ARG;  // one set per map
    if (s.n_scans > max_scans) max_scans = s.n_scans;
  }
  L->n_groups = (max_scans + G - 1) / G;
  // direction bins of every non-empty scan (when ordering)
  // (strip s of the plan owns bins [256 s, 256 s + 256))
  std::vector<std::vector<uint32_t>> sbase(n_sets);
  L->host_scans.clear();
  size_t strips = 0;
  for (uint32_t si = 0; si < n_sets; ++si) {
    sbase[si].assign(sets[si].n_scans, 0u);
    for (uint32_t sc = 0; sc < sets[si].n_scans && order; ++sc) {
      const uint32_t n = sets[si].h_scan_offsets[sc + 1] - sets[si].h_scan_offsets[sc];
      if (n == 0) continue;
      const uint32_t ns = order_strips(n, kOrderStripRaysPlan);
      if ((strips + ns) * kOrderElevationBins > 0xFFFFFFFFull) return OHM_E_UNSUPPORTED;
      sbase[si][sc] = (uint32_t)strips;
      L->host_scans.push_back({(uint32_t)strips, ns});
      strips += ns;
    }
  }
  L->strips = strips;
  L->hist_bins = strips * kOrderElevationBins;
  L->host_descs.clear();
  L->group_first.assign(L->n_groups, 0);
  L->group_blocks.assign(L->n_groups, 0);
  for (uint32_t g = 0; g < L->n_groups; ++g) {
    L->group_first[g] = (uint32_t)L->host_descs.size();
    for (uint32_t si = 0; si < n_sets; ++si) {
      const ohm_scan_set& s = sets[si];
      for (uint32_t pos = 0; pos < G; ++pos) {
        const uint32_t sc = g * G + pos;
        if (sc >= s.n_scans) break;
        const uint32_t r0 = s.h_scan_offsets[sc];
        const uint32_t n = s.h_scan_offsets[sc + 1] - r0;
        for (uint32_t b = 0; b * (uint32_t)kTileRays < n; ++b)
          L->host_descs.push_back(
              {si, pos, sc, r0, n, b, sbase[si][sc] * kOrderElevationBins, sbase[si][sc]});
      }
    }
    L->group_blocks[g] = (uint32_t)L->host_descs.size() - L->group_first[g];
  }
  size_t off = 0;
  L->maps = off;
  off = align_b(off + n_sets * sizeof(DevMap));
  L->sets = off;
  off = align_b(off + n_sets * sizeof(SetPtrs));
  L->descs = off;
  off = align_b(off + L->host_descs.size() * sizeof(BlockDesc));
  L->scans = off;
  off = align_b(off + L->host_scans.size() * sizeof(ScanDesc));
  L->hist = off;
  off = align_b(off + L->hist_bins * sizeof(uint32_t));
  L->sums = off;
  off = align_b(off + L->strips * sizeof(uint32_t));
  L->perm.assign(n_sets, 0);
  for (uint32_t si = 0; si < n_sets && order; ++si) {
    L->perm[si] = off;
    off = align_b(off + (size_t)sets[si].h_scan_offsets[sets[si].n_scans] * sizeof(uint32_t));
  }
  L->acc.resize(n_sets);
  L->mask.resize(n_sets);
  for (uint32_t si = 0; si < n_sets; ++si) {
    L->acc[si] = off;
    off = align_b(off + (size_t)G * acc_slot_floats(sets[si].map->dm, weighted) * sizeof(float));
    L->mask[si] = off;
    off = align_b(off + (size_t)G * sets[si].map->dm.capacity * sizeof(unsigned long long));
  }
  L->total = off;
  return OHM_OK;
}

}  // namespace

extern "C" {

ohm_status ohm_batch_workspace_size(const ohm_scan_set* sets, uint32_t n_sets, const ohm_batch_tuning* tuning,
                                    size_t* bytes) {
  if (!bytes) return OHM_E_INVALID_ARG;
  BatchLayout L;
  ohm_status s = plan_layout(sets, n_sets, tuning, &L);
  if (s != OHM_OK) return s;
  *bytes = L.total;
  return OHM_OK;
}

ohm_status ohm_batch_create(const ohm_scan_set* sets, uint32_t n_sets, const ohm_batch_tuning* tuning,
                            void* d_workspace, size_t workspace_bytes, void* stream, ohm_batch* out) {
  if (!out) return OHM_E_INVALID_ARG;
  *out = nullptr;
  BatchLayout L;
  ohm_status s = plan_layout(sets, n_sets, tuning, &L);
  if (s != OHM_OK) return s;
  if (!d_workspace || ((uintptr_t)d_workspace & (kAlignB - 1))) return OHM_E_INVALID_ARG;
  if (workspace_bytes < L.total) return OHM_E_WORKSPACE_TOO_SMALL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  ohm_batch_s* b = new (std::nothrow) ohm_batch_s();
  if (!b) return OHM_E_INVALID_ARG;
  b->n_sets = n_sets;
  b->group = tuning->group_scans;
  b->seg_major_steps = tuning->seg_major_steps ? (int)tuning->seg_major_steps : kDefaultSegMajorSteps;
  b->tile_threads = tuning->tile_threads ? tuning->tile_threads : kDefaultTileThreads;
  b->n_groups = L.n_groups;
  b->weighted = sets[0].d_weights != nullptr;
  b->order = tuning->keep_ray_order == 0;
  b->hist_bins = L.hist_bins;
  b->n_blocks = (uint32_t)L.host_descs.size();
  b->n_scans = (uint32_t)L.host_scans.size();
  b->n_strips = (uint32_t)L.strips;
  b->group_first = L.group_first;
  b->group_blocks = L.group_blocks;
  char* base = static_cast<char*>(d_workspace);
  b->d_maps = reinterpret_cast<DevMap*>(base + L.maps);
  b->d_sets = reinterpret_cast<SetPtrs*>(base + L.sets);
  b->d_descs = reinterpret_cast<BlockDesc*>(base + L.descs);
  b->d_scans = reinterpret_cast<ScanDesc*>(base + L.scans);
  b->d_hist = reinterpret_cast<uint32_t*>(base + L.hist);
  b->d_sums = reinterpret_cast<uint32_t*>(base + L.sums);
  std::vector<DevMap> hm(n_sets);
  std::vector<SetPtrs> hs(n_sets);
  for (uint32_t si = 0; si < n_sets; ++si) {
    b->maps.push_back(sets[si].map);
    uint32_t ne = 0;
    for (uint32_t sc = 0; sc < sets[si].n_scans; ++sc)
      ne += sets[si].h_scan_offsets[sc + 1] > sets[si].h_scan_offsets[sc] ? 1u : 0u;
    b->nonempty.push_back(ne);
    hm[si] = sets[si].map->dm;
    hm[si].acc = reinterpret_cast<float*>(base + L.acc[si]);
    hm[si].brick_mask = reinterpret_cast<unsigned long long*>(base + L.mask[si]);
    hm[si].clampscan = nullptr;  // per-scan clamp records are kept by the per-scan path only
    hs[si] = {sets[si].d_origins, sets[si].d_samples, sets[si].d_weights,
              b->order ? reinterpret_cast<uint32_t*>(base + L.perm[si]) : nullptr};
  }
  bool ok = hipMemcpyAsync(b->d_maps, hm.data(), n_sets * sizeof(DevMap), hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(b->d_sets, hs.data(), n_sets * sizeof(SetPtrs), hipMemcpyHostToDevice, st) == hipSuccess;
  if (!L.host_descs.empty())
    ok = ok && hipMemcpyAsync(b->d_descs, L.host_descs.data(), L.host_descs.size() * sizeof(BlockDesc),
                              hipMemcpyHostToDevice, st) == hipSuccess;
  if (!L.host_scans.empty())
    ok = ok && hipMemcpyAsync(b->d_scans, L.host_scans.data(), L.host_scans.size() * sizeof(ScanDesc),
                              hipMemcpyHostToDevice, st) == hipSuccess;
  for (uint32_t si = 0; si < n_sets && ok; ++si) {
    const size_t nf = (size_t)b->group * acc_slot_floats(hm[si], b->weighted);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(8192), dim3(256), 0, st, reinterpret_cast<uint32_t*>(hm[si].acc), nf,
                       0u);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(256), dim3(256), 0, st, reinterpret_cast<uint32_t*>(hm[si].brick_mask),
                       (size_t)b->group * hm[si].capacity * 2, 0u);
  }
  // the host copies above must land before `hm` / `L` go out of scope
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  ok = ok && hipStreamCreate(&b->capture) == hipSuccess;
  if (!ok) {
    delete b;
    return OHM_E_HIP;
  }
  // capture the whole sequence
  ok = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    hipLaunchKernelGGL(batch_begin_kernel, dim3(1), dim3(64), 0, b->capture, b->d_maps, n_sets);
    if (b->order && b->n_scans) {
      // direction order of every scan (a fill kernel, not a memset: the graph is replayed)
      hipLaunchKernelGGL(fill_u32_kernel, dim3(8192), dim3(256), 0, b->capture, b->d_hist, b->hist_bins, 0u);
      hipLaunchKernelGGL(order_hist_kernel, dim3(b->n_blocks), dim3(kTileRays), 0, b->capture, b->d_sets,
                         b->d_descs, b->d_hist);
      hipLaunchKernelGGL(order_strip_kernel, dim3(b->n_strips), dim3(kOrderElevationBins), 0, b->capture, b->d_hist,
                         b->d_sums);
      hipLaunchKernelGGL(order_sums_kernel, dim3(b->n_scans), dim3(kOrderMaxStrips), 0, b->capture, b->d_scans,
                         b->d_sums);
      hipLaunchKernelGGL(order_scatter_kernel, dim3(b->n_blocks), dim3(kTileRays), 0, b->capture, b->d_sets,
                         b->d_descs, b->d_hist, b->d_sums);
    }
    for (uint32_t g = 0; g < b->n_groups; ++g) {
      if (b->group_blocks[g]) {
        if (b->weighted)
          hipLaunchKernelGGL(batch_walk_kernel<true>, dim3(b->group_blocks[g]), dim3(b->tile_threads), 0,
                             b->capture, b->d_maps, b->d_sets, b->d_descs + b->group_first[g], b->seg_major_steps);
        else
          hipLaunchKernelGGL(batch_walk_kernel<false>, dim3(b->group_blocks[g]), dim3(b->tile_threads), 0,
                             b->capture, b->d_maps, b->d_sets, b->d_descs + b->group_first[g], b->seg_major_steps);
      }
      if (b->weighted)
        hipLaunchKernelGGL(batch_finalize_kernel<true>, dim3(kFinalizeBlocks), dim3(256), 0, b->capture, b->d_maps,
                           n_sets, b->group);
      else
        hipLaunchKernelGGL(batch_finalize_kernel<false>, dim3(kFinalizeBlocks), dim3(256), 0, b->capture, b->d_maps,
                           n_sets, b->group);
      hipLaunchKernelGGL(batch_clear_masks_kernel, dim3(64), dim3(256), 0, b->capture, b->d_maps, n_sets, b->group);
      hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(64), 0, b->capture, b->d_maps, n_sets);
    }
    hipLaunchKernelGGL(batch_end_kernel, dim3(1), dim3(64), 0, b->capture, b->d_maps, n_sets);
    ok = hipStreamEndCapture(b->capture, &b->graph) == hipSuccess;
  }
  ok = ok && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    if (b->graph) (void)hipGraphDestroy(b->graph);
    (void)hipStreamDestroy(b->capture);
    delete b;
    return OHM_E_HIP;
  }
  *out = b;
  return OHM_OK;
}

ohm_status ohm_batch_run(ohm_batch b, void* stream) {
  if (!b) return OHM_E_INVALID_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (ohm_map m : b->maps) clear_pending(m, st);
  if (hipGraphLaunch(b->exec, st) != hipSuccess) return OHM_E_HIP;
  for (uint32_t si = 0; si < b->n_sets; ++si) {
    b->maps[si]->scans_done += b->nonempty[si];
    b->maps[si]->batched = true;  // no per-scan clamp record: the adjoint refuses the map
  }
  return OHM_OK;
}

ohm_status ohm_batch_destroy(ohm_batch b) {
  if (!b) return OHM_E_INVALID_ARG;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
  return OHM_OK;
}

}  // extern "C"
