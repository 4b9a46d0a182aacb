// Host-side map handle shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "ohm.h"
#include "ohm_device.h"

struct ohm_map_s {
  ohm_params params;
  ohm::DevMap dm;
  uint32_t layers;
  uint32_t group_slots;  // accumulator slots (1 without OHM_LAYER_SCAN_GROUPS)
  size_t regions;
  void* workspace;
  size_t workspace_bytes;
  int device;
  uint32_t count_batches;  // count-mode scans so far (tags and list parity)
  uint32_t scans_done;     // scans integrated since create / reset
  bool batched;            // a batched plan ran on the map since create / reset
  bool acc_dirty;          // the last count-mode scan's accumulators are still set
  bool ndt_ready_stale;    // ndt_min_samples changed since the NDT ready bits were last computed
  uint32_t last_parity;
  uint32_t kept_slot;      // accumulator slot holding those counts (scan groups), else 0
  bool kept_wide;          // ... as Q32.32 weight sums (a weighted scan), two f32 slots wide
  int seg_major_steps;     // walk tuning (ohm_map_set_tuning)
  uint32_t walk_threads;
  uint32_t column_rays;    // scans' column layout (ohm_map_set_scan_layout), 0: none
  // direction ordering of scans (ohm_map_set_ray_order): caller scratch
  uint32_t* order_hist;
  uint32_t* order_sums;
  uint32_t* order_perm;
  uint32_t order_max_rays;  // 0: scans walk in their given order
  // kernel timing (ohm_map_set_profiling)
  bool profiling;
  std::vector<hipEvent_t> event_pool;
  struct TimedLaunch {
    int kind;
    hipEvent_t start, stop;
  };
  std::vector<TimedLaunch> timed;
  size_t events_used;
};

namespace ohm {

constexpr int kFinalizeBlocks = 2048;
constexpr uint32_t kGroupSlots = 8;      // default accumulator slots of OHM_LAYER_SCAN_GROUPS
constexpr uint32_t kMaxGroupSlots = 64;  // most slots a map may ask for

// Accumulator slots a layer mask asks for: 1 without OHM_LAYER_SCAN_GROUPS,
// 0 when the mask is invalid.
inline uint32_t group_slots_of(uint32_t layers) {
  const uint32_t n = (layers >> 8) & 0xffu;
  if (!(layers & OHM_LAYER_SCAN_GROUPS)) return n ? 0u : 1u;
  if (n == 0) return kGroupSlots;
  return n <= kMaxGroupSlots ? n : 0u;
}
constexpr int kDefaultSegMajorSteps = 16;
constexpr uint32_t kMaxColumnRays = 65536;  // ohm_map_set_scan_layout
constexpr uint32_t kDefaultTileThreads = 512;

// kernels shared across translation units
__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v);
__global__ __launch_bounds__(256) void ndt_finalize_kernel(DevMap m, uint32_t parity, int count_mode,
                                                           uint32_t scan_tag);

// Direction-ordering scratch of the per-scan path: scans of at most
// max_rays rays walk in direction order (max_rays = 0: none do).
struct OrderScratch {
  uint32_t* hist;
  uint32_t* sums;
  uint32_t* perm;
  uint32_t max_rays;
};

// Bytes of direction-ordering scratch for scans of up to max_rays rays, and
// its three parts at base (256-byte aligned).
size_t order_scratch_bytes(uint32_t max_rays);
OrderScratch order_scratch_at(void* base, uint32_t max_rays);

ohm_status integrate_rays_impl(ohm_map map, const float* d_origins, const float* d_samples,
                               const uint32_t* h_scan_offsets, uint32_t n_scans, const float* d_weights,
                               hipStream_t st, const OrderScratch& ord, bool prof);

ohm_status map_initialise(ohm_map_s* map, hipStream_t st);
ohm_status check_scans(ohm_map map, const float* d_origins, const float* d_samples, const uint32_t* h_offsets,
                       uint32_t n_scans);
void clear_pending(ohm_map_s* map, hipStream_t st, bool prof = true);
// Add the hit samples of one scan (n rays from r0, origin `scan`) whose end
// voxels lie in `box` to the per-scan NDT moments and sample counts, after
// a walk of the scan that allocated their regions; weights (or null) as
// given to the walk.  (The NDT integration itself adds them in extra blocks
// of its walk launch; this is the adjoint's statistics replay.)
void launch_ndt_hits(const DevMap& m, hipStream_t st, const float* origins, uint32_t scan, const float* samples,
                     const float* weights, uint32_t r0, uint32_t n, HitBox box);
// Brackets one kernel launch with HIP events when profiling is enabled.
class ProfScope {
 public:
  ProfScope(ohm_map_s* map, int kind, hipStream_t st, bool on = true);
  ~ProfScope();

 private:
  ohm_map_s* map_;
  hipStream_t st_;
  int kind_;
  hipEvent_t stop_;
};

}  // namespace ohm
