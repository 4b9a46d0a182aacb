// Host-side map handle shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ohm.h"
#include "ohm_device.h"

struct ohm_map_s {
  ohm_params params;
  ohm::DevMap dm;
  uint32_t layers;
  size_t regions;
  void* workspace;
  size_t workspace_bytes;
  int device;
  uint32_t count_batches;  // count-mode scans so far (tags and list parity)
  uint32_t scans_done;     // scans integrated since create / reset
  bool acc_dirty;          // the last count-mode scan's accumulators are still set
  uint32_t last_parity;
};

namespace ohm {

constexpr int kFinalizeBlocks = 2048;

ohm_status map_initialise(ohm_map_s* map, hipStream_t st);
ohm_status check_scans(ohm_map map, const float* d_origins, const float* d_samples, const uint32_t* h_offsets,
                       uint32_t n_scans);
void clear_pending(ohm_map_s* map, hipStream_t st);
void launch_prepass(ohm_map_s* map, const float* d_origins, uint32_t scan, const float* d_samples, uint32_t r0,
                    uint32_t n, bool touch, uint32_t tag, uint32_t parity, hipStream_t st);

}  // namespace ohm
