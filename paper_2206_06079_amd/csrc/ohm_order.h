// Direction ordering of a scan's rays.  A walk tile is most efficient when
// its 256 rays point close together: they then share the voxels and regions
// near the sensor, adjacent lanes step through the same voxels (lane-run
// merging), and the tile stages few regions.  Scans that arrive in sensor
// order (a spinning lidar's columns) already are; scans of unordered
// directions are bucketed by direction first: azimuth strips of about 256
// rays (n / 256 strips), each cut into 256 elevation bins, strip-major.
// Only the order in which rays are walked changes, never which voxels they
// update.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ohm {

constexpr uint32_t kOrderElevationBins = 256;

// Azimuth strips of a scan of n rays.
__host__ __device__ __forceinline__ uint32_t order_strips(uint32_t n) { return n >= 512u ? n / 256u : 1u; }

// Bins of a scan of n rays.
__host__ __device__ __forceinline__ uint32_t order_bins(uint32_t n) { return order_strips(n) * kOrderElevationBins; }

// floor(x) clamped to [0, hi]; 0 for NaN.
__device__ __forceinline__ uint32_t bin_index(float x, uint32_t hi) {
  if (!(x >= 1.f)) return 0u;
  return x >= (float)hi ? hi : (uint32_t)x;
}

// Direction bin of the ray from o to e in a scan of n rays.
__device__ __forceinline__ uint32_t direction_key(const float o[3], const float e[3], uint32_t n) {
  const float dx = e[0] - o[0], dy = e[1] - o[1], dz = e[2] - o[2];
  const float kPi = 3.14159265358979f;
  const uint32_t strips = order_strips(n);
  const float az = atan2f(dy, dx);                        // [-pi, pi]
  const float el = atan2f(dz, sqrtf(dx * dx + dy * dy));  // [-pi/2, pi/2]
  const uint32_t s = bin_index((az + kPi) * ((float)strips / (2.f * kPi)), strips - 1u);
  const uint32_t b = bin_index((el + 0.5f * kPi) * ((float)kOrderElevationBins / kPi), kOrderElevationBins - 1u);
  return s * kOrderElevationBins + b;
}

}  // namespace ohm
