// Direction ordering of a scan's rays.  A walk tile is most efficient when
// its 256 rays point close together: they then share the voxels and regions
// near the sensor, adjacent lanes step through the same voxels (lane-run
// merging), and the tile stages few regions.  Scans that arrive in sensor
// order (a spinning lidar's columns) already are; scans of unordered
// directions are bucketed by direction first: azimuth strips of a given
// number of rays (n / strip_rays strips), each cut into 256 elevation bins,
// strip-major.  Only the order in which rays are walked changes, never which
// voxels they update.
//
// The batched plan cuts strips of eight tiles (kOrderStripRaysPlan): a tile
// then spans an eighth of the scan's elevation range across its strip's
// width, about square in angle for a scan over a 45-degree band (the
// spinning lidar: 32 columns by 8 beams).  A square patch of rays shares
// the most voxels: on such a scan a tile of 256 rays sees a distinct
// (voxel, hit or miss) pair per 17.3 updates, against 9.5 for a strip one
// tile wide, which is also what the sensor's own column order gives; and
// every distinct pair costs the tile one global atomic.  The per-scan path
// keeps strips one tile wide (kOrderStripRaysScan): its launches hold one
// scan's tiles, too few to even out the unequal lengths of square patches
// (a patch of upward beams is short, one down a tunnel long), while a strip
// holding every elevation gives tiles of about equal work.
//
// The bucketing is a counting sort in four parallel steps: count the rays of
// every bin; per strip (one 256-thread block each) turn its 256 bin counts
// into offsets within the strip; per scan (one block) turn the strip totals
// into strip offsets; place every ray at its strip offset plus the next free
// position of its bin.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ohm {

constexpr uint32_t kOrderElevationBins = 256;
constexpr uint32_t kOrderMaxStrips = 1024;
constexpr uint32_t kOrderStripRaysScan = 256;   // per-scan launches: one tile
constexpr uint32_t kOrderStripRaysPlan = 2048;  // batched plan: eight tiles

// Azimuth strips of a scan of n rays.
__host__ __device__ __forceinline__ uint32_t order_strips(uint32_t n, uint32_t strip_rays) {
  const uint32_t s = n / strip_rays;
  return s < 1u ? 1u : (s > kOrderMaxStrips ? kOrderMaxStrips : s);
}

// Bins of a scan of n rays.
__host__ __device__ __forceinline__ uint32_t order_bins(uint32_t n, uint32_t strip_rays) {
  return order_strips(n, strip_rays) * kOrderElevationBins;
}

// floor(x) clamped to [0, hi]; 0 for NaN.
__device__ __forceinline__ uint32_t bin_index(float x, uint32_t hi) {
  if (!(x >= 1.f)) return 0u;
  return x >= (float)hi ? hi : (uint32_t)x;
}

// Direction bin of the ray from o to e in a scan of n rays.
__device__ __forceinline__ uint32_t direction_key(const float o[3], const float e[3], uint32_t n,
                                                  uint32_t strip_rays) {
  const float dx = e[0] - o[0], dy = e[1] - o[1], dz = e[2] - o[2];
  const float kPi = 3.14159265358979f;
  const uint32_t strips = order_strips(n, strip_rays);
  const float az = atan2f(dy, dx);                        // [-pi, pi]
  const float el = atan2f(dz, sqrtf(dx * dx + dy * dy));  // [-pi/2, pi/2]
  const uint32_t s = bin_index((az + kPi) * ((float)strips / (2.f * kPi)), strips - 1u);
  const uint32_t b = bin_index((el + 0.5f * kPi) * ((float)kOrderElevationBins / kPi), kOrderElevationBins - 1u);
  return s * kOrderElevationBins + b;
}

// Count ray i of a scan (origin o, samples from the scan's first ray) in its
// direction bin.
__device__ __forceinline__ void order_count(const float* __restrict__ o, const float* __restrict__ samples,
                                            uint32_t n, uint32_t strip_rays, uint32_t i,
                                            uint32_t* __restrict__ hist) {
  const float oo[3] = {o[0], o[1], o[2]};
  const float e[3] = {samples[3 * (size_t)i + 0], samples[3 * (size_t)i + 1], samples[3 * (size_t)i + 2]};
  atomicAdd(hist + direction_key(oo, e, n, strip_rays), 1u);
}

// Inclusive scan over the block (blockDim.x a multiple of 64, at most 1024);
// `total` receives the block's sum.  Every thread must call it.
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t& total) {
  __shared__ uint32_t wave_sums[16];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t u = __shfl_up(v, off);
    if (lane >= (uint32_t)off) v += u;
  }
  if (lane == 63u) wave_sums[wave] = v;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) {
    const uint32_t ws = wave_sums[w];
    before += w < wave ? ws : 0u;
    all += ws;
  }
  __syncthreads();  // wave_sums may be reused by the next call
  total = all;
  return v + before;
}

// One block of kOrderElevationBins threads per strip: the strip's bin counts
// become offsets within the strip; the strip's total goes to *strip_sum.
__device__ __forceinline__ void order_strip_prefix(uint32_t* __restrict__ bins, uint32_t* __restrict__ strip_sum) {
  const uint32_t c = bins[threadIdx.x];
  uint32_t total;
  const uint32_t incl = block_inclusive_scan(c, total);
  bins[threadIdx.x] = incl - c;
  if (threadIdx.x == 0) *strip_sum = total;
}

// One block of kOrderMaxStrips threads per scan: strip totals become strip
// offsets.
__device__ __forceinline__ void order_scan_prefix(uint32_t* __restrict__ sums, uint32_t strips) {
  const uint32_t c = threadIdx.x < strips ? sums[threadIdx.x] : 0u;
  uint32_t total;
  const uint32_t incl = block_inclusive_scan(c, total);
  if (threadIdx.x < strips) sums[threadIdx.x] = incl - c;
}

// Place ray i of a scan: position = its strip's offset + the next free
// position of its bin within the strip; perm[position] = i.
__device__ __forceinline__ void order_place(const float* __restrict__ o, const float* __restrict__ samples,
                                            uint32_t n, uint32_t strip_rays, uint32_t i, uint32_t* __restrict__ hist,
                                            const uint32_t* __restrict__ strip_off, uint32_t* __restrict__ perm) {
  const float oo[3] = {o[0], o[1], o[2]};
  const float e[3] = {samples[3 * (size_t)i + 0], samples[3 * (size_t)i + 1], samples[3 * (size_t)i + 2]};
  const uint32_t key = direction_key(oo, e, n, strip_rays);
  perm[strip_off[key / kOrderElevationBins] + atomicAdd(hist + key, 1u)] = i;
}

}  // namespace ohm
