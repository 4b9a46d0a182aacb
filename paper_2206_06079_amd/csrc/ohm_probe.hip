// Measurement helper: the device's rate of independent f32 atomic adds at a
// given footprint -- the ceiling the walk's voxel updates are compared with
// (the walk applies one f32 atomic add per merged update into a
// region-chunked accumulator layer of about that size).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ohm.h"

namespace ohm {
namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// Every lane adds 1.0f to `iters` words of buf[0, n): pseudo-random words,
// or consecutive words across the wave when `sequential`.
__global__ __launch_bounds__(256) void atomic_rate_kernel(float* __restrict__ buf, uint32_t n, uint32_t iters,
                                                           int sequential) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t i = 0; i < iters; ++i) {
    const uint32_t h = sequential ? tid + i * 977u : mix32(tid * 131u + i * 7919u);
    unsafeAtomicAdd(buf + h % n, 1.0f);
  }
}

}  // namespace
}  // namespace ohm

extern "C" ohm_status ohm_probe_atomic_rate(void* d_buffer, size_t bytes, int sequential, double* h_ops_per_s,
                                            void* stream) {
  if (!d_buffer || !h_ops_per_s || bytes < sizeof(float) || bytes / sizeof(float) > 0xFFFFFFFFu)
    return OHM_E_INVALID_ARG;
  const uint32_t n = (uint32_t)(bytes / sizeof(float));
  const uint32_t blocks = 8192, iters = 64;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return OHM_E_HIP;
  }
  float* buf = static_cast<float*>(d_buffer);
  hipLaunchKernelGGL(ohm::atomic_rate_kernel, dim3(blocks), dim3(256), 0, st, buf, n, iters, sequential);  // warm-up
  (void)hipEventRecord(a, st);
  hipLaunchKernelGGL(ohm::atomic_rate_kernel, dim3(blocks), dim3(256), 0, st, buf, n, iters, sequential);
  (void)hipEventRecord(b, st);
  float ms = 0.f;
  const bool ok = hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess && ms > 0.f;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (!ok || hipGetLastError() != hipSuccess) return OHM_E_HIP;
  *h_ops_per_s = (double)blocks * 256.0 * iters / ((double)ms * 1e-3);
  return OHM_OK;
}
