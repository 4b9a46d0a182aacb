// Measurement helpers: the device's rate of independent atomic updates at a
// given footprint -- the ceilings the walks' voxel updates are compared with
// (the count walk applies one f32 atomic add per merged update into a
// region-chunked accumulator layer of about that size, the per-update walk
// one f32 clamp-add by compare-and-swap into the occupancy layer) -- and its
// streaming bandwidth (a copy, or a read alone).
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

// Every lane updates `iters` words of buf[0, n): pseudo-random words, or
// consecutive words across the wave when `sequential`.  kOp: 0 = f32
// atomic add of 1.0f, 1 = f32 clamp-add by compare-and-swap (retried until
// it lands, as the per-update walk does), 2 = u64 atomic add of 1.
template <int kOp>
__global__ __launch_bounds__(256) void atomic_rate_kernel(void* __restrict__ buf, uint32_t n, uint32_t iters,
                                                           int sequential) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t i = 0; i < iters; ++i) {
    const uint32_t h = (sequential ? tid + i * 977u : mix32(tid * 131u + i * 7919u)) % n;
    if (kOp == 0) {
      unsafeAtomicAdd(static_cast<float*>(buf) + h, 1.0f);
    } else if (kOp == 1) {
      uint32_t* u = static_cast<uint32_t*>(buf) + h;
      uint32_t old = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (;;) {
        const float nv = fminf(fmaxf(__uint_as_float(old) + 1.0f, -1e30f), 1e30f);
        const uint32_t prev = atomicCAS(u, old, __float_as_uint(nv));
        if (prev == old) break;
        old = prev;
      }
    } else {
      atomicAdd(static_cast<unsigned long long*>(buf) + h, 1ull);
    }
  }
}

// Stream n 16-byte words from src: copy them to dst, or (kReadOnly) fold
// them into a per-thread value that reaches dst only in the unlikely case
// that it equals a fixed pattern (so that no load can be dropped).  Four
// loads per thread are in flight per iteration; the grid strides the buffer.
template <bool kReadOnly>
__global__ __launch_bounds__(256) void stream_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                     size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t fold = 0;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride], v3 = src[i + 3 * stride];
    if (kReadOnly) {
      fold ^= v0.x ^ v0.y ^ v0.z ^ v0.w ^ v1.x ^ v1.y ^ v1.z ^ v1.w;
      fold ^= v2.x ^ v2.y ^ v2.z ^ v2.w ^ v3.x ^ v3.y ^ v3.z ^ v3.w;
    } else {
      dst[i] = v0;
      dst[i + stride] = v1;
      dst[i + 2 * stride] = v2;
      dst[i + 3 * stride] = v3;
    }
  }
  for (; i < n; i += stride) {
    const uint4 v = src[i];
    if (kReadOnly)
      fold ^= v.x ^ v.y ^ v.z ^ v.w;
    else
      dst[i] = v;
  }
  if (kReadOnly && fold == 0x9E3779B1u)
    dst[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = make_uint4(fold, 0u, 0u, 0u);
}

}  // namespace
}  // namespace ohm

extern "C" ohm_status ohm_probe_atomic_rate(void* d_buffer, size_t bytes, int flags, double* h_ops_per_s,
                                            void* stream) {
  const int op = (flags & OHM_PROBE_U64_ADD) ? 2 : ((flags & OHM_PROBE_F32_CAS) ? 1 : 0);
  const size_t word = op == 2 ? sizeof(unsigned long long) : sizeof(float);
  if (!d_buffer || !h_ops_per_s || bytes < word || bytes / word > 0xFFFFFFFFu) return OHM_E_INVALID_ARG;
  if (flags & ~(OHM_PROBE_SEQUENTIAL | OHM_PROBE_F32_CAS | OHM_PROBE_U64_ADD)) return OHM_E_INVALID_ARG;
  if ((flags & OHM_PROBE_F32_CAS) && (flags & OHM_PROBE_U64_ADD)) return OHM_E_INVALID_ARG;
  const uint32_t n = (uint32_t)(bytes / word);
  const int seq = (flags & OHM_PROBE_SEQUENTIAL) ? 1 : 0;
  const uint32_t blocks = 8192, iters = 64;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return OHM_E_HIP;
  }
  for (int rep = 0; rep < 2; ++rep) {  // the first launch warms up
    if (rep == 1) (void)hipEventRecord(a, st);
    if (op == 0)
      hipLaunchKernelGGL(ohm::atomic_rate_kernel<0>, dim3(blocks), dim3(256), 0, st, d_buffer, n, iters, seq);
    else if (op == 1)
      hipLaunchKernelGGL(ohm::atomic_rate_kernel<1>, dim3(blocks), dim3(256), 0, st, d_buffer, n, iters, seq);
    else
      hipLaunchKernelGGL(ohm::atomic_rate_kernel<2>, dim3(blocks), dim3(256), 0, st, d_buffer, n, iters, seq);
  }
  (void)hipEventRecord(b, st);
  float ms = 0.f;
  const bool ok = hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess && ms > 0.f;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (!ok || hipGetLastError() != hipSuccess) return OHM_E_HIP;
  *h_ops_per_s = (double)blocks * 256.0 * iters / ((double)ms * 1e-3);
  return OHM_OK;
}

extern "C" ohm_status ohm_probe_stream_rate(const void* d_src, void* d_dst, size_t bytes, int flags,
                                            double* h_bytes_per_s, void* stream) {
  // 4096 blocks of 256 threads: the read-only fold may write one word per
  // thread, 16 MiB in all, inside the required minimum size
  constexpr uint32_t kBlocks = 4096;
  constexpr size_t kMinBytes = (size_t)kBlocks * 256 * 16;
  if (!d_src || !d_dst || !h_bytes_per_s || bytes < kMinBytes || bytes % 16 != 0) return OHM_E_INVALID_ARG;
  if (((uintptr_t)d_src | (uintptr_t)d_dst) & 15u) return OHM_E_INVALID_ARG;
  if (flags & ~OHM_PROBE_READ_ONLY) return OHM_E_INVALID_ARG;
  const bool read_only = (flags & OHM_PROBE_READ_ONLY) != 0;
  const uint4* src = static_cast<const uint4*>(d_src);
  uint4* dst = static_cast<uint4*>(d_dst);
  const size_t n = bytes / 16;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return OHM_E_HIP;
  }
  for (int rep = 0; rep < 2; ++rep) {  // the first launch warms up
    if (rep == 1) (void)hipEventRecord(a, st);
    if (read_only)
      hipLaunchKernelGGL(ohm::stream_kernel<true>, dim3(kBlocks), dim3(256), 0, st, src, dst, n);
    else
      hipLaunchKernelGGL(ohm::stream_kernel<false>, dim3(kBlocks), dim3(256), 0, st, src, dst, n);
  }
  (void)hipEventRecord(b, st);
  float ms = 0.f;
  const bool ok = hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess && ms > 0.f;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (!ok || hipGetLastError() != hipSuccess) return OHM_E_HIP;
  *h_bytes_per_s = (double)bytes * (read_only ? 1.0 : 2.0) / ((double)ms * 1e-3);
  return OHM_OK;
}
