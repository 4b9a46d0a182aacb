// Optional per-voxel layers updated by the occupancy walk: the voxel mean
// layer and the decay-rate layer.
//
// Voxel mean (paper Sec. III-A: a 32-bit discretised mean position, 10 bits
// of sub-voxel position per axis, and a 32-bit sample count; updated by
// compare-and-swap like occupancy, Sec. III-B).  A sample's code per axis is
// its position inside its voxel in 1/1024 voxel, rounded down, taken from
// the quantised sample, so it is exact integer arithmetic.  Merging k
// samples with code sum S into (count n, code c) gives the rational mean
// (n c + S) / (n + k) rounded half up per axis and count n + k (saturated).
// The packed code and the count share one 64-bit word, so a per-update
// merge is one 64-bit compare-and-swap.  Count mode sums each scan's samples
// per voxel (exact integer atomics into the scan's slot, plus a mask bit for
// the slot) and merges the scan in one step in the finalize, in scan order.
//
// Decay rate (paper Sec. II-E): per voxel the summed distance rays travel
// through it and the samples that fell in it; the rate is their quotient.
// The distance of a visit is (t_exit - t_entry) L along the quantised
// segment, with the walk's own crossing parameters t = N_a / A_a
// (N_a = b_a + j 2^F) and the segment length L, summed as Q32.32 metres
// (integer atomics: the result does not depend on the order of the adds).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ohm_device.h"
#include "ohm_seg_math.h"

namespace ohm {

// ---------------------------------------------------------------------------
// voxel mean
// ---------------------------------------------------------------------------

// 10-bit sub-voxel code of fixed-point coordinate q (F fractional bits).
__device__ __forceinline__ uint32_t subvoxel_code(int64_t q, int F) {
  const int64_t f = q & (((int64_t)1 << F) - 1);  // q - floor(q / 2^F) 2^F
  return (uint32_t)(F >= 10 ? (f >> (F - 10)) : (f << (10 - F)));
}

__device__ __forceinline__ uint32_t pack_codes(const int64_t q[3], int F) {
  return subvoxel_code(q[0], F) | (subvoxel_code(q[1], F) << 10) | (subvoxel_code(q[2], F) << 20);
}

// Merge k samples with per-axis code sums sx, sy, sz into a mean word.
__device__ __forceinline__ unsigned long long mean_merge(unsigned long long word, uint64_t k, uint64_t sx,
                                                         uint64_t sy, uint64_t sz) {
  const uint64_t n = word >> 32;
  const uint32_t c = (uint32_t)word;
  const uint64_t tot = n + k;
  const uint64_t den = 2 * tot;
  const uint64_t s[3] = {sx, sy, sz};
  uint32_t out = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint64_t ca = (c >> (10 * a)) & 1023u;
    out |= (uint32_t)((2 * (n * ca + s[a]) + tot) / den) << (10 * a);
  }
  const uint64_t cnt = tot > 0xFFFFFFFFull ? 0xFFFFFFFFull : tot;
  return (cnt << 32) | out;
}

// One sample in voxel vi.  Count mode: add it to the scan's sums and mark
// the slot; per-update mode: merge it at once by compare-and-swap.
template <bool kCount>
__device__ __forceinline__ void mean_sample(const DevMap& m, size_t vi, uint32_t codes) {
  const uint64_t cx = codes & 1023u, cy = (codes >> 10) & 1023u, cz = (codes >> 20) & 1023u;
  if (kCount) {
    unsigned long long* a = m.mean_acc + 2 * vi;
    atomicAdd(a, 1ull | (cx << 32));
    atomicAdd(a + 1, cy | (cz << 32));
    atomicOr(m.mean_mask + vi, 1ull << m.mean_slot);
  } else {
    unsigned long long old = __hip_atomic_load(m.mean + vi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
      const unsigned long long nv = mean_merge(old, 1, cx, cy, cz);
      const unsigned long long prev = atomicCAS(m.mean + vi, old, nv);
      if (prev == old) break;
      old = prev;
    }
  }
}

// Count mode: merge the scans whose slots voxel vi's mask lists, in slot
// order, and clear their sums (slot_stride: u64 words between slots).
__device__ __forceinline__ void mean_finalize_voxel(const DevMap& m, size_t vi, size_t slot_stride) {
  unsigned long long mask = m.mean_mask[vi];
  if (!mask) return;
  unsigned long long word = m.mean[vi];
  while (mask) {
    const int j = __builtin_ctzll(mask);
    mask &= mask - 1;
    unsigned long long* a = m.mean_acc + (size_t)j * slot_stride + 2 * vi;
    const unsigned long long w0 = a[0], w1 = a[1];
    word = mean_merge(word, w0 & 0xFFFFFFFFull, w0 >> 32, w1 & 0xFFFFFFFFull, w1 >> 32);
    a[0] = 0ull;
    a[1] = 0ull;
  }
  m.mean[vi] = word;
  m.mean_mask[vi] = 0ull;
}

// ---------------------------------------------------------------------------
// decay rate
// ---------------------------------------------------------------------------

// Per-segment state of the distance measure: for each axis the numerator
// of the crossing parameter after its last crossing (N = nend - rem 2^F
// gives the next crossing's numerator from the walk's remaining count), the
// reciprocal of A_a, the segment length L and the current voxel's entry t.
struct DecayState {
  int64_t nend[3];
  double inv_a[3];
  double len;    // metres
  double t_in;   // entry parameter of the current voxel
};

// Set up at the start of segment `seg` of ray (q0, q1); s is the segment
// state from seg_init (its remaining counts).  M: the ray's major axis.
__device__ __forceinline__ void decay_init(DecayState& d, const DevMap& m, const int64_t q0[3], const int64_t q1[3],
                                           const SegState& s, int seg, int M) {
#pragma clang fp contract(off)
  const int S = m.F;
  const int32_t hi[3] = {m.kmax[0] - 1, m.kmax[1] - 1, m.kmax[2] - 1};
  int32_t k0[3], k1[3];
  for (int a = 0; a < 3; ++a) {
    k0[a] = (int32_t)(q0[a] >> S);
    k1[a] = (int32_t)(q1[a] >> S);
  }
  Walk w0;  // the ray's whole walk: its initial remaining counts R_a
  walk_init(w0, q0, q1, k0, k1, m.kmin, hi, S);
  int64_t A[3], b[3];
  int32_t n[3];
  crossing_geometry(q0, q1, S, A, b, n);
  double l2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    d.nend[a] = b[a] + ((int64_t)w0.rem[a] << S);
    d.inv_a[a] = A[a] > 0 ? 1.0 / (double)A[a] : 0.0;
    const double D = (double)(q1[a] - q0[a]);
    l2 = l2 + D * D;
  }
  d.len = sqrt(l2) * (m.voxel_size / (double)((int64_t)1 << S));
  d.t_in = 0.0;
  if (seg > 0) {
    // entered through the segment's boundary major crossing, the last one applied
    const int32_t remM = pick3(M, s.w.rem[0], s.w.rem[1], s.w.rem[2]);
    const int64_t N = pick3(M, d.nend[0], d.nend[1], d.nend[2]) - ((int64_t)(remM + 1) << S);
    d.t_in = (double)N * pick3(M, d.inv_a[0], d.inv_a[1], d.inv_a[2]);
  }
}

// Q32.32 distance through the current voxel (before the walk steps on), and
// move the entry parameter to its exit.  Requires the segment to be alive.
__device__ __forceinline__ long long decay_visit(DecayState& d, const DevMap& m, const SegState& s) {
#pragma clang fp contract(off)
  double t_out = 1.0;
  if (s.w.total > 0) {
    const int a = walk_pick(s.w);
    const int32_t ra = pick3(a, s.w.rem[0], s.w.rem[1], s.w.rem[2]);
    const int64_t N = pick3(a, d.nend[0], d.nend[1], d.nend[2]) - ((int64_t)ra << m.F);
    t_out = (double)N * pick3(a, d.inv_a[0], d.inv_a[1], d.inv_a[2]);
  }
  const long long q = llrint((t_out - d.t_in) * d.len * kQ32);
  d.t_in = t_out;
  return q < 0 ? 0 : q;
}

}  // namespace ohm
