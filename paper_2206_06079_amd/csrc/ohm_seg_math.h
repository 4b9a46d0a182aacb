// Closed-form segmentation of the exact voxel walk (pure integer code,
// callable on the host as well as in kernels).
//
// Each ray's canonical walk is cut into segments of K crossings of its major
// axis M (the axis with the largest extent).  Segment j starts right after
// major crossing c = jK - 1 and may apply K - 1 further major crossings
// (the last of kMaxLevels segments runs to the end of the ray).  The walk
// state at a segment start follows in closed form from the crossing
// parameters t_{b,i} = (b_b + i 2^S) / A_b: for every other axis b the
// number of its crossings applied before c is the number of i with
//   (b_b + i 2^S) A_M <  N_c A_b   (b after M in the tie order),
//   (b_b + i 2^S) A_M <= N_c A_b   (b before M),
// N_c = b_M + c 2^S, one exact 64-bit division.  Keys, error terms and
// remaining counts follow, so the concatenated segments reproduce the
// canonical walk voxel for voxel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ohm_device.h"

namespace ohm {

constexpr int kTileRays = 256;     // rays per block tile
constexpr int kMaxLevels = 32;     // segment levels per tile (the last one absorbs the rest)
constexpr int kMaxItems = kTileRays * kMaxLevels;

struct SegState {
  WalkH w;
  int32_t k[3];
  int32_t allowed;   // major crossings this segment may still apply
  uint32_t pos;      // index of the segment's first voxel in the ray's update list
  bool empty;        // the walk ended before the segment starts
};

// value i of three registers (kept as selects, never as an indexed stack load)
template <typename T>
__host__ __device__ __forceinline__ T pick3(int i, T a, T b, T c) {
  const T ab = i == 0 ? a : b;
  return i == 2 ? c : ab;
}

__host__ __device__ __forceinline__ int major_axis(const int64_t A[3]) {
  return (A[0] >= A[1] && A[0] >= A[2]) ? 0 : (A[1] >= A[2] ? 1 : 2);
}

// Crossings of axis `a` applied before the event "crossing of axis ae with
// numerator Ne" in the canonical order (ties: lower axis first), capped at n.
__host__ __device__ __forceinline__ int64_t crossings_before(int a, int ae, int64_t Ne, const int64_t A[3],
                                                    const int64_t b[3], const int32_t n[3], int S) {
  const int64_t Aa = pick3(a, A[0], A[1], A[2]);
  if (Aa == 0) return 0;
  const int64_t Ae = pick3(ae, A[0], A[1], A[2]);
  const int64_t ba = pick3(a, b[0], b[1], b[2]);
  const int64_t X = Ne * Aa - ba * Ae;
  const int64_t Y = Ae << S;
  const int64_t c = a < ae ? (X >= 0 ? X / Y + 1 : 0) : (X > 0 ? (X + Y - 1) / Y : 0);
  const int32_t na = pick3(a, n[0], n[1], n[2]);
  return c > na ? na : c;
}

// Per-axis crossing geometry of a prepared ray at resolution S.
__host__ __device__ __forceinline__ void crossing_geometry(const int64_t q0[3], const int64_t q1[3], int S, int64_t A[3],
                                                  int64_t b[3], int32_t n[3]) {
  for (int a = 0; a < 3; ++a) {
    const int64_t D = q1[a] - q0[a];
    A[a] = D < 0 ? -D : D;
    const int32_t k0 = (int32_t)(q0[a] >> S), k1 = (int32_t)(q1[a] >> S);
    b[a] = D > 0 ? ((int64_t)(k0 + 1) << S) - q0[a] : q0[a] - ((int64_t)k0 << S);
    const int32_t nn = k1 - k0;
    n[a] = nn < 0 ? -nn : nn;
  }
}

// Voxels the walk visits inside the map: all 1 + crossings when the end voxel
// is inside, else 1 + the crossings applied before the first exit.
__host__ __device__ __forceinline__ uint32_t walk_voxels(const Walk& w, const int64_t q0[3], const int64_t q1[3], int S) {
  if (w.clip == 0) return (uint32_t)w.total + 1u;
  int64_t A[3], b[3];
  int32_t n[3];
  crossing_geometry(q0, q1, S, A, b, n);
  int ae = -1;
  int64_t Ne = 0;
  for (int a = 0; a < 3; ++a) {
    if (!((w.clip >> a) & 1u)) continue;
    const int32_t ra = pick3(a, w.rem[0], w.rem[1], w.rem[2]);
    const int64_t ba = pick3(a, b[0], b[1], b[2]);
    const int64_t Aa = pick3(a, A[0], A[1], A[2]);
    const int64_t Na = ba + ((int64_t)(ra - 1) << S);
    if (ae < 0) {
      ae = a;
      Ne = Na;
    } else {
      const int64_t Ae = pick3(ae, A[0], A[1], A[2]);
      if (Na * Ae < Ne * Aa) {  // strictly earlier (ties keep the lower axis)
        ae = a;
        Ne = Na;
      }
    }
  }
  uint32_t v = 1u;
  for (int a = 0; a < 3; ++a) {
    if (a == ae) {
      const int32_t ra = pick3(a, w.rem[0], w.rem[1], w.rem[2]);
      v += (uint32_t)(ra - 1);
    } else {
      v += (uint32_t)crossings_before(a, ae, Ne, A, b, n, S);
    }
  }
  return v;
}

// Walk state at the start of segment `seg` (K major crossings per segment).
__host__ __device__ __forceinline__ void seg_init(SegState& s, const int64_t q0[3], const int64_t q1[3], const DevMap& m,
                                         int seg, int K) {
  const int S = m.F;
  const int32_t hi[3] = {m.kmax[0] - 1, m.kmax[1] - 1, m.kmax[2] - 1};
  int32_t k0[3], k1[3];
  for (int a = 0; a < 3; ++a) {
    k0[a] = (int32_t)(q0[a] >> S);
    k1[a] = (int32_t)(q1[a] >> S);
    s.k[a] = k0[a];
  }
  Walk w;  // the 64-bit form while the start state is computed
  walk_init(w, q0, q1, k0, k1, m.kmin, hi, S);
  s.allowed = seg + 1 == kMaxLevels ? 0x7fffffff : K - 1;  // the last level runs to the end
  s.pos = 0;
  s.empty = false;
  s.w = walk_half(w, S);
  if (seg == 0) return;
  int64_t A[3], b[3];
  int32_t n[3];
  crossing_geometry(q0, q1, S, A, b, n);
  const int M = major_axis(A);
  const int64_t c = (int64_t)seg * K - 1;  // the boundary's major crossing
  const int32_t remM = pick3(M, w.rem[0], w.rem[1], w.rem[2]);
  if (c >= remM || (((w.clip >> M) & 1u) && c + 1 == remM)) {
    s.empty = true;
    return;
  }
  const int64_t bM = pick3(M, b[0], b[1], b[2]);
  const int64_t Nc = bM + (c << S);
  int64_t cnt[3];
  uint32_t pos = 0;
  for (int a = 0; a < 3; ++a) {
    cnt[a] = a == M ? c + 1 : crossings_before(a, M, Nc, A, b, n, S);
    const int32_t ra = pick3(a, w.rem[0], w.rem[1], w.rem[2]);
    if (((w.clip >> a) & 1u) && cnt[a] >= ra) s.empty = true;  // left the map earlier
    pos += (uint32_t)cnt[a];
  }
  if (s.empty) return;
  int64_t N[3];
  for (int a = 0; a < 3; ++a) {
    N[a] = b[a] + (cnt[a] << S);
    s.k[a] = k0[a] + w.sg[a] * (int32_t)cnt[a];
  }
  w.rem[0] -= (int32_t)cnt[0];
  w.rem[1] -= (int32_t)cnt[1];
  w.rem[2] -= (int32_t)cnt[2];
  w.total -= (int32_t)pos;
  w.dxy = N[0] * A[1] - N[1] * A[0];
  w.dxz = N[0] * A[2] - N[2] * A[0];
  w.dyz = N[1] * A[2] - N[2] * A[1];
  s.w = walk_half(w, S);
  s.pos = pos;
}

// Number of segments of a ray (capped at kMaxLevels; the last level then runs
// to the end of the ray).
__host__ __device__ __forceinline__ uint32_t seg_count(const Walk& w, const int64_t q0[3], const int64_t q1[3], int K) {
  int64_t A[3];
  for (int a = 0; a < 3; ++a) {
    const int64_t D = q1[a] - q0[a];
    A[a] = D < 0 ? -D : D;
  }
  const int M = major_axis(A);
  const int32_t remM = pick3(M, w.rem[0], w.rem[1], w.rem[2]);
  const uint32_t n = 1u + (uint32_t)(remM / K);
  return n > (uint32_t)kMaxLevels ? (uint32_t)kMaxLevels : n;
}

// Move a segment walk one voxel on (requires s.w.total > 0).  Returns the
// axis stepped, with s.k updated, or -1 when the segment ends instead: its
// next step is a major crossing beyond its budget (the next segment's first),
// or the step leaves the map.  The step is applied either way (branch-free);
// after -1 the state is not used again.
__host__ __device__ __forceinline__ int seg_advance(SegState& s, int M) {
  const int a = walk_pick(s.w);
  const bool over_budget = a == M && s.allowed == 0;
  s.allowed -= a == M ? 1 : 0;
  walk_apply(s.w, a);
  const int32_t ra = pick3(a, s.w.rem[0], s.w.rem[1], s.w.rem[2]);
  const bool leaves = ra == 0 && ((s.w.clip >> a) & 1u);
  const int32_t sg = pick3(a, s.w.sg[0], s.w.sg[1], s.w.sg[2]);
  s.k[0] += a == 0 ? sg : 0;
  s.k[1] += a == 1 ? sg : 0;
  s.k[2] += a == 2 ? sg : 0;
  return (over_budget || leaves) ? -1 : a;
}

// A box holding every voxel of a segment (keys, inclusive), from its start
// state: the walk is monotone per axis, the segment applies at most
// K - 1 further crossings of the major axis M, and between two major
// crossings an axis b crosses at most ceil(A_b / A_M) + 1 times, so at most
// ceil(K A_b / A_M) + 1 times in the segment.  The last level (no budget)
// runs to the ray's end key (q1), which bounds it.
__host__ __device__ __forceinline__ void seg_bounds(const SegState& s, const int64_t q0[3], const int64_t q1[3],
                                                    int M, int K, bool last_level, int S, int32_t lo[3],
                                                    int32_t hi[3]) {
  int64_t A[3];
  for (int a = 0; a < 3; ++a) {
    const int64_t D = q1[a] - q0[a];
    A[a] = D < 0 ? -D : D;
  }
  const int64_t AM = pick3(M, A[0], A[1], A[2]);
  for (int a = 0; a < 3; ++a) {
    int64_t span;
    if (last_level || AM == 0) {
      const int32_t k1 = (int32_t)(q1[a] >> S);
      span = k1 > s.k[a] ? (int64_t)k1 - s.k[a] : (int64_t)s.k[a] - k1;
    } else if (a == M) {
      span = K - 1;
    } else {
      span = ((int64_t)K * A[a] + AM - 1) / AM + 1;
    }
    const int64_t end = (int64_t)s.k[a] + (int64_t)s.w.sg[a] * span;
    lo[a] = (int32_t)(end < s.k[a] ? end : s.k[a]);
    hi[a] = (int32_t)(end < s.k[a] ? s.k[a] : end);
  }
}

// Major axis of a prepared ray.
__host__ __device__ __forceinline__ int ray_major_axis(const int64_t q0[3], const int64_t q1[3]) {
  int64_t A[3];
  for (int a = 0; a < 3; ++a) {
    const int64_t D = q1[a] - q0[a];
    A[a] = D < 0 ? -D : D;
  }
  return major_axis(A);
}

}  // namespace ohm
