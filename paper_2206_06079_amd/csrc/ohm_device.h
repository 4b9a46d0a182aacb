// Device-side definitions shared by the library's kernels: the map view that
// kernels receive by value, ray preparation (quantisation, truncation,
// validity) and the exact integer line walk.
//
// The walk is the Amanatides & Woo traversal the paper uses (Sec. III-B), in
// exact arithmetic: along each axis a the segment crosses voxel faces at ray
// parameters t = (b_a + j 2^S) / A_a (j = 0, 1, ...), with A_a = |q1_a - q0_a|
// and b_a the fixed-point distance from the start point to the first face.
// Comparing two axes' next crossings is the sign of N_a A_b - N_b A_a with
// N_a = b_a + j_a 2^S; the walk keeps the three pairwise differences as int64
// error terms and moves each by a constant when an axis steps, so every step
// is three compares and three adds.  Ties go to the lower axis.  With
// |q1 - q0| < 2^31 per axis all terms stay below 2^63.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ohm {

constexpr int kRegionLog2 = 5;
constexpr int kRegionEdge = 1 << kRegionLog2;
constexpr int kRegionMask = kRegionEdge - 1;
constexpr int kRegionVoxels = kRegionEdge * kRegionEdge * kRegionEdge;
constexpr uint32_t kMaxCapacity = 65534;  // keeps (slot * V + v) * 2 + 1 below the lane sentinels

enum : int32_t { kSlotEmpty = -1, kSlotClaimed = -2, kSlotExhausted = -3 };
enum : int { kRayOk = 0, kRayInvalid = 1, kRayOriginOob = 2 };

// header words at the start of the workspace
enum : int {
  kHdrPoolCount = 0,
  kHdrTouched0 = 1,
  kHdrTouched1 = 2,
  kHdrSticky = 3,
  kHdrBatchTag = 4,  // scan tag of the batched path (device-resident, survives graph replays)
  kHdrWords = 64
};
// sticky error bits (header word kHdrSticky)
enum : int32_t {
  kStickyPoolExhausted = 1,  // a region did not fit in the pool
  kStickySlotTimeout = 2,    // a region slot another block was publishing never appeared
  kStickyBadWeight = 4       // a ray weight was negative or not finite (the ray was skipped)
};
enum : int {
  kStatRays = 0,
  kStatInvalid,
  kStatOriginOob,
  kStatTruncated,
  kStatClipped,
  kStatHits,
  kStatUpdates,
  kStatDropped,
  kStatCount
};

struct NdtVoxel {       // 40 bytes, one per voxel of an NDT map
  uint32_t n;           // samples folded in
  float mean[3];        // metres, relative to the voxel centre
  float cov[6];         // xx, xy, xz, yy, yz, zz  (population covariance, m^2)
};

struct TmVoxel {      // 12 bytes, one per voxel of an NDT-TM map
  uint32_t miss;      // checked misses M (permeability H / (H + M), H = the NDT sample count)
  float imean;        // intensity mean of the voxel's samples
  float ivar;         // intensity population variance
};

struct DevMap {
  double origin[3];
  double scale;       // 2^F / voxel_size
  double voxel_size;
  double max_range;   // <= 0: none
  double max_range2;
  int32_t kmin[3], kmax[3];
  int32_t rlo[3], rdim[3];
  int32_t F;
  uint32_t capacity;
  float l_hit, l_miss, l_min, l_max, l_init;
  float sensor_noise, adaptation_rate, ndt_clear_below;
  uint32_t ndt_min_samples;
  uint32_t* hdr;
  unsigned long long* stats;
  int32_t* table;
  uint32_t* stamp;
  uint32_t* touched;  // [2][capacity]
  float* occ;         // [capacity][V]
  float* acc;         // [capacity][V][2]: miss weight, hit weight
  NdtVoxel* ndt;      // [capacity][V] or null
  uint32_t* ndt_ready;  // [capacity][V / 32]: bit set where the voxel holds >= ndt_min_samples samples
  long long* nacc;    // NDT per-scan accumulators [capacity][V][kNaccWords] or null
  uint32_t* nsamp;    // NDT per-scan sample counts [capacity][V] or null
  double* mom;        // NDT per-scan sample moments [capacity][V][kMomWords] or null
  uint32_t* clampscan;// [capacity][V] or null
  // voxel mean layer (or null): per voxel the packed 10-bit sub-voxel codes
  // (bits 0-29) and the sample count (bits 32-63); in count mode the per-scan
  // sample sums of slot j at mean_acc + 2 j capacity V (k | sum x << 32,
  // sum y | sum z << 32 per voxel) and a per-voxel mask of the slots holding
  // samples; mean_slot is the slot of the scan being walked
  unsigned long long* mean;
  unsigned long long* mean_acc;
  unsigned long long* mean_mask;
  uint32_t mean_slot;
  // decay-rate layer (or null): summed distance rays travel through each
  // voxel (Q32.32 metres) and the samples that fell in it
  unsigned long long* decay_len;
  uint32_t* decay_hits;
  // NDT-TM layer (or null): per voxel the checked misses and the intensity
  // Gaussian; per scan the intensity moments (sum i, sum i^2; fp64) of the
  // samples that fell in each voxel
  TmVoxel* tm;
  double* tm_mom;     // [capacity][V][2]
  double tm_gate;     // largest squared Mahalanobis distance of a checked miss
  // TSDF layer (or null): per voxel the distance D (bits 0-31) and weight W
  // (bits 32-63) as floats in one 64-bit word; per scan the Q32.32 sum of
  // the distances and the number of updates of each voxel
  unsigned long long* tsdf;
  long long* tsdf_acc;  // [capacity][V][2]
  double tsdf_tau, tsdf_wmax;
  // batched plans (or null): per region one 64-bit mask of the 8^3 bricks in
  // which the scan being walked left a non-zero count (the walk points it at
  // that scan's slot: [capacity] words per slot), so that the finalize skips
  // the slots a brick never received
  unsigned long long* brick_mask;
};

// Brick (8^3 voxels, 64 per region) of a region-local voxel index.
__host__ __device__ __forceinline__ uint32_t brick_of(uint32_t lidx) {
  return ((lidx >> 13) << 4) | (((lidx >> 8) & 3u) << 2) | ((lidx >> 3) & 3u);
}

// Q32.32 fixed point of the exact (order-independent) sums of weights and
// NDT increments: each term is rounded to a multiple of 2^-32 once, and the
// integer sums do not depend on the order the GPU adds them in.
constexpr double kQ32 = 4294967296.0;
constexpr double kInvQ32 = 1.0 / 4294967296.0;

// Floats per count-mode accumulator slot: [capacity][V] pairs (miss, hit),
// f32 counts for unit weights, int64 Q32.32 weight sums (wide) with weights.
__host__ __device__ __forceinline__ size_t acc_slot_floats(const DevMap& m, bool wide) {
  return (size_t)m.capacity * kRegionVoxels * (wide ? 4 : 2);
}

// u64 words per slot of the voxel mean layer's per-scan sums.
__host__ __device__ __forceinline__ size_t mean_slot_words(const DevMap& m) {
  return (size_t)m.capacity * kRegionVoxels * 2;
}

// The count-then-clamp update of one voxel from wide (Q32.32 weight sum)
// accumulators: s = (l + H l_hit) + M l_miss in fp64, recorded in the clamp
// layer (when present) if outside the clamp range, clamped, stored as float.
__device__ __forceinline__ float apply_wide(const DevMap& m, float l, long long miss_q, long long hit_q, size_t vi,
                                            uint32_t scan_tag) {
#pragma clang fp contract(off)
  const double hw = (double)hit_q * kInvQ32, mw = (double)miss_q * kInvQ32;
  const double lmin = m.l_min, lmax = m.l_max;
  double s = ((double)l + hw * (double)m.l_hit) + mw * (double)m.l_miss;
  if (m.clampscan && (s < lmin || s > lmax)) m.clampscan[vi] = scan_tag;
  s = s < lmin ? lmin : (s > lmax ? lmax : s);
  return (float)s;
}

// NDT per-scan accumulators, exact integers: summed miss increment and summed
// hit weight in Q32.32 fixed point, and the number of samples
constexpr int kNaccWords = 2;  // Q32.32 miss and hit sums (16 B: four voxels per 64-byte line)
enum : int { kNaccMiss = 0, kNaccHit = 1 };
// per-voxel sample moments of one scan: sum x (3), sum x x^T (6), x = sample
// minus voxel centre (metres)
constexpr int kMomWords = 9;

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

struct Ray {
  int64_t q0[3], q1[3];
  int32_t k0[3], k1[3];
  double end[3];  // world end point after truncation
  bool truncated;
};

// Quantise one coordinate to fixed point; false when unrepresentable.
__device__ __forceinline__ bool quantise(double p, double m, double scale, int64_t& q) {
#pragma clang fp contract(off)
  double x = (p - m) * scale;
  if (!(fabs(x) < 0x1p46)) return false;
  q = (int64_t)rint(x);
  return true;
}

// Validate, truncate and quantise one ray (origin o, sample e).
__device__ __forceinline__ int prepare_ray(const DevMap& m, const float o[3], const float e[3], Ray& r) {
#pragma clang fp contract(off)
  r.truncated = false;
  bool finite = true;
  for (int a = 0; a < 3; ++a) finite = finite && __builtin_isfinite(o[a]) && __builtin_isfinite(e[a]);
  if (!finite) return kRayInvalid;
  double end[3] = {(double)e[0], (double)e[1], (double)e[2]};
  if (m.max_range > 0.0) {
    double d0 = (double)e[0] - (double)o[0];
    double d1 = (double)e[1] - (double)o[1];
    double d2v = (double)e[2] - (double)o[2];
    double d2 = d0 * d0;
    d2 = d2 + d1 * d1;
    d2 = d2 + d2v * d2v;
    if (d2 > m.max_range2) {
      double f = m.max_range / __dsqrt_rn(d2);
      end[0] = (double)o[0] + d0 * f;
      end[1] = (double)o[1] + d1 * f;
      end[2] = (double)o[2] + d2v * f;
      r.truncated = true;
    }
  }
  for (int a = 0; a < 3; ++a) {
    r.end[a] = end[a];
    if (!quantise((double)o[a], m.origin[a], m.scale, r.q0[a]) || !quantise(end[a], m.origin[a], m.scale, r.q1[a]))
      return kRayInvalid;
    int64_t span = r.q1[a] - r.q0[a];
    if (span >= (int64_t(1) << 31) || -span >= (int64_t(1) << 31)) return kRayInvalid;
    r.k0[a] = (int32_t)(r.q0[a] >> m.F);
    r.k1[a] = (int32_t)(r.q1[a] >> m.F);
  }
  for (int a = 0; a < 3; ++a)
    if (r.k0[a] < m.kmin[a] || r.k0[a] >= m.kmax[a]) return kRayOriginOob;
  return kRayOk;
}

// Exact walk state at one level of detail: S = F for voxels, F + 5 for regions.
// walk_init and walk_step are pure integer code, callable on the host too.
struct Walk {
  int64_t dxy, dxz, dyz;   // pairwise error terms
  int64_t cx, cy, cz;      // A_a << S
  int32_t rem[3];          // crossings still to apply per axis
  int32_t total;           // sum of rem
  int32_t sg[3];           // step direction per axis
  uint32_t clip;           // bit a: axis a's last counted crossing leaves the bounds
};

// k0/k1 are the start/end cells at this level; lo/hi the inclusive cell
// bounds (hi inclusive) at this level.
__host__ __device__ __forceinline__ void walk_init(Walk& w, const int64_t q0[3], const int64_t q1[3], const int32_t k0[3],
                                          const int32_t k1[3], const int32_t lo[3], const int32_t hi[3], int S) {
  int64_t b[3], A[3];
  w.total = 0;
  w.clip = 0;
  for (int a = 0; a < 3; ++a) {
    int64_t D = q1[a] - q0[a];
    w.sg[a] = (D > 0) - (D < 0);
    A[a] = D < 0 ? -D : D;
    int32_t n = k1[a] - k0[a];
    n = n < 0 ? -n : n;
    b[a] = (w.sg[a] > 0) ? ((int64_t)(k0[a] + 1) << S) - q0[a] : q0[a] - ((int64_t)k0[a] << S);
    int32_t inb = (w.sg[a] > 0) ? (hi[a] - k0[a]) : (k0[a] - lo[a]);
    if (n > inb) {
      n = inb + 1;
      w.clip |= 1u << a;
    }
    w.rem[a] = n;
    w.total += n;
  }
  w.dxy = b[0] * A[1] - b[1] * A[0];
  w.dxz = b[0] * A[2] - b[2] * A[0];
  w.dyz = b[1] * A[2] - b[2] * A[1];
  w.cx = A[0] << S;
  w.cy = A[1] << S;
  w.cz = A[2] << S;
}

// Axis of the next crossing (ties to the lower axis).  Requires w.total > 0.
__host__ __device__ __forceinline__ int walk_pick(const Walk& w) {
  const bool ex = w.rem[0] > 0, ey = w.rem[1] > 0, ez = w.rem[2] > 0;
  const bool sx = ex && (!ey || w.dxy <= 0) && (!ez || w.dxz <= 0);
  const bool sy = !sx && ey && (!ez || w.dyz <= 0);
  return sx ? 0 : (sy ? 1 : 2);
}

// Apply the crossing of axis a: advance the error terms and the counts.
// (Two's-complement wrapping adds: a walk that has ended may be stepped on
// without meaning, and must not overflow.)
__host__ __device__ __forceinline__ void walk_apply(Walk& w, int a) {
  const bool sx = a == 0, sy = a == 1, sz = a == 2;
  w.dxy = (int64_t)((uint64_t)w.dxy + (uint64_t)(sx ? w.cy : (sy ? -w.cx : 0)));
  w.dxz = (int64_t)((uint64_t)w.dxz + (uint64_t)(sx ? w.cz : (sz ? -w.cx : 0)));
  w.dyz = (int64_t)((uint64_t)w.dyz + (uint64_t)(sy ? w.cz : (sz ? -w.cy : 0)));
  w.rem[0] -= sx ? 1 : 0;
  w.rem[1] -= sy ? 1 : 0;
  w.rem[2] -= sz ? 1 : 0;
  w.total -= 1;
}

// Pick and apply the next crossing; returns its axis.  Requires w.total > 0.
__host__ __device__ __forceinline__ int walk_step(Walk& w) {
  const int a = walk_pick(w);
  walk_apply(w, a);
  return a;
}

// The same walk with its error terms held in 32 bits, for the voxel loops.
// Every crossing moves a pairwise term d by a multiple of 2^S (A_a << S), so
// d's low S bits never change: c = ceil(d / 2^S) moves by A_a exactly, and
// d <= 0 exactly when c <= 0.  Along a walk the next crossings of two axes
// lie within one cell of each other in t, so |d| <= 2^S max_a A_a and
// |c| <= max_a A_a < 2^31 (ray preparation rejects spans of 2^31 or more).
// The loop then keeps three int32 terms and three int32 steps instead of
// six int64 values.
struct WalkH {
  int32_t exy, exz, eyz;   // ceil(d / 2^S) of the pairwise error terms
  int32_t ax, ay, az;      // A_a: what a crossing adds to or takes from them
  int32_t rem[3];          // crossings still to apply per axis
  int32_t total;           // sum of rem
  int32_t sg[3];           // step direction per axis
  uint32_t clip;           // bit a: axis a's last counted crossing leaves the bounds
};

__host__ __device__ __forceinline__ int32_t ceil_shift(int64_t d, int S) {
  return (int32_t)((d + (((int64_t)1 << S) - 1)) >> S);
}

__host__ __device__ __forceinline__ WalkH walk_half(const Walk& w, int S) {
  WalkH h;
  h.exy = ceil_shift(w.dxy, S);
  h.exz = ceil_shift(w.dxz, S);
  h.eyz = ceil_shift(w.dyz, S);
  h.ax = (int32_t)(w.cx >> S);
  h.ay = (int32_t)(w.cy >> S);
  h.az = (int32_t)(w.cz >> S);
  for (int a = 0; a < 3; ++a) {
    h.rem[a] = w.rem[a];
    h.sg[a] = w.sg[a];
  }
  h.total = w.total;
  h.clip = w.clip;
  return h;
}

__host__ __device__ __forceinline__ int walk_pick(const WalkH& w) {
  const bool ex = w.rem[0] > 0, ey = w.rem[1] > 0, ez = w.rem[2] > 0;
  const bool sx = ex && (!ey || w.exy <= 0) && (!ez || w.exz <= 0);
  const bool sy = !sx && ey && (!ez || w.eyz <= 0);
  return sx ? 0 : (sy ? 1 : 2);
}

// (Wrapping adds, as for Walk: an ended walk may be stepped on without meaning.)
__host__ __device__ __forceinline__ void walk_apply(WalkH& w, int a) {
  const bool sx = a == 0, sy = a == 1, sz = a == 2;
  w.exy = (int32_t)((uint32_t)w.exy + (uint32_t)(sx ? w.ay : (sy ? -w.ax : 0)));
  w.exz = (int32_t)((uint32_t)w.exz + (uint32_t)(sx ? w.az : (sz ? -w.ax : 0)));
  w.eyz = (int32_t)((uint32_t)w.eyz + (uint32_t)(sy ? w.az : (sz ? -w.ay : 0)));
  w.rem[0] -= sx ? 1 : 0;
  w.rem[1] -= sy ? 1 : 0;
  w.rem[2] -= sz ? 1 : 0;
  w.total -= 1;
}

__device__ __forceinline__ int32_t region_index(const DevMap& m, int32_t rx, int32_t ry, int32_t rz) {
  return ((rz - m.rlo[2]) * m.rdim[1] + (ry - m.rlo[1])) * m.rdim[0] + (rx - m.rlo[0]);
}

__device__ __forceinline__ uint32_t local_index(int32_t kx, int32_t ky, int32_t kz) {
  return ((uint32_t)(kz & kRegionMask) << (2 * kRegionLog2)) | ((uint32_t)(ky & kRegionMask) << kRegionLog2) |
         (uint32_t)(kx & kRegionMask);
}

// A box of voxel keys, [lo, hi) per axis.
struct HitBox {
  int32_t lo[3], hi[3];
};

// Slot of the region holding key k (negative when not allocated).
__device__ __forceinline__ int32_t lookup_slot(const DevMap& m, int32_t kx, int32_t ky, int32_t kz) {
  int32_t r = region_index(m, kx >> kRegionLog2, ky >> kRegionLog2, kz >> kRegionLog2);
  return __hip_atomic_load(m.table + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace ohm
