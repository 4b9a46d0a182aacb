// Adjoint of count-mode integration: gradients of a loss on the final
// log-odds with respect to the hit / miss increments, the NDT sensor noise
// and every ray's weight.
//
// Forward (per scan k, per voxel v): s = (l + H l_hit) + U, l <- clamp(s),
// with H the scan's summed hit weight and U its summed weighted miss
// increments; the map records c_v, the last scan whose s left the clamp
// range.  The clamp passes gradient only while inactive, so with
// G_v = dL/dl_v (final) every increment of scan k into v has gradient
// G_v [k > c_v].  The backward re-walks each ray (traversals are recomputed,
// never stored) and gathers
//     dL/dw_r      = sum_v G_v [k > c_v] delta_{r,v}          (no atomics)
//     dL/dl_hit    = sum_r w_r G_hit(r) [k > c]
//     dL/dl_miss   = sum_r w_r sum_miss G_v [k > c_v] d delta / d l_miss
//     dL/dsigma_n  = sum_r w_r sum_miss G_v [k > c_v] d delta / d sigma_n
// where an NDT-weighted miss delta = logit(p), p = 1/2 - lambda g (1/2 - s),
// g = exp(-q/2), q = D^T S^-1 D, S = Sigma + sigma_n^2 I, s = sigmoid(l_miss):
//     d delta / d l_miss  = lambda g s (1 - s) / (p (1 - p))
//     d delta / d sigma_n = -lambda (1/2 - s) g sigma_n |S^-1 D|^2 / (p (1 - p)).
// The NDT statistics each scan saw are replayed for the voxels whose
// statistics the gradient reads, those of the loss box (G_v = 0 elsewhere):
// their statistics are emptied, and scan k's gradient walk, which reads the
// statistics as they were before scan k, also adds each hit's sample that
// falls in the box to the voxel's moment accumulators, which a fold after the
// walk merges into the statistics for scan k + 1.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ohm.h"
#include "ohm_device.h"
#include "ohm_host.h"
#include "ohm_regions.h"
#include "ohm_walk_seg.h"
#include "ohm_wave.h"

namespace ohm {

namespace {

struct GradBox {
  const float* g;
  int32_t bmin[3], bdim[3];
};

__device__ __forceinline__ bool in_box(const GradBox& gb, int32_t x, int32_t y, int32_t z) {
  return (uint32_t)(x - gb.bmin[0]) < (uint32_t)gb.bdim[0] && (uint32_t)(y - gb.bmin[1]) < (uint32_t)gb.bdim[1] &&
         (uint32_t)(z - gb.bmin[2]) < (uint32_t)gb.bdim[2];
}

// Empty the NDT statistics of every voxel of the loss box (the ones the
// replay rebuilds); one thread per box voxel.
__global__ __launch_bounds__(256) void clear_box_stats_kernel(DevMap m, GradBox gb) {
  const size_t nbox = (size_t)gb.bdim[0] * gb.bdim[1] * gb.bdim[2];
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbox) return;
  const int32_t x = gb.bmin[0] + (int32_t)(i % (size_t)gb.bdim[0]);
  const int32_t y = gb.bmin[1] + (int32_t)((i / (size_t)gb.bdim[0]) % (size_t)gb.bdim[1]);
  const int32_t z = gb.bmin[2] + (int32_t)(i / ((size_t)gb.bdim[0] * gb.bdim[1]));
  if (x < m.kmin[0] || x >= m.kmax[0] || y < m.kmin[1] || y >= m.kmax[1] || z < m.kmin[2] || z >= m.kmax[2]) return;
  const int32_t slot = lookup_slot(m, x, y, z);
  if (slot < 0) return;
  m.ndt[(size_t)slot * kRegionVoxels + local_index(x, y, z)] = NdtVoxel{};
}

// What the gradient needs of one visited voxel, loaded together: its
// upstream gradient, clamp record and (NDT) sample count.  Voxels outside
// the loss box have zero gradient and load nothing.
struct VisitData {
  float G;
  uint32_t clamp;  // last scan whose pre-clamp value left the clamp range
  uint32_t n;      // NDT sample count
};

template <bool kNdt>
__device__ __forceinline__ VisitData visit_data(const DevMap& m, const GradBox& gb, bool alive, int32_t slot,
                                                uint32_t lidx, int32_t x, int32_t y, int32_t z) {
  VisitData d = {0.f, 0u, 0u};
  if (alive && slot >= 0 && in_box(gb, x, y, z)) {
    const size_t v = (size_t)slot * kRegionVoxels + lidx;
    d.G = gb.g[((size_t)(z - gb.bmin[2]) * gb.bdim[1] + (y - gb.bmin[1])) * gb.bdim[0] + (x - gb.bmin[0])];
    d.clamp = m.clampscan[v];
    if (kNdt) d.n = m.ndt[v].n;
  }
  return d;
}


// NDT miss increment and its derivatives with respect to l_miss and sigma_n.
__device__ void ndt_terms(const DevMap& m, const double o[3], const double d[3], double dd, const double c[3],
                          const NdtVoxel& nv, double sig_miss, double& delta, double& d_lm, double& d_sig) {
#pragma clang fp contract(off)
  double mu[3], w[3];
  double wd = 0.0;
  for (int a = 0; a < 3; ++a) {
    mu[a] = c[a] + (double)nv.mean[a];
    w[a] = mu[a] - o[a];
    wd = wd + w[a] * d[a];
  }
  double t = dd > 0.0 ? wd / dd : 0.0;
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  double D[3];
  for (int a = 0; a < 3; ++a) D[a] = (o[a] + t * d[a]) - mu[a];
  const double sn = m.sensor_noise, s2 = sn * sn;
  const double a00 = (double)nv.cov[0] + s2, a10 = nv.cov[1], a20 = nv.cov[2];
  const double a11 = (double)nv.cov[3] + s2, a21 = nv.cov[4], a22 = (double)nv.cov[5] + s2;
  // Cholesky S = L L^T; z = L^-1 D (q = |z|^2), y = L^-T z = S^-1 D
  const double l00 = sqrt(a00);
  const double l10 = a10 / l00, l20 = a20 / l00;
  const double l11 = sqrt(a11 - l10 * l10);
  const double l21 = (a21 - l20 * l10) / l11;
  const double l22 = sqrt(a22 - l20 * l20 - l21 * l21);
  const double z0 = D[0] / l00;
  const double z1 = (D[1] - l10 * z0) / l11;
  const double z2 = (D[2] - l20 * z0 - l21 * z1) / l22;
  const double y2 = z2 / l22;
  const double y1 = (z1 - l21 * y2) / l11;
  const double y0 = (z0 - l10 * y1 - l20 * y2) / l00;
  const double q = z0 * z0 + z1 * z1 + z2 * z2;
  const double yy = y0 * y0 + y1 * y1 + y2 * y2;
  const double g = exp(-0.5 * q);
  const double lam = m.adaptation_rate;
  const double p = 0.5 - lam * g * (0.5 - sig_miss);
  const double inv = 1.0 / (p * (1.0 - p));
  delta = log(p / (1.0 - p));
  d_lm = lam * g * sig_miss * (1.0 - sig_miss) * inv;
  d_sig = -lam * (0.5 - sig_miss) * g * sn * yy * inv;
}

constexpr uint32_t kBackwardMaxThreads = 512;  // keeps the kernel within its registers

// A miss in a voxel with enough samples, whose fp64 NDT terms are evaluated
// with 63 others by the whole wave instead of by the few lanes that meet one
// at a given step.
struct BwdPending {
  uint32_t v;      // voxel index (slot * 32^3 + local)
  int32_t k[3];    // voxel key
  uint32_t ray_t;  // tile-local ray
  float G;         // dL/dl of the voxel
};

__device__ __forceinline__ void bwd_drain(const DevMap& m, const BwdPending* pend, uint32_t n, uint32_t lane,
                                          const double od[3], const double (*ray_end)[kTileRays], double* ray_gw,
                                          const TileRays& tr, const float* __restrict__ weights, uint32_t r0,
                                          double sig_miss, bool weighted, double& g_miss, double& g_sig) {
#pragma clang fp contract(off)
  __threadfence_block();  // the queue was written by other lanes of this wave
  if (lane < n) {
    const BwdPending e = pend[lane];
    double dv[3];
    double dd = 0.0;
    for (int a = 0; a < 3; ++a) {
      dv[a] = ray_end[a][e.ray_t] - od[a];
      dd = dd + dv[a] * dv[a];
    }
    const double wt = weighted ? (double)weights[(size_t)r0 + tr.src[e.ray_t]] : 1.0;
    const NdtVoxel nv = m.ndt[e.v];
    const double c[3] = {m.origin[0] + ((double)e.k[0] + 0.5) * m.voxel_size,
                         m.origin[1] + ((double)e.k[1] + 0.5) * m.voxel_size,
                         m.origin[2] + ((double)e.k[2] + 0.5) * m.voxel_size};
    double delta, dlm, dsg;
    ndt_terms(m, od, dv, dd, c, nv, sig_miss, delta, dlm, dsg);
    const double Gd = (double)e.G;
    atomicAdd(&ray_gw[e.ray_t], Gd * delta);
    g_miss += wt * Gd * dlm;
    g_sig += wt * Gd * dsg;
  }
}

// One tile of 256 rays, walked segment by segment (see ohm_walk_seg.h).  A
// ray's weight gradient is the sum over its segments (fp64 LDS atomics);
// the scalar gradients are reduced per block.  `tag` is the scan's 1-based
// index (compared with the clamp record); with kNdt the touched regions are
// listed under (fold_tag, fold_parity) for the statistics replay that
// follows (the scan's hit samples in the box, then the fold).
template <bool kNdt, bool kWeighted>
__global__ __launch_bounds__(kBackwardMaxThreads, 4) void backward_seg_kernel(
    DevMap m, GradBox gb, const float* __restrict__ origins, uint32_t scan, const float* __restrict__ samples,
    const float* __restrict__ weights, uint32_t r0, uint32_t n, int K, uint32_t tag, uint32_t fold_tag,
    uint32_t fold_parity, float* __restrict__ grad_w, double* __restrict__ grad_s, double sig_miss) {
#pragma clang fp contract(off)
  __shared__ TileRays tr;
  __shared__ RegionCache rc;
  __shared__ double ray_end[3][kTileRays];
  __shared__ double ray_gw[kTileRays];
  __shared__ BwdPending pend[kBackwardMaxThreads / 64][64];
  const uint32_t tid = threadIdx.x;
  const uint32_t tile0 = xcd_tile(blockIdx.x, gridDim.x) * kTileRays;
  const float* origin = origins + 3 * (size_t)scan;
  TileRay t;
  RegionWindow rw;
  const uint32_t items =
      tile_prologue<kNdt ? kStageTouch : kStageResolve>(m, tr, rc, rw, origin, samples, kWeighted ? weights : nullptr,
                                                        nullptr, r0, n, tile0, K, fold_tag, fold_parity, t);
  if (tid < (uint32_t)kTileRays) {
    ray_gw[tid] = 0.0;
    if (t.ok)
      for (int a = 0; a < 3; ++a) ray_end[a][tid] = t.r.end[a];
  }
  __syncthreads();
  const double od[3] = {(double)origin[0], (double)origin[1], (double)origin[2]};
  double g_hit = 0.0, g_miss = 0.0, g_sig = 0.0;
  const uint32_t lane = lane_id();
  BwdPending* wpend = pend[tid >> 6];
  uint32_t pend_n = 0;  // this wave's queued sample-weighted misses (wave-uniform)

  // segment walks, one item per thread per round; the waves step in lockstep
  // so that misses needing the fp64 NDT terms can be evaluated 64 at a time
  const uint32_t rounds = (items + blockDim.x - 1) / blockDim.x;
  for (uint32_t round = 0; round < rounds; ++round) {
    const uint32_t it = round * blockDim.x + tid;
    bool alive = it < items;
    uint32_t ray_t = 0;
    int M = 0;
    SegState s = {};
    bool trunc = false;
    double wt = 1.0;
    int32_t slot = -1;
    uint32_t lidx = 0;
    if (alive) {
      uint32_t level = 0;
      alive = tile_item(m, tr, it, K, s, ray_t, M, &level);
      if (alive) {
        // a segment whose voxels all lie outside the loss box contributes
        // nothing (zero upstream gradient there, and no replayed sample)
        const int64_t q0[3] = {tr.q0[0], tr.q0[1], tr.q0[2]};
        const int64_t q1[3] = {tr.q1[0][ray_t], tr.q1[1][ray_t], tr.q1[2][ray_t]};
        int32_t lo[3], hi[3];
        seg_bounds(s, q0, q1, M, K, level + 1 == (uint32_t)kMaxLevels, m.F, lo, hi);
        for (int a = 0; a < 3; ++a)
          alive = alive && hi[a] >= gb.bmin[a] && lo[a] < gb.bmin[a] + gb.bdim[a];
      }
      trunc = tr.trunc[ray_t] != 0;
      if (kWeighted) wt = (double)weights[(size_t)r0 + tr.src[ray_t]];
      slot = staged_slot(m, rc, rw, s.k[0], s.k[1], s.k[2]);
      lidx = local_index(s.k[0], s.k[1], s.k[2]);
    }
    double gw = 0.0;
    // the current voxel's gradient data, loaded one step ahead so the loads'
    // latency overlaps the previous voxel's work
    VisitData vd = visit_data<kNdt>(m, gb, alive, slot, lidx, s.k[0], s.k[1], s.k[2]);
    while (__ballot(alive)) {
      bool deferred = false;
      const float G = vd.G;
      size_t v = 0;
      const int32_t k0 = s.k[0], k1 = s.k[1], k2 = s.k[2];
      bool last = false;
      if (alive) {
        last = s.w.total == 0;
        const bool is_hit = last && !trunc;
        if (G != 0.f && slot >= 0) {
          v = (size_t)slot * kRegionVoxels + lidx;
          if (tag > vd.clamp) {
            const double Gd = (double)G;
            if (is_hit) {
              gw += Gd * (double)m.l_hit;
              g_hit += wt * Gd;
            } else if (kNdt && vd.n >= m.ndt_min_samples) {
              deferred = true;
            } else {
              gw += Gd * (double)m.l_miss;
              g_miss += wt * Gd;
            }
          }
        }
        alive = !last && tile_advance<true>(m, rc, rw, s, M, slot, lidx);
        if (!alive && gw != 0.0) atomicAdd(&ray_gw[ray_t], gw);
      }
      vd = visit_data<kNdt>(m, gb, alive, slot, lidx, s.k[0], s.k[1], s.k[2]);
      if (kNdt) {
        const unsigned long long dmask = __ballot(deferred);
        if (dmask) {
          const uint32_t nd = (uint32_t)__popcll(dmask);
          if (pend_n + nd > 64u) {
            bwd_drain(m, wpend, pend_n, lane, od, ray_end, ray_gw, tr, weights, r0, sig_miss, kWeighted, g_miss,
                      g_sig);
            pend_n = 0;
          }
          if (deferred) {
            const uint32_t rank = (uint32_t)__popcll(dmask & ((1ull << lane) - 1ull));
            BwdPending e;
            e.v = (uint32_t)v;
            e.k[0] = k0;
            e.k[1] = k1;
            e.k[2] = k2;
            e.ray_t = ray_t;
            e.G = G;
            wpend[pend_n + rank] = e;
          }
          pend_n += nd;
        }
      }
    }
  }
  if (kNdt && pend_n)
    bwd_drain(m, wpend, pend_n, lane, od, ray_end, ray_gw, tr, weights, r0, sig_miss, kWeighted, g_miss, g_sig);
  __syncthreads();
  if (t.inrange && grad_w) grad_w[(size_t)r0 + tr.src[tid]] = (float)ray_gw[tid];
  // block reduction of the scalar gradients, one fp64 atomic per block each
  __shared__ double part[3][kBackwardMaxThreads / 64];
  double vals[3] = {g_hit, g_miss, g_sig};
  const uint32_t wave = tid >> 6;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double x = vals[c];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if (lane == 0) part[c][wave] = x;
  }
  __syncthreads();
  if (tid < 3) {
    double x = 0.0;
    for (uint32_t k = 0; k < (blockDim.x >> 6); ++k) x += part[tid][k];
    if (x != 0.0) unsafeAtomicAdd(grad_s + tid, x);
  }
}

__global__ void zero_f64_kernel(double* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

}  // namespace

}  // namespace ohm

using namespace ohm;

extern "C" ohm_status ohm_backward(ohm_map map, int32_t ndt, const float* d_grad, const int32_t h_box_min[3],
                                   const int32_t h_box_dim[3], const float* d_origins, const float* d_samples,
                                   const uint32_t* h_scan_offsets, uint32_t n_scans, const float* d_weights,
                                   float* d_grad_weights, double* d_grad_scalars, void* stream) {
  ohm_status s = check_scans(map, d_origins, d_samples, h_scan_offsets, n_scans);
  if (s != OHM_OK) return s;
  if (!d_grad || !h_box_min || !h_box_dim || !d_grad_scalars || !map->dm.clampscan) return OHM_E_INVALID_ARG;
  if (ndt && !map->dm.ndt) return OHM_E_INVALID_ARG;
  if (map->params.mode != OHM_MODE_COUNT_CLAMP) return OHM_E_UNSUPPORTED;
  // a batched plan keeps no per-scan clamp record, so its scans cannot be differentiated
  if (map->batched) return OHM_E_UNSUPPORTED;
  if (ndt && !(isinf(map->params.ndt_clear_below) && map->params.ndt_clear_below < 0)) return OHM_E_UNSUPPORTED;
  for (int a = 0; a < 3; ++a)
    if (h_box_dim[a] <= 0) return OHM_E_INVALID_ARG;
  if ((size_t)h_box_dim[0] * h_box_dim[1] * h_box_dim[2] > ((size_t)1 << 38)) return OHM_E_INVALID_ARG;
  // the map must hold exactly these scans since its last create / reset
  uint32_t nonempty = 0;
  for (uint32_t sc = 0; sc < n_scans; ++sc) nonempty += h_scan_offsets[sc + 1] > h_scan_offsets[sc] ? 1u : 0u;
  if (nonempty != map->scans_done) return OHM_E_INVALID_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  GradBox gb;
  gb.g = d_grad;
  for (int a = 0; a < 3; ++a) {
    gb.bmin[a] = h_box_min[a];
    gb.bdim[a] = h_box_dim[a];
  }
  const double sig_miss = 1.0 / (1.0 + exp(-(double)map->params.l_miss));
  const bool weighted = d_weights != nullptr;
  // the replay rebuilds the NDT statistics only: an NDT-TM layer keeps its
  // final state (the replay adds no intensity moments for it to merge)
  DevMap bm = map->dm;
  bm.tm = nullptr;
  bm.tm_mom = nullptr;
  hipLaunchKernelGGL(zero_f64_kernel, dim3(1), dim3(64), 0, st, d_grad_scalars, 3);
  if (ndt) {
    clear_pending(map, st);
    // empty the statistics of the box's voxels, the only ones the gradient
    // reads; they are replayed scan by scan below (the others keep their
    // final values)
    const size_t nbox = (size_t)gb.bdim[0] * gb.bdim[1] * gb.bdim[2];
    hipLaunchKernelGGL(clear_box_stats_kernel, dim3((unsigned)((nbox + 255) / 256)), dim3(256), 0, st, bm, gb);
  }
  uint32_t tag = 0;
  for (uint32_t sc = 0; sc < n_scans; ++sc) {
    const uint32_t r0 = h_scan_offsets[sc];
    const uint32_t n = h_scan_offsets[sc + 1] - r0;
    if (n == 0) continue;
    ++tag;
    const dim3 tiles((n + kTileRays - 1) / kTileRays);
    const dim3 threads(map->walk_threads < kBackwardMaxThreads ? map->walk_threads : kBackwardMaxThreads);
    const int K = map->seg_major_steps;
    // NDT: the walk lists its regions under a fresh tag for the fold below
    const uint32_t ftag = ndt ? ++map->count_batches : 0u;
    const uint32_t fparity = ftag & 1u;
    {
      ProfScope ps(map, OHM_KERNEL_OTHER, st);
      if (ndt) {
        if (weighted)
          hipLaunchKernelGGL((backward_seg_kernel<true, true>), tiles, threads, 0, st, bm, gb, d_origins, sc,
                             d_samples, d_weights, r0, n, K, tag, ftag, fparity, d_grad_weights, d_grad_scalars,
                             sig_miss);
        else
          hipLaunchKernelGGL((backward_seg_kernel<true, false>), tiles, threads, 0, st, bm, gb, d_origins, sc,
                             d_samples, d_weights, r0, n, K, tag, ftag, fparity, d_grad_weights, d_grad_scalars,
                             sig_miss);
      } else {
        if (weighted)
          hipLaunchKernelGGL((backward_seg_kernel<false, true>), tiles, threads, 0, st, bm, gb, d_origins, sc,
                             d_samples, d_weights, r0, n, K, tag, 0u, 0u, d_grad_weights, d_grad_scalars, sig_miss);
        else
          hipLaunchKernelGGL((backward_seg_kernel<false, false>), tiles, threads, 0, st, bm, gb, d_origins, sc,
                             d_samples, d_weights, r0, n, K, tag, 0u, 0u, d_grad_weights, d_grad_scalars, sig_miss);
      }
    }
    if (ndt) {
      // the statistics replay, for the voxels whose statistics the gradient
      // reads (the box's): the scan's hit samples there, as the forward adds them
      ProfScope ps(map, OHM_KERNEL_NDT_SAMPLES, st);
      HitBox box;
      for (int a = 0; a < 3; ++a) {
        const int64_t hi = (int64_t)gb.bmin[a] + gb.bdim[a];
        box.lo[a] = gb.bmin[a];
        box.hi[a] = hi > INT32_MAX ? INT32_MAX : (int32_t)hi;
      }
      launch_ndt_hits(bm, st, d_origins, sc, d_samples, d_weights, r0, n, box);
    }
    if (ndt) {
      // fold only: the accumulators hold no increments, so occupancy is unchanged
      ProfScope ps(map, OHM_KERNEL_NDT_HIT, st);
      hipLaunchKernelGGL(ndt_finalize_kernel, dim3(kFinalizeBlocks), dim3(256), 0, st, bm, fparity, 1, 0u);
    }
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? OHM_OK : OHM_E_HIP;
}
