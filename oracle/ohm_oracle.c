/*
 * CPU oracle for OHM lidar ray integration -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded reference of what the GPU path computes.
 * Only the test suite, the package smoke check and the benchmark's CPU
 * baseline may load this library; the product path never calls it.  It
 * shares no code, header or table with the HIP library.
 *
 * What it follows (paper: "OHM: GPU Based Occupancy Map Generation"):
 *   - Sec. II-B, Eq. (2)-(3): log-odds occupancy, hit increment positive,
 *     miss increment negative; the clamping paragraph after Eq. (3).
 *   - Sec. III-B: one ray from sensor origin to sample, walked voxel by voxel
 *     with the Amanatides & Woo line walk, one voxel per step; misses along
 *     the ray, a hit in the sample's voxel.
 *   - Sec. IV-A: rays truncated to a maximum range.
 * Readings where the paper is silent are fixed as follows (all are listed
 * in the design notes):
 *   - Points are quantised to fixed point, q = rint((p - m) * 2^F / s) in
 *     IEEE double, key = floor(q / 2^F).  No float enters a key decision
 *     after that.
 *   - The walk visits the start voxel and then applies every voxel-boundary
 *     crossing of the segment in increasing order of its ray parameter t;
 *     simultaneous crossings go to the lower axis first (x, y, z).  This
 *     oracle lists all crossings and sorts them by exact 128-bit
 *     cross-multiplication.
 *   - The walk stops at the first key outside the map bounds (no hit then).
 *     Rays whose origin key lies outside the bounds are rejected whole.
 *   - A ray longer than max_range is shortened to max_range and carries no
 *     hit: every voxel it visits, the last included, takes a miss.
 *   - The sample voxel takes the hit and no miss.
 *   - Count-then-clamp batch semantics: per scan, per voxel,
 *     l <- clamp((l + H*l_hit) + M*l_miss) in fp32.
 *   - Per-update semantics (the paper's CAS updates in an unspecified order):
 *     the set of reachable results is bracketed by applying all hits before
 *     all misses (lower bound) and all misses before all hits (upper bound).
 * Parity pins for this file live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double voxel_size;
  double map_origin[3];
  int32_t key_min[3];
  int32_t key_max[3];
  int32_t fixed_bits;
  float l_hit, l_miss, l_min, l_max, l_init;
  double max_range;
  double sensor_noise;
  double adaptation_rate;
  int32_t ndt_min_samples;
  double ndt_clear_below;
  double ndt_tm_gate;
  double tsdf_truncation;
  double tsdf_max_weight;
} orc_params;

enum { ORC_RAY_OK = 0, ORC_RAY_INVALID = 1, ORC_RAY_ORIGIN_OOB = 2 };

/* per-ray flag bits reported by orc_trace */
enum {
  ORC_F_TRUNCATED = 1,
  ORC_F_CLIPPED = 2,
  ORC_F_HAS_HIT = 4,
  ORC_F_INVALID = 8,
  ORC_F_ORIGIN_OOB = 16
};

/* stats vector layout */
enum {
  ORC_S_RAYS = 0,
  ORC_S_INVALID,
  ORC_S_ORIGIN_OOB,
  ORC_S_TRUNCATED,
  ORC_S_CLIPPED,
  ORC_S_HITS,
  ORC_S_UPDATES,
  ORC_S_COUNT
};

typedef struct {
  int status;
  int truncated;
  int64_t q0[3], q1[3];
  int64_t k0[3], k1[3];
  double end[3]; /* world endpoint after truncation */
} orc_ray;

typedef struct {
  int64_t num; /* crossing parameter t = num / den */
  int64_t den;
  int axis;
} orc_event;

static int64_t floor_div_pow2(int64_t q, int f) {
  /* floor(q / 2^f) for either sign */
  int64_t d = (int64_t)1 << f;
  int64_t r = q / d;
  if ((q % d) != 0 && q < 0) r -= 1;
  return r;
}

/* Quantise one coordinate; returns 0 when the value is not representable. */
static int quantise(double p, double m, double scale, int64_t* q) {
  double x = (p - m) * scale;
  if (!(fabs(x) < 0x1p46)) return 0;
  *q = (int64_t)rint(x);
  return 1;
}

static int in_bounds(const orc_params* p, const int64_t k[3]) {
  for (int a = 0; a < 3; ++a)
    if (k[a] < p->key_min[a] || k[a] >= p->key_max[a]) return 0;
  return 1;
}

static void prepare_ray(const orc_params* p, const float o[3], const float e[3], orc_ray* r) {
  memset(r, 0, sizeof(*r));
  for (int a = 0; a < 3; ++a)
    if (!isfinite(o[a]) || !isfinite(e[a])) {
      r->status = ORC_RAY_INVALID;
      return;
    }
  double end[3];
  for (int a = 0; a < 3; ++a) end[a] = (double)e[a];
  if (p->max_range > 0.0) {
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = (double)e[a] - (double)o[a];
    double d2 = d[0] * d[0];
    d2 = d2 + d[1] * d[1];
    d2 = d2 + d[2] * d[2];
    if (d2 > p->max_range * p->max_range) {
      double f = p->max_range / sqrt(d2);
      for (int a = 0; a < 3; ++a) end[a] = (double)o[a] + d[a] * f;
      r->truncated = 1;
    }
  }
  double scale = ldexp(1.0, p->fixed_bits) / p->voxel_size;
  for (int a = 0; a < 3; ++a) {
    if (!quantise((double)o[a], p->map_origin[a], scale, &r->q0[a]) ||
        !quantise(end[a], p->map_origin[a], scale, &r->q1[a])) {
      r->status = ORC_RAY_INVALID;
      return;
    }
    int64_t span = r->q1[a] - r->q0[a];
    if (span >= ((int64_t)1 << 31) || -span >= ((int64_t)1 << 31)) {
      r->status = ORC_RAY_INVALID;
      return;
    }
    r->k0[a] = floor_div_pow2(r->q0[a], p->fixed_bits);
    r->k1[a] = floor_div_pow2(r->q1[a], p->fixed_bits);
    r->end[a] = end[a];
  }
  if (!in_bounds(p, r->k0)) {
    r->status = ORC_RAY_ORIGIN_OOB;
    return;
  }
  r->status = ORC_RAY_OK;
}

/* A ray whose weight is negative or not finite is rejected whole, like a
   non-finite ray (the library's input contract for per-ray weights). */
static void prepare_weighted_ray(const orc_params* p, const float o[3], const float* samples, const float* weights,
                                 uint32_t i, orc_ray* r) {
  prepare_ray(p, o, samples + 3 * (size_t)i, r);
  if (weights && !(weights[i] >= 0.0f && isfinite(weights[i]))) r->status = ORC_RAY_INVALID;
}

static int cmp_event(const void* va, const void* vb) {
  const orc_event* x = (const orc_event*)va;
  const orc_event* y = (const orc_event*)vb;
  __int128 l = (__int128)x->num * (__int128)y->den;
  __int128 r = (__int128)y->num * (__int128)x->den;
  if (l < r) return -1;
  if (l > r) return 1;
  return (x->axis > y->axis) - (x->axis < y->axis);
}

typedef struct {
  orc_event* ev;
  size_t ev_cap;
  int32_t* keys;
  size_t key_cap;
} orc_scratch;

static void scratch_free(orc_scratch* s) {
  free(s->ev);
  free(s->keys);
  memset(s, 0, sizeof(*s));
}

/*
 * Walk one prepared ray.  Writes the in-bounds visited keys (x,y,z triples)
 * into s->keys and returns how many there are; *clipped is set when the walk
 * left the map before reaching the end voxel.
 */
static int64_t walk_ray(const orc_params* p, const orc_ray* r, orc_scratch* s, int* clipped) {
  const int F = p->fixed_bits;
  const int64_t one = (int64_t)1 << F;
  int64_t sg[3], n[3], b[3], A[3];
  size_t total = 0;
  for (int a = 0; a < 3; ++a) {
    int64_t D = r->q1[a] - r->q0[a];
    sg[a] = (D > 0) - (D < 0);
    A[a] = D < 0 ? -D : D;
    n[a] = r->k1[a] - r->k0[a];
    if (n[a] < 0) n[a] = -n[a];
    b[a] = (sg[a] > 0) ? ((r->k0[a] + 1) * one - r->q0[a]) : (r->q0[a] - r->k0[a] * one);
    total += (size_t)n[a];
  }
  if (total > s->ev_cap) {
    s->ev_cap = total + 64;
    s->ev = (orc_event*)realloc(s->ev, s->ev_cap * sizeof(orc_event));
  }
  if (3 * (total + 1) > s->key_cap) {
    s->key_cap = 3 * (total + 1) + 192;
    s->keys = (int32_t*)realloc(s->keys, s->key_cap * sizeof(int32_t));
  }
  size_t ne = 0;
  for (int a = 0; a < 3; ++a)
    for (int64_t j = 0; j < n[a]; ++j) {
      s->ev[ne].num = b[a] + j * one;
      s->ev[ne].den = A[a];
      s->ev[ne].axis = a;
      ++ne;
    }
  qsort(s->ev, ne, sizeof(orc_event), cmp_event);

  int64_t k[3] = {r->k0[0], r->k0[1], r->k0[2]};
  int64_t nk = 0;
  *clipped = 0;
  for (int a = 0; a < 3; ++a) s->keys[a] = (int32_t)k[a];
  nk = 1;
  for (size_t i = 0; i < ne; ++i) {
    int a = s->ev[i].axis;
    k[a] += sg[a];
    if (!in_bounds(p, k)) {
      *clipped = 1;
      break;
    }
    for (int c = 0; c < 3; ++c) s->keys[3 * nk + c] = (int32_t)k[c];
    ++nk;
  }
  return nk;
}

static int64_t box_index(const int32_t* key, const int32_t box_min[3], const int32_t box_dim[3]) {
  int64_t x = (int64_t)key[0] - box_min[0];
  int64_t y = (int64_t)key[1] - box_min[1];
  int64_t z = (int64_t)key[2] - box_min[2];
  if (x < 0 || y < 0 || z < 0 || x >= box_dim[0] || y >= box_dim[1] || z >= box_dim[2]) return -1;
  return (z * box_dim[1] + y) * box_dim[0] + x;
}

/* ---------------------------------------------------------------------- */
/* Per-ray trace                                                           */
/* ---------------------------------------------------------------------- */

/*
 * For every ray: its update list (kx, ky, kz, kind) with kind 0 = miss,
 * 1 = hit, in walk order.  ray_counts[i] receives the number of updates of
 * ray i and ray_flags[i] its ORC_F_* bits.  keys may be NULL (count pass).
 * Returns the total number of updates.
 */
int64_t orc_trace(const orc_params* p, int32_t n_scans, const uint32_t* offsets, const float* origins,
                  const float* samples, int64_t* ray_counts, int32_t* ray_flags, int32_t* keys) {
  orc_scratch s = {0};
  int64_t written = 0;
  for (int32_t sc = 0; sc < n_scans; ++sc) {
    for (uint32_t i = offsets[sc]; i < offsets[sc + 1]; ++i) {
      orc_ray r;
      prepare_ray(p, origins + 3 * sc, samples + 3 * (size_t)i, &r);
      int flags = 0;
      int64_t nk = 0;
      if (r.status == ORC_RAY_INVALID) flags |= ORC_F_INVALID;
      if (r.status == ORC_RAY_ORIGIN_OOB) flags |= ORC_F_ORIGIN_OOB;
      if (r.status == ORC_RAY_OK) {
        int clipped = 0;
        nk = walk_ray(p, &r, &s, &clipped);
        int has_hit = !r.truncated && !clipped;
        flags |= (r.truncated ? ORC_F_TRUNCATED : 0) | (clipped ? ORC_F_CLIPPED : 0) | (has_hit ? ORC_F_HAS_HIT : 0);
        if (keys) {
          for (int64_t j = 0; j < nk; ++j) {
            int32_t* out = keys + 4 * (written + j);
            out[0] = s.keys[3 * j + 0];
            out[1] = s.keys[3 * j + 1];
            out[2] = s.keys[3 * j + 2];
            out[3] = (has_hit && j == nk - 1) ? 1 : 0;
          }
        }
      }
      if (ray_counts) ray_counts[i] = nk;
      if (ray_flags) ray_flags[i] = flags;
      written += nk;
    }
  }
  scratch_free(&s);
  return written;
}

/* ---------------------------------------------------------------------- */
/* Batch integration                                                       */
/* ---------------------------------------------------------------------- */

static float clampf_(float v, float lo, float hi) {
  if (v < lo) v = lo;
  if (v > hi) v = hi;
  return v;
}

static double clampd_(double v, double lo, double hi) {
  if (v < lo) v = lo;
  if (v > hi) v = hi;
  return v;
}

/*
 * Shared driver: walks every ray of one scan and accumulates, per voxel of the
 * box window, the hit weight and the miss weight (unit weights when weights is
 * NULL).  Voxels outside the window are still walked (and counted in stats)
 * but not recorded.
 */
static void accumulate_scan(const orc_params* p, const float* origin, uint32_t r0, uint32_t r1,
                            const float* samples, const float* weights, int unit_weights, const int32_t box_min[3],
                            const int32_t box_dim[3], double* wh, double* wm, uint64_t* stats,
                            orc_scratch* s) {
  for (uint32_t i = r0; i < r1; ++i) {
    orc_ray r;
    prepare_weighted_ray(p, origin, samples, weights, i, &r);
    if (stats) stats[ORC_S_RAYS] += 1;
    if (r.status == ORC_RAY_INVALID) {
      if (stats) stats[ORC_S_INVALID] += 1;
      continue;
    }
    if (r.status == ORC_RAY_ORIGIN_OOB) {
      if (stats) stats[ORC_S_ORIGIN_OOB] += 1;
      continue;
    }
    int clipped = 0;
    int64_t nk = walk_ray(p, &r, s, &clipped);
    int has_hit = !r.truncated && !clipped;
    double w = (weights && !unit_weights) ? (double)weights[i] : 1.0;
    if (stats) {
      stats[ORC_S_TRUNCATED] += r.truncated ? 1 : 0;
      stats[ORC_S_CLIPPED] += clipped ? 1 : 0;
      stats[ORC_S_HITS] += has_hit ? 1 : 0;
      stats[ORC_S_UPDATES] += (uint64_t)nk;
    }
    for (int64_t j = 0; j < nk; ++j) {
      int64_t v = box_index(s->keys + 3 * j, box_min, box_dim);
      if (v < 0) continue;
      if (has_hit && j == nk - 1)
        wh[v] += w;
      else
        wm[v] += w;
    }
  }
}

/*
 * Count-then-clamp integration of n_scans scans into the box window.
 *   occ       [dz][dy][dx] fp32, in/out (callers initialise it to l_init)
 *   last_hit, last_miss   optional outputs: the hit / miss weight of the last
 *             scan per voxel (integer counts when weights is NULL)
 *   stats     ORC_S_COUNT uint64 counters (accumulated)
 * Without weights the update is the exact fp32 expression
 *   t = (float)H * l_hit; u = (float)M * l_miss; l = clamp((l + t) + u).
 * With weights the per-voxel sums and the update are evaluated in fp64.
 */
int orc_integrate_count(const orc_params* p, int32_t n_scans, const uint32_t* offsets, const float* origins,
                        const float* samples, const float* weights, const int32_t box_min[3],
                        const int32_t box_dim[3], float* occ, float* last_hit, float* last_miss,
                        uint64_t* stats) {
  size_t nv = (size_t)box_dim[0] * box_dim[1] * box_dim[2];
  double* wh = (double*)calloc(nv, sizeof(double));
  double* wm = (double*)calloc(nv, sizeof(double));
  if (!wh || !wm) {
    free(wh);
    free(wm);
    return -1;
  }
  orc_scratch s = {0};
  for (int32_t sc = 0; sc < n_scans; ++sc) {
    memset(wh, 0, nv * sizeof(double));
    memset(wm, 0, nv * sizeof(double));
    accumulate_scan(p, origins + 3 * sc, offsets[sc], offsets[sc + 1], samples, weights, 0, box_min, box_dim, wh,
                    wm, stats, &s);
    for (size_t v = 0; v < nv; ++v) {
      if (wh[v] == 0.0 && wm[v] == 0.0) continue;
      if (!weights) {
        float t = (float)wh[v] * p->l_hit;
        float u = (float)wm[v] * p->l_miss;
        float l = occ[v] + t;
        l = l + u;
        occ[v] = clampf_(l, p->l_min, p->l_max);
      } else {
        double l = ((double)occ[v] + wh[v] * (double)p->l_hit) + wm[v] * (double)p->l_miss;
        occ[v] = (float)clampd_(l, (double)p->l_min, (double)p->l_max);
      }
    }
  }
  if (last_hit)
    for (size_t v = 0; v < nv; ++v) last_hit[v] = (float)wh[v];
  if (last_miss)
    for (size_t v = 0; v < nv; ++v) last_miss[v] = (float)wm[v];
  scratch_free(&s);
  free(wh);
  free(wm);
  return 0;
}

/*
 * Per-update semantics: each hit (+w*l_hit) and miss (+w*l_miss) is applied
 * as l <- clamp(l + delta) in some order.  For each scan, a voxel's result over
 * all orders lies between applying its hits first then its misses (lo) and its
 * misses first then its hits (hi); these maps are monotone, so the bracket
 * carries from scan to scan.  Same-sign runs are summed before clamping (the
 * same value as clamping after each, since a same-sign run can cross a bound
 * only once).  Evaluated in fp64.
 *   lo, hi       [dz][dy][dx] fp64, in/out (initialise both to l_init)
 *   n_updates    [dz][dy][dx] uint32, in/out: updates applied per voxel
 */
int orc_integrate_envelope(const orc_params* p, int32_t n_scans, const uint32_t* offsets, const float* origins,
                           const float* samples, const float* weights, const int32_t box_min[3],
                           const int32_t box_dim[3], double* lo, double* hi, uint32_t* n_updates,
                           uint64_t* stats) {
  size_t nv = (size_t)box_dim[0] * box_dim[1] * box_dim[2];
  double* wh = (double*)calloc(nv, sizeof(double));
  double* wm = (double*)calloc(nv, sizeof(double));
  if (!wh || !wm) {
    free(wh);
    free(wm);
    return -1;
  }
  orc_scratch s = {0};
  double lmin = (double)p->l_min, lmax = (double)p->l_max;
  for (int32_t sc = 0; sc < n_scans; ++sc) {
    memset(wh, 0, nv * sizeof(double));
    memset(wm, 0, nv * sizeof(double));
    accumulate_scan(p, origins + 3 * sc, offsets[sc], offsets[sc + 1], samples, weights, 0, box_min, box_dim, wh,
                    wm, stats, &s);
    if (n_updates) {
      /* re-walk with unit weights to count updates */
      double* ch = (double*)calloc(nv, sizeof(double));
      double* cm = (double*)calloc(nv, sizeof(double));
      accumulate_scan(p, origins + 3 * sc, offsets[sc], offsets[sc + 1], samples, weights, 1, box_min, box_dim, ch,
                      cm, NULL, &s);
      for (size_t v = 0; v < nv; ++v) n_updates[v] += (uint32_t)(ch[v] + cm[v]);
      free(ch);
      free(cm);
    }
    for (size_t v = 0; v < nv; ++v) {
      if (wh[v] == 0.0 && wm[v] == 0.0) continue;
      double a = wh[v] * (double)p->l_hit;
      double b = wm[v] * (double)p->l_miss;
      lo[v] = clampd_(clampd_(lo[v] + a, lmin, lmax) + b, lmin, lmax);
      hi[v] = clampd_(clampd_(hi[v] + b, lmin, lmax) + a, lmin, lmax);
    }
  }
  scratch_free(&s);
  free(wh);
  free(wm);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* NDT-OM                                                                  */
/* ---------------------------------------------------------------------- */
/*
 * NDT-OM (paper Sec. II-D and III-C).  Each voxel keeps a sample count n, a
 * mean mu and a population covariance Sigma of the samples that fell in it
 * (voxel-centred coordinates, metres).  Per scan:
 *   1. misses: for every ray and every voxel it passes (all visited voxels
 *      but a hit voxel), with the voxel's statistics as they were before the
 *      scan: when n >= ndt_min_samples,
 *        x* = the point of the ray segment closest to mu (Euclidean),
 *        D  = x* - mu,  S = Sigma + sensor_noise^2 I,
 *        g  = exp(-D^T S^-1 D / 2),
 *        p  = 1/2 - adaptation_rate * g * (1/2 - sigmoid(l_miss)),
 *        delta = ln(p / (1 - p));
 *      otherwise delta = l_miss.  The ray weight scales delta.
 *   2. occupancy: count mode l = clamp((l + sum_hits w l_hit) + sum_misses w delta);
 *      per-update mode (misses applied first, then hits, as the paper's two
 *      phases) l = clamp(clamp(l + sum_misses w delta) + sum_hits w l_hit).
 *   3. voxels whose new l is below ndt_clear_below lose their statistics.
 *   4. every sample of the scan is folded into its voxel, in ascending ray
 *      order, by Welford's update:
 *        n <- n + 1; d = x - mu; mu <- mu + d / n;
 *        Sigma <- Sigma (n-1)/n + d d^T (n-1)/n^2.
 * All in fp64; occupancy is stored as float after each scan.
 */

static double sigmoid_d(double x) { return 1.0 / (1.0 + exp(-x)); }

/* Solve S y = D for a symmetric positive-definite 3x3 S (xx, xy, xz, yy, yz, zz)
   by Cholesky factorisation; returns D^T y. */
static double quad_form_inv(const double S6[6], const double D[3]) {
  double a00 = S6[0], a10 = S6[1], a20 = S6[2], a11 = S6[3], a21 = S6[4], a22 = S6[5];
  double l00 = sqrt(a00);
  double l10 = a10 / l00, l20 = a20 / l00;
  double l11 = sqrt(a11 - l10 * l10);
  double l21 = (a21 - l20 * l10) / l11;
  double l22 = sqrt(a22 - l20 * l20 - l21 * l21);
  /* forward substitution L z = D; D^T S^-1 D = |z|^2 */
  double z0 = D[0] / l00;
  double z1 = (D[1] - l10 * z0) / l11;
  double z2 = (D[2] - l20 * z0 - l21 * z1) / l22;
  return z0 * z0 + z1 * z1 + z2 * z2;
}

/* Squared Mahalanobis distance q = D^T S^-1 D of the ray's closest point to
   the voxel's mean (see above).  o and e are the ray's world start and
   (possibly truncated) end; mu_w the voxel's world mean; cov its covariance. */
static double ndt_closest_q(const orc_params* p, const double o[3], const double e[3], const double mu_w[3],
                            const double cov[6]) {
  double d[3], w[3];
  double dd = 0.0, wd = 0.0;
  for (int a = 0; a < 3; ++a) {
    d[a] = e[a] - o[a];
    w[a] = mu_w[a] - o[a];
    dd += d[a] * d[a];
    wd += w[a] * d[a];
  }
  double t = dd > 0.0 ? wd / dd : 0.0;
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  double D[3];
  for (int a = 0; a < 3; ++a) D[a] = (o[a] + t * d[a]) - mu_w[a];
  double s2 = p->sensor_noise * p->sensor_noise;
  double S[6] = {cov[0] + s2, cov[1], cov[2], cov[3] + s2, cov[4], cov[5] + s2};
  return quad_form_inv(S, D);
}

/* The NDT-weighted miss increment for one voxel (see above). */
double orc_ndt_miss_delta(const orc_params* p, const double o[3], const double e[3], const double mu_w[3],
                          const double cov[6], uint32_t n) {
  if (n < (uint32_t)p->ndt_min_samples) return (double)p->l_miss;
  double g = exp(-0.5 * ndt_closest_q(p, o, e, mu_w, cov));
  double pr = 0.5 - p->adaptation_rate * g * (0.5 - sigmoid_d((double)p->l_miss));
  return log(pr / (1.0 - pr));
}

static void welford_add(uint32_t* n, double mu[3], double cov[6], const double x[3]) {
  *n += 1;
  double nn = (double)*n;
  double d[3];
  for (int a = 0; a < 3; ++a) {
    d[a] = x[a] - mu[a];
    mu[a] += d[a] / nn;
  }
  double f = (nn - 1.0) / nn;
  double g = (nn - 1.0) / (nn * nn);
  cov[0] = cov[0] * f + d[0] * d[0] * g;
  cov[1] = cov[1] * f + d[0] * d[1] * g;
  cov[2] = cov[2] * f + d[0] * d[2] * g;
  cov[3] = cov[3] * f + d[1] * d[1] * g;
  cov[4] = cov[4] * f + d[1] * d[2] * g;
  cov[5] = cov[5] * f + d[2] * d[2] * g;
}

static void voxel_centre(const orc_params* p, const int32_t* k, double c[3]) {
  for (int a = 0; a < 3; ++a) c[a] = p->map_origin[a] + ((double)k[a] + 0.5) * p->voxel_size;
}

/*
 * NDT-TM (paper Sec. II-D, III-C) keeps, beside the NDT-OM statistics, the
 * counts behind a voxel's permeability H / (H + M) and a 1D Gaussian of the
 * intensity of the samples that fell in it:
 *   H  = the voxel's samples (the NDT sample count n: both start together
 *        and are cleared together);
 *   M  = misses through the voxel that passed the check that the ray came
 *        close to the voxel's data: the voxel holds >= ndt_min_samples
 *        samples (so it has a Gaussian, from the statistics before the scan,
 *        as the NDT-OM weighting uses) and the ray's closest point lies
 *        within ndt_tm_gate of it in squared Mahalanobis distance
 *        (q = D^T S^-1 D <= ndt_tm_gate);
 *   intensity mean and population variance of the samples, by Welford's
 *        update in ascending ray order alongside the position statistics.
 * Counts are plain (ray weights scale only occupancy increments).  Voxels
 * whose statistics are cleared lose M and the intensity Gaussian too.
 */
typedef struct {
  uint32_t* miss;     /* M, [dz][dy][dx] */
  uint32_t* near;     /* misses with q within a relative 1e-9 of the gate (either side): the
                         decision there rests on the last bits of q; the GPU may take either */
  double* in_mean;    /* intensity mean */
  double* in_var;     /* intensity population variance */
  const float* intensities; /* per ray */
} orc_ndt_tm;

/*
 * NDT-OM integration of n_scans scans into the box window (paper Sec. II-D,
 * III-C; formulas above).  mode 1 = count-then-clamp, 0 = per-update.
 *   occ        [dz][dy][dx] float, in/out
 *   nd_n       [dz][dy][dx] uint32, in/out sample counts
 *   nd_mu      [dz][dy][dx][3] fp64, in/out means (voxel-centred, metres)
 *   nd_cov     [dz][dy][dx][6] fp64, in/out covariances
 *   miss_sum   optional out: last scan's summed miss increments per voxel
 *   tm         optional NDT-TM state (see above), in/out
 *   stats      ORC_S_COUNT counters (accumulated)
 * Updates landing outside the window are ignored; so is the NDT state there.
 */
static int ndt_integrate_core(const orc_params* p, int32_t mode, int32_t n_scans, const uint32_t* offsets,
                              const float* origins, const float* samples, const float* weights,
                              const int32_t box_min[3], const int32_t box_dim[3], float* occ, uint32_t* nd_n,
                              double* nd_mu, double* nd_cov, double* miss_sum, orc_ndt_tm* tm, uint64_t* stats) {
  size_t nv = (size_t)box_dim[0] * box_dim[1] * box_dim[2];
  double* wh = (double*)calloc(nv, sizeof(double));
  double* dm = (double*)calloc(nv, sizeof(double));
  unsigned char* touched = (unsigned char*)calloc(nv, 1);
  if (!wh || !dm || !touched) {
    free(wh);
    free(dm);
    free(touched);
    return -1;
  }
  /* pre-scan snapshot of the statistics used by the miss pass */
  uint32_t* n0 = (uint32_t*)malloc(nv * sizeof(uint32_t));
  double* mu0 = (double*)malloc(nv * 3 * sizeof(double));
  double* cov0 = (double*)malloc(nv * 6 * sizeof(double));
  orc_scratch s = {0};
  for (int32_t sc = 0; sc < n_scans; ++sc) {
    memset(wh, 0, nv * sizeof(double));
    memset(dm, 0, nv * sizeof(double));
    memset(touched, 0, nv);
    memcpy(n0, nd_n, nv * sizeof(uint32_t));
    memcpy(mu0, nd_mu, nv * 3 * sizeof(double));
    memcpy(cov0, nd_cov, nv * 6 * sizeof(double));
    const float* of = origins + 3 * sc;
    double o[3] = {(double)of[0], (double)of[1], (double)of[2]};
    /* phase 1: misses (and hit weights) */
    for (uint32_t i = offsets[sc]; i < offsets[sc + 1]; ++i) {
      orc_ray r;
      prepare_weighted_ray(p, of, samples, weights, i, &r);
      if (stats) stats[ORC_S_RAYS] += 1;
      if (r.status != ORC_RAY_OK) {
        if (stats) stats[r.status == ORC_RAY_INVALID ? ORC_S_INVALID : ORC_S_ORIGIN_OOB] += 1;
        continue;
      }
      int clipped = 0;
      int64_t nk = walk_ray(p, &r, &s, &clipped);
      int has_hit = !r.truncated && !clipped;
      double w = weights ? (double)weights[i] : 1.0;
      if (stats) {
        stats[ORC_S_TRUNCATED] += r.truncated ? 1 : 0;
        stats[ORC_S_CLIPPED] += clipped ? 1 : 0;
        stats[ORC_S_HITS] += has_hit ? 1 : 0;
        stats[ORC_S_UPDATES] += (uint64_t)nk;
      }
      for (int64_t j = 0; j < nk; ++j) {
        const int32_t* key = s.keys + 3 * j;
        int64_t v = box_index(key, box_min, box_dim);
        if (v < 0) continue;
        touched[v] = 1;
        if (has_hit && j == nk - 1) {
          wh[v] += w;
        } else {
          double c[3], muw[3];
          voxel_centre(p, key, c);
          for (int a = 0; a < 3; ++a) muw[a] = c[a] + mu0[3 * v + a];
          dm[v] += w * orc_ndt_miss_delta(p, o, r.end, muw, cov0 + 6 * v, n0[v]);
          if (tm && n0[v] >= (uint32_t)p->ndt_min_samples) {
            double q = ndt_closest_q(p, o, r.end, muw, cov0 + 6 * v);
            if (q <= p->ndt_tm_gate) tm->miss[v] += 1;
            if (fabs(q - p->ndt_tm_gate) <= 1e-9 * fabs(p->ndt_tm_gate)) tm->near[v] += 1;
          }
        }
      }
    }
    /* phase 2a: occupancy and clearing */
    double lmin = (double)p->l_min, lmax = (double)p->l_max;
    for (size_t v = 0; v < nv; ++v) {
      if (!touched[v]) continue;
      double l = (double)occ[v];
      if (mode == 1)
        l = clampd_((l + wh[v] * (double)p->l_hit) + dm[v], lmin, lmax);
      else
        l = clampd_(clampd_(l + dm[v], lmin, lmax) + wh[v] * (double)p->l_hit, lmin, lmax);
      occ[v] = (float)l;
      if ((double)occ[v] < p->ndt_clear_below) {
        nd_n[v] = 0;
        for (int a = 0; a < 3; ++a) nd_mu[3 * v + a] = 0.0;
        for (int a = 0; a < 6; ++a) nd_cov[6 * v + a] = 0.0;
        if (tm) {
          tm->miss[v] = 0;
          tm->in_mean[v] = 0.0;
          tm->in_var[v] = 0.0;
        }
      }
    }
    /* phase 2b: fold this scan's samples, ascending ray order */
    for (uint32_t i = offsets[sc]; i < offsets[sc + 1]; ++i) {
      orc_ray r;
      prepare_weighted_ray(p, of, samples, weights, i, &r);
      if (r.status != ORC_RAY_OK || r.truncated) continue;
      int clipped = 0;
      int64_t nk = walk_ray(p, &r, &s, &clipped);
      if (clipped) continue;
      const int32_t* key = s.keys + 3 * (nk - 1);
      int64_t v = box_index(key, box_min, box_dim);
      if (v < 0) continue;
      double c[3], x[3];
      voxel_centre(p, key, c);
      const float* e = samples + 3 * (size_t)i;
      for (int a = 0; a < 3; ++a) x[a] = (double)e[a] - c[a];
      if (tm) {
        /* intensity Welford over the same samples: count n + 1 after this one */
        double nn = (double)nd_n[v] + 1.0;
        double d = (double)tm->intensities[i] - tm->in_mean[v];
        tm->in_mean[v] += d / nn;
        tm->in_var[v] = tm->in_var[v] * ((nn - 1.0) / nn) + d * d * ((nn - 1.0) / (nn * nn));
      }
      welford_add(nd_n + v, nd_mu + 3 * v, nd_cov + 6 * v, x);
    }
    if (miss_sum && sc == n_scans - 1) memcpy(miss_sum, dm, nv * sizeof(double));
  }
  scratch_free(&s);
  free(wh);
  free(dm);
  free(touched);
  free(n0);
  free(mu0);
  free(cov0);
  return 0;
}

int orc_ndt_integrate(const orc_params* p, int32_t mode, int32_t n_scans, const uint32_t* offsets,
                      const float* origins, const float* samples, const float* weights, const int32_t box_min[3],
                      const int32_t box_dim[3], float* occ, uint32_t* nd_n, double* nd_mu, double* nd_cov,
                      double* miss_sum, uint64_t* stats) {
  return ndt_integrate_core(p, mode, n_scans, offsets, origins, samples, weights, box_min, box_dim, occ, nd_n,
                            nd_mu, nd_cov, miss_sum, NULL, stats);
}

/* NDT-TM integration: NDT-OM (above) plus the permeability counts and the
   intensity Gaussian (tm_miss, tm_near, in_mean, in_var: in/out over the
   window; intensities: one per ray). */
int orc_ndt_tm_integrate(const orc_params* p, int32_t mode, int32_t n_scans, const uint32_t* offsets,
                         const float* origins, const float* samples, const float* intensities, const float* weights,
                         const int32_t box_min[3], const int32_t box_dim[3], float* occ, uint32_t* nd_n, double* nd_mu,
                         double* nd_cov, uint32_t* tm_miss, uint32_t* tm_near, double* in_mean, double* in_var,
                         uint64_t* stats) {
  if (!intensities || !tm_miss || !tm_near || !in_mean || !in_var) return -2;
  orc_ndt_tm tm = {tm_miss, tm_near, in_mean, in_var, intensities};
  return ndt_integrate_core(p, mode, n_scans, offsets, origins, samples, weights, box_min, box_dim, occ, nd_n,
                            nd_mu, nd_cov, NULL, &tm, stats);
}

/* The squared Mahalanobis distance behind the NDT-TM miss check of one voxel
   (exposed for tests). */
double orc_ndt_closest_q(const orc_params* p, const double o[3], const double e[3], const double mu_w[3],
                         const double cov[6]) {
  return ndt_closest_q(p, o, e, mu_w, cov);
}

/* ---------------------------------------------------------------------- */
/* TSDF                                                                    */
/* ---------------------------------------------------------------------- */
/*
 * Truncated signed distance (paper Sec. II-F: voxels within a truncation
 * distance in front of and behind the measured point, along the ray from
 * the sensor, take a projective distance; Sec. III-B: updated like the
 * other 64-bit layers).  Readings:
 *   - only a ray with a surface takes part: valid, origin in the map, not
 *     truncated by max range, sample voxel in the map, and of non-zero
 *     length (the occupancy rules for a hit);
 *   - with r = |e - o| and u = (e - o) / r (fp64), the band is the segment
 *     from o + max(r - tau, 0) u to o + (r + tau) u; its two ends are
 *     quantised like ray ends and walked exactly (clipped at the map's
 *     bounds; a band whose first voxel lies outside the map is skipped);
 *   - each voxel of the band takes sdf = clamp(r - (c - o).u, -tau, tau),
 *     c its centre: positive in front of the surface, negative behind;
 *   - a voxel keeps a distance D and a weight W (both 0 until observed);
 *     n updates of summed distance S (unit weight each) give
 *     D <- (W D + S) / (W + n), W <- min(W + n, tsdf_max_weight);
 *     count mode applies each scan's updates at once, per-update mode one at
 *     a time (here in ray order, band order); D and W are stored as float
 *     after every application.
 * tau = tsdf_truncation.  Arithmetic fp64.
 */

/* The band of a prepared ray (see above); returns 0 when the ray has none. */
static int tsdf_band(const orc_params* p, const float o[3], const float e[3], const orc_ray* r, orc_ray* band,
                     double* range, double u[3]) {
  if (r->status != ORC_RAY_OK || r->truncated || !in_bounds(p, r->k1)) return 0;
  double d[3];
  for (int a = 0; a < 3; ++a) d[a] = (double)e[a] - (double)o[a];
  double r2 = d[0] * d[0];
  r2 = r2 + d[1] * d[1];
  r2 = r2 + d[2] * d[2];
  if (!(r2 > 0.0)) return 0;
  double len = sqrt(r2);
  double tau = p->tsdf_truncation;
  double s0 = len - tau;
  if (s0 < 0.0) s0 = 0.0;
  double s1 = len + tau;
  double scale = ldexp(1.0, p->fixed_bits) / p->voxel_size;
  memset(band, 0, sizeof(*band));
  for (int a = 0; a < 3; ++a) {
    u[a] = d[a] / len;
    double b0 = (double)o[a] + s0 * u[a];
    double b1 = (double)o[a] + s1 * u[a];
    if (!quantise(b0, p->map_origin[a], scale, &band->q0[a]) || !quantise(b1, p->map_origin[a], scale, &band->q1[a]))
      return 0;
    band->k0[a] = floor_div_pow2(band->q0[a], p->fixed_bits);
    band->k1[a] = floor_div_pow2(band->q1[a], p->fixed_bits);
  }
  if (!in_bounds(p, band->k0)) return 0;
  *range = len;
  return 1;
}

static double tsdf_distance(const orc_params* p, const float o[3], double range, const double u[3],
                            const int32_t* key) {
  double c[3];
  voxel_centre(p, key, c);
  double proj = (c[0] - (double)o[0]) * u[0];
  proj = proj + (c[1] - (double)o[1]) * u[1];
  proj = proj + (c[2] - (double)o[2]) * u[2];
  double v = range - proj;
  double tau = p->tsdf_truncation;
  return v < -tau ? -tau : (v > tau ? tau : v);
}

static void tsdf_apply(const orc_params* p, float* dist, float* weight, double sum, double n) {
  double W = (double)*weight;
  double D = ((double)*dist * W + sum) / (W + n);
  double Wn = W + n;
  if (Wn > p->tsdf_max_weight) Wn = p->tsdf_max_weight;
  *dist = (float)D;
  *weight = (float)Wn;
}

/*
 * TSDF integration of n_scans scans into the box window.  mode 1 = count
 * (per-scan sums), 0 = per-update (sequential).  dist / weight:
 * [dz][dy][dx] float in/out.  stats: ORC_S_RAYS / INVALID / ORIGIN_OOB /
 * TRUNCATED / CLIPPED as for occupancy, ORC_S_HITS = rays with a band,
 * ORC_S_UPDATES = band voxel updates (inside the map).
 */
int orc_tsdf_integrate(const orc_params* p, int32_t mode, int32_t n_scans, const uint32_t* offsets,
                       const float* origins, const float* samples, const int32_t box_min[3], const int32_t box_dim[3],
                       float* dist, float* weight, uint64_t* stats) {
  size_t nv = (size_t)box_dim[0] * box_dim[1] * box_dim[2];
  double* sum = (double*)calloc(nv, sizeof(double));
  double* cnt = (double*)calloc(nv, sizeof(double));
  if (!sum || !cnt) {
    free(sum);
    free(cnt);
    return -1;
  }
  orc_scratch s = {0};
  for (int32_t sc = 0; sc < n_scans; ++sc) {
    const float* of = origins + 3 * sc;
    for (uint32_t i = offsets[sc]; i < offsets[sc + 1]; ++i) {
      const float* e = samples + 3 * (size_t)i;
      orc_ray r, band;
      prepare_ray(p, of, e, &r);
      if (stats) stats[ORC_S_RAYS] += 1;
      if (r.status != ORC_RAY_OK) {
        if (stats) stats[r.status == ORC_RAY_INVALID ? ORC_S_INVALID : ORC_S_ORIGIN_OOB] += 1;
        continue;
      }
      if (stats) {
        stats[ORC_S_TRUNCATED] += r.truncated ? 1 : 0;
        stats[ORC_S_CLIPPED] += (!r.truncated && !in_bounds(p, r.k1)) ? 1 : 0;
      }
      double range, u[3];
      if (!tsdf_band(p, of, e, &r, &band, &range, u)) continue;
      int clipped = 0;
      int64_t nk = walk_ray(p, &band, &s, &clipped);
      if (stats) {
        stats[ORC_S_HITS] += 1;
        stats[ORC_S_UPDATES] += (uint64_t)nk;
      }
      for (int64_t j = 0; j < nk; ++j) {
        const int32_t* key = s.keys + 3 * j;
        int64_t v = box_index(key, box_min, box_dim);
        if (v < 0) continue;
        double sd = tsdf_distance(p, of, range, u, key);
        if (mode == 1) {
          sum[v] += sd;
          cnt[v] += 1.0;
        } else {
          tsdf_apply(p, dist + v, weight + v, sd, 1.0);
        }
      }
    }
    if (mode == 1) {
      for (size_t v = 0; v < nv; ++v)
        if (cnt[v] > 0.0) tsdf_apply(p, dist + v, weight + v, sum[v], cnt[v]);
      memset(sum, 0, nv * sizeof(double));
      memset(cnt, 0, nv * sizeof(double));
    }
  }
  scratch_free(&s);
  free(sum);
  free(cnt);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Adjoint                                                                 */
/* ---------------------------------------------------------------------- */
/*
 * Differentiable forward: count-then-clamp per scan in fp64 (no float
 * storage), over a window (the loss box; voxels are independent, so voxels
 * outside it cannot influence the loss).  With ndt != 0 misses use the
 * NDT-weighted increment of orc_ndt_integrate (statistics before the scan,
 * clearing disabled).  Per scan k (1-based tag k):
 *     s_v = (l_v + H_v l_hit) + U_v,   l_v <- clamp(s_v),
 * H_v = sum of hit weights, U_v = sum of weighted miss increments; c_v is
 * the last k with s_v outside [l_min, l_max].  Loss
 *     L = sum_v m_v BCE(sigmoid(l_v), y_v),   G_v = m_v (sigmoid(l_v) - y_v).
 * Because the clamp passes gradients only while inactive, dL/dDelta_{k,v} =
 * G_v [k > c_v], so for ray r of scan k
 *     dL/dw_r      = sum_{v in walk(r)} G_v [k > c_v] delta_{r,v},
 *     dL/dl_hit    = sum_r w_r G_{hit(r)} [k > c],
 *     dL/dl_miss   = sum_r w_r sum_{miss v} G_v [k > c_v] d delta/d l_miss,
 *     dL/dsigma_n  = sum_r w_r sum_{miss v} G_v [k > c_v] d delta/d sigma_n,
 * with, for an NDT-weighted miss (q = D^T S^-1 D, g = exp(-q/2)),
 *     d delta/d l_miss  = lambda g s(1-s) / (p (1-p)),   s = sigmoid(l_miss),
 *     d delta/d sigma_n = -lambda (1/2 - s) g sigma_n |S^-1 D|^2 / (p (1-p)),
 * and 1, 0 for a plain miss.  The backward replays the sample statistics
 * scan by scan (they depend on no differentiated parameter).
 */

/* NDT miss increment and its two partial derivatives. */
static void ndt_miss_terms(const orc_params* p, const double o[3], const double e[3], const double mu_w[3],
                           const double cov[6], uint32_t n, double* delta, double* d_lmiss, double* d_sig) {
  double lm = (double)p->l_miss;
  if (n < (uint32_t)p->ndt_min_samples) {
    *delta = lm;
    *d_lmiss = 1.0;
    *d_sig = 0.0;
    return;
  }
  double d[3], w[3];
  double dd = 0.0, wd = 0.0;
  for (int a = 0; a < 3; ++a) {
    d[a] = e[a] - o[a];
    w[a] = mu_w[a] - o[a];
    dd += d[a] * d[a];
    wd += w[a] * d[a];
  }
  double t = dd > 0.0 ? wd / dd : 0.0;
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  double D[3];
  for (int a = 0; a < 3; ++a) D[a] = (o[a] + t * d[a]) - mu_w[a];
  double sn = p->sensor_noise, s2 = sn * sn;
  double S[3][3] = {{cov[0] + s2, cov[1], cov[2]}, {cov[1], cov[3] + s2, cov[4]}, {cov[2], cov[4], cov[5] + s2}};
  /* y = S^-1 D by Gaussian elimination (S is SPD, no pivoting needed) */
  double A[3][4];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) A[i][j] = S[i][j];
    A[i][3] = D[i];
  }
  for (int c = 0; c < 3; ++c)
    for (int r = c + 1; r < 3; ++r) {
      double f = A[r][c] / A[c][c];
      for (int j = c; j < 4; ++j) A[r][j] -= f * A[c][j];
    }
  double y[3];
  for (int r = 2; r >= 0; --r) {
    double acc = A[r][3];
    for (int j = r + 1; j < 3; ++j) acc -= A[r][j] * y[j];
    y[r] = acc / A[r][r];
  }
  double q = D[0] * y[0] + D[1] * y[1] + D[2] * y[2];
  double yy = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
  double g = exp(-0.5 * q);
  double sg = sigmoid_d(lm);
  double lam = p->adaptation_rate;
  double pr = 0.5 - lam * g * (0.5 - sg);
  double inv = 1.0 / (pr * (1.0 - pr));
  *delta = log(pr / (1.0 - pr));
  *d_lmiss = lam * g * sg * (1.0 - sg) * inv;
  *d_sig = -lam * (0.5 - sg) * g * sn * yy * inv;
}

static double bce_logit(double l, double y) {
  /* -[y log s(l) + (1-y) log(1 - s(l))], stable in l */
  double a = l > 0 ? l : 0.0;
  return a - l * y + log(exp(-a) + exp(l - a));
}

/*
 * Forward + (optionally) analytic gradients.  Window = loss box.
 *   labels, mask   [dz][dy][dx] fp64 (y_v, m_v)
 *   loss           out: L
 *   occ            optional out [dz][dy][dx] fp64: final l
 *   clamp_last     optional out [dz][dy][dx] uint32: c_v
 *   near           optional out [dz][dy][dx] uint8: pre-clamp value came within
 *                  near_eps of a bound in some scan
 *   grad_w         optional out [N] fp64 (only with grads != 0)
 *   grad_s         optional out [3] fp64: d/d(l_hit, l_miss, sensor_noise)
 */
int orc_adjoint(const orc_params* p, int32_t ndt, int32_t n_scans, const uint32_t* offsets, const float* origins,
                const float* samples, const float* weights, const int32_t box_min[3], const int32_t box_dim[3],
                const double* labels, const double* mask, double near_eps, int32_t grads, double* loss,
                double* occ_out, uint32_t* clamp_last_out, unsigned char* near_out, double* grad_w,
                double* grad_s) {
  size_t nv = (size_t)box_dim[0] * box_dim[1] * box_dim[2];
  double* l = (double*)malloc(nv * sizeof(double));
  double* wh = (double*)calloc(nv, sizeof(double));
  double* um = (double*)calloc(nv, sizeof(double));
  unsigned char* touched = (unsigned char*)calloc(nv, 1);
  uint32_t* cl = (uint32_t*)calloc(nv, sizeof(uint32_t));
  unsigned char* nr = (unsigned char*)calloc(nv, 1);
  uint32_t* nn = (uint32_t*)calloc(nv, sizeof(uint32_t));
  double* mu = (double*)calloc(nv * 3, sizeof(double));
  double* cv = (double*)calloc(nv * 6, sizeof(double));
  double* G = (double*)calloc(nv, sizeof(double));
  if (!l || !wh || !um || !touched || !cl || !nr || !nn || !mu || !cv || !G) return -1;
  for (size_t v = 0; v < nv; ++v) l[v] = (double)p->l_init;
  double lmin = (double)p->l_min, lmax = (double)p->l_max;
  orc_scratch s = {0};
  for (int pass = 0; pass < (grads ? 2 : 1); ++pass) {
    if (pass == 1) {
      /* backward: replay statistics from empty */
      memset(nn, 0, nv * sizeof(uint32_t));
      memset(mu, 0, nv * 3 * sizeof(double));
      memset(cv, 0, nv * 6 * sizeof(double));
      if (grad_s) grad_s[0] = grad_s[1] = grad_s[2] = 0.0;
    }
    for (int32_t sc = 0; sc < n_scans; ++sc) {
      uint32_t tag = (uint32_t)sc + 1;
      if (pass == 0) {
        memset(wh, 0, nv * sizeof(double));
        memset(um, 0, nv * sizeof(double));
        memset(touched, 0, nv);
      }
      const float* of = origins + 3 * sc;
      double o[3] = {(double)of[0], (double)of[1], (double)of[2]};
      for (uint32_t i = offsets[sc]; i < offsets[sc + 1]; ++i) {
        orc_ray r;
        prepare_weighted_ray(p, of, samples, weights, i, &r);
        if (pass == 1 && grad_w) grad_w[i] = 0.0;
        if (r.status != ORC_RAY_OK) continue;
        int clipped = 0;
        int64_t nk = walk_ray(p, &r, &s, &clipped);
        int has_hit = !r.truncated && !clipped;
        double w = weights ? (double)weights[i] : 1.0;
        double gw = 0.0;
        for (int64_t j = 0; j < nk; ++j) {
          const int32_t* key = s.keys + 3 * j;
          int64_t v = box_index(key, box_min, box_dim);
          if (v < 0) continue;
          int is_hit = has_hit && j == nk - 1;
          double delta, dlm, dsig;
          if (is_hit) {
            delta = (double)p->l_hit;
            dlm = dsig = 0.0;
          } else if (ndt) {
            double c[3], muw[3];
            voxel_centre(p, key, c);
            for (int a = 0; a < 3; ++a) muw[a] = c[a] + mu[3 * v + a];
            ndt_miss_terms(p, o, r.end, muw, cv + 6 * v, nn[v], &delta, &dlm, &dsig);
          } else {
            delta = (double)p->l_miss;
            dlm = 1.0;
            dsig = 0.0;
          }
          if (pass == 0) {
            touched[v] = 1;
            if (is_hit)
              wh[v] += w;
            else
              um[v] += w * delta;
          } else if (G[v] != 0.0 && tag > cl[v]) {
            gw += G[v] * delta;
            if (grad_s) {
              if (is_hit)
                grad_s[0] += w * G[v];
              else {
                grad_s[1] += w * G[v] * dlm;
                grad_s[2] += w * G[v] * dsig;
              }
            }
          }
        }
        if (pass == 1 && grad_w) grad_w[i] = gw;
      }
      if (pass == 0) {
        for (size_t v = 0; v < nv; ++v) {
          if (!touched[v]) continue;
          double sv = (l[v] + wh[v] * (double)p->l_hit) + um[v];
          if (sv < lmin || sv > lmax) cl[v] = tag;
          if (fabs(sv - lmin) < near_eps || fabs(sv - lmax) < near_eps) nr[v] = 1;
          l[v] = clampd_(sv, lmin, lmax);
        }
      }
      if (ndt) {
        /* fold the scan's samples (ascending ray order) */
        for (uint32_t i = offsets[sc]; i < offsets[sc + 1]; ++i) {
          orc_ray r;
          prepare_weighted_ray(p, of, samples, weights, i, &r);
          if (r.status != ORC_RAY_OK || r.truncated) continue;
          int clipped = 0;
          int64_t nk = walk_ray(p, &r, &s, &clipped);
          if (clipped) continue;
          const int32_t* key = s.keys + 3 * (nk - 1);
          int64_t v = box_index(key, box_min, box_dim);
          if (v < 0) continue;
          double c[3], x[3];
          voxel_centre(p, key, c);
          const float* e = samples + 3 * (size_t)i;
          for (int a = 0; a < 3; ++a) x[a] = (double)e[a] - c[a];
          welford_add(nn + v, mu + 3 * v, cv + 6 * v, x);
        }
      }
    }
    if (pass == 0) {
      double L = 0.0;
      for (size_t v = 0; v < nv; ++v) {
        if (mask[v] == 0.0) continue;
        L += mask[v] * bce_logit(l[v], labels[v]);
        G[v] = mask[v] * (sigmoid_d(l[v]) - labels[v]);
      }
      *loss = L;
    }
  }
  if (occ_out) memcpy(occ_out, l, nv * sizeof(double));
  if (clamp_last_out) memcpy(clamp_last_out, cl, nv * sizeof(uint32_t));
  if (near_out) memcpy(near_out, nr, nv);
  scratch_free(&s);
  free(l);
  free(wh);
  free(um);
  free(touched);
  free(cl);
  free(nr);
  free(nn);
  free(mu);
  free(cv);
  free(G);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Voxel mean layer                                                        */
/* ---------------------------------------------------------------------- */
/*
 * The voxel mean layer (paper Sec. III-A: a 32-bit discretised mean
 * position, 10 bits of sub-voxel position per axis packed into one word,
 * beside a 32-bit count of the samples behind it; updated like occupancy,
 * by compare-and-swap, Sec. III-B).  Readings (design notes):
 *   - A sample's code per axis is its position inside its voxel in units of
 *     1/1024 voxel, rounded down: from the fixed-point sample q (2^F units
 *     per voxel), c = (q - k 2^F) >> (F - 10) (or << (10 - F) when F < 10).
 *   - Packed word: x | y << 10 | z << 20.
 *   - Merging k samples with code sum S into a voxel holding count n and
 *     code c gives, per axis, the rational mean (n c + S) / (n + k) rounded
 *     half up: floor((2 (n c + S) + (n + k)) / (2 (n + k))); the count
 *     becomes n + k (saturating at 2^32 - 1).
 *   - Count mode merges each scan's samples of a voxel in one step (per scan,
 *     like count-then-clamp); per-update mode merges one sample at a time,
 *     here in ascending ray order (the GPU's order is unspecified).
 *   - Samples come from the rays that carry a hit (not truncated, end voxel
 *     in the map); ray weights do not weight samples.
 *   packed, count  [dz][dy][dx] uint32, in/out
 */
static uint32_t subvoxel_code(int64_t q, int64_t k, int F) {
  int64_t f = q - k * ((int64_t)1 << F); /* in [0, 2^F) */
  return (uint32_t)(F >= 10 ? (f >> (F - 10)) : (f << (10 - F)));
}

static uint32_t mean_merge_axis(uint64_t n, uint32_t c, uint64_t k, uint64_t sum) {
  uint64_t tot = n + k;
  uint64_t num = 2 * (n * (uint64_t)c + sum) + tot;
  return (uint32_t)(num / (2 * tot));
}

static void mean_merge(uint32_t* packed, uint32_t* count, uint64_t k, const uint64_t sum[3]) {
  if (k == 0) return;
  uint64_t n = *count;
  uint32_t out = 0;
  for (int a = 0; a < 3; ++a) {
    uint32_t c = (*packed >> (10 * a)) & 1023u;
    out |= mean_merge_axis(n, c, k, sum[a]) << (10 * a);
  }
  *packed = out;
  uint64_t t = n + k;
  *count = t > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)t;
}

int orc_mean_integrate(const orc_params* p, int32_t mode, int32_t n_scans, const uint32_t* offsets,
                       const float* origins, const float* samples, const float* weights, const int32_t box_min[3],
                       const int32_t box_dim[3], uint32_t* packed, uint32_t* count) {
  size_t nv = (size_t)box_dim[0] * box_dim[1] * box_dim[2];
  uint64_t* acc = (uint64_t*)calloc(nv * 4, sizeof(uint64_t)); /* k, sum x, sum y, sum z */
  if (!acc) return -1;
  orc_scratch s = {0};
  for (int32_t sc = 0; sc < n_scans; ++sc) {
    memset(acc, 0, nv * 4 * sizeof(uint64_t));
    const float* of = origins + 3 * sc;
    for (uint32_t i = offsets[sc]; i < offsets[sc + 1]; ++i) {
      orc_ray r;
      prepare_weighted_ray(p, of, samples, weights, i, &r);
      if (r.status != ORC_RAY_OK || r.truncated) continue;
      int clipped = 0;
      int64_t nk = walk_ray(p, &r, &s, &clipped);
      if (clipped) continue;
      const int32_t* key = s.keys + 3 * (nk - 1);
      int64_t v = box_index(key, box_min, box_dim);
      if (v < 0) continue;
      uint64_t code[3];
      for (int a = 0; a < 3; ++a) code[a] = subvoxel_code(r.q1[a], r.k1[a], p->fixed_bits);
      if (mode == 1) {
        acc[4 * v] += 1;
        for (int a = 0; a < 3; ++a) acc[4 * v + 1 + a] += code[a];
      } else {
        mean_merge(packed + v, count + v, 1, code);
      }
    }
    if (mode == 1)
      for (size_t v = 0; v < nv; ++v) mean_merge(packed + v, count + v, acc[4 * v], acc + 4 * v + 1);
  }
  scratch_free(&s);
  free(acc);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Decay-rate layer                                                        */
/* ---------------------------------------------------------------------- */
/*
 * Decay-rate map (paper Sec. II-E): reflections occur at a constant rate
 * lambda_i inside voxel i, estimated as H_i / sum_j d_i(j), H_i the samples
 * that fell in the voxel and d_i(j) the distance ray j travels through it.
 * Readings (design notes): the distance is measured along the quantised
 * segment the walk traverses (the same exact crossings), so a voxel entered
 * at ray parameter t0 and left at t1 receives (t1 - t0) L, with L the
 * segment's length in metres, t = (b_a + j 2^F) / A_a the crossing
 * parameters and t = 0, 1 at the segment ends; a clipped ray stops at the
 * crossing that leaves the map.  Every voxel the walk visits is counted
 * (zero-length visits add 0); H counts the rays that carry a hit.  Pure
 * sums: both batch modes give the same result.
 *   length  [dz][dy][dx] fp64, in/out (metres)
 *   hits    [dz][dy][dx] uint32, in/out
 */
int orc_decay_integrate(const orc_params* p, int32_t n_scans, const uint32_t* offsets, const float* origins,
                        const float* samples, const float* weights, const int32_t box_min[3],
                        const int32_t box_dim[3], double* length, uint32_t* hits) {
  orc_scratch s = {0};
  const double unit = p->voxel_size / ldexp(1.0, p->fixed_bits); /* metres per fixed-point unit */
  for (int32_t sc = 0; sc < n_scans; ++sc) {
    const float* of = origins + 3 * sc;
    for (uint32_t i = offsets[sc]; i < offsets[sc + 1]; ++i) {
      orc_ray r;
      prepare_weighted_ray(p, of, samples, weights, i, &r);
      if (r.status != ORC_RAY_OK) continue;
      int clipped = 0;
      int64_t nk = walk_ray(p, &r, &s, &clipped);
      double d2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        double D = (double)(r.q1[a] - r.q0[a]);
        d2 += D * D;
      }
      const double L = sqrt(d2) * unit;
      /* after walk_ray, s.ev[j] is the crossing that enters visited voxel j + 1
         (or, for a clipped ray, event nk - 1 leaves the map) */
      double t0 = 0.0;
      for (int64_t j = 0; j < nk; ++j) {
        double t1 = 1.0;
        if (j + 1 < nk || clipped) t1 = (double)s.ev[j].num / (double)s.ev[j].den;
        int64_t v = box_index(s.keys + 3 * j, box_min, box_dim);
        if (v >= 0) length[v] += (t1 - t0) * L;
        t0 = t1;
      }
      if (!r.truncated && !clipped) {
        int64_t v = box_index(s.keys + 3 * (nk - 1), box_min, box_dim);
        if (v >= 0) hits[v] += 1;
      }
    }
  }
  scratch_free(&s);
  return 0;
}

/* Library self-identification for the loaders. */
int orc_abi_version(void) { return 1; }

#ifndef ORC_SOURCE_DIGEST
#define ORC_SOURCE_DIGEST "unknown"
#endif
/* sha256 of the source this library was built from (set by the build). */
const char* orc_source_digest(void) { return ORC_SOURCE_DIGEST; }
