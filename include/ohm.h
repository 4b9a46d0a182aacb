/*
 * ohm.h -- C ABI of the MI355X lidar ray-integration library.
 *
 * The library integrates batches of lidar rays (sensor origin -> sample
 * point) into a 3D log-odds occupancy map held in GPU memory, following
 * Stepanas et al., "OHM: GPU Based Occupancy Map Generation":
 *   - Sec. II-B, Eq. (2)-(3) and the clamping paragraph: each voxel keeps a
 *     log-odds value l; a ray adds l_miss (< 0) to every voxel it passes
 *     through and l_hit (> 0) to the voxel holding its sample, and l is kept
 *     inside [l_min, l_max].
 *   - Sec. III-A: space is split into dense cubic regions (here 32^3 voxels)
 *     found through a region table, each region holding contiguous per-voxel
 *     layers.
 *   - Sec. III-B: one GPU thread per ray walks the ray voxel by voxel (the
 *     Amanatides & Woo line walk, one face-adjacent voxel per step) and
 *     updates global memory atomically.
 *   - Sec. II-D and III-C: the NDT-OM variant keeps per-voxel sample
 *     statistics and weights a miss by how well the ray agrees with them;
 *     misses are applied first, then all of a batch's samples per voxel.
 *   - Sec. IV-A: rays are truncated to a maximum range.
 *
 * Conventions (all entry points):
 *   - Device pointers (prefix d_) are HIP device pointers owned by the
 *     caller.  Host pointers (prefix h_) are read before the call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls enqueue their kernels on it and return without synchronising,
 *     except ohm_map_sync_status and the *_size queries.
 *   - The library allocates no device memory: a map lives in a caller-
 *     provided workspace whose size ohm_map_workspace_size reports.  The
 *     handle (host memory) is owned by the library until ohm_map_destroy.
 *   - Argument errors are returned synchronously and enqueue nothing.
 *     Data-dependent conditions are not errors: non-finite or unrepresentable
 *     rays and rays whose origin is outside the map are skipped and counted;
 *     updates into regions that do not fit in the region pool are dropped,
 *     counted and flag `sticky_error` (see ohm_map_stats).
 *   - A handle is not thread-safe; use one stream per map at a time.
 *   - No C++ exception crosses this interface.
 *
 * Frame and exactness.  A voxel key k covers [m + k s, m + (k+1) s) per axis
 * (m = map_origin, s = voxel_size).  Each point is quantised once to fixed
 * point, q = rint((p - m) * 2^F / s) in IEEE double (F = fixed_bits); its key
 * is floor(q / 2^F).  The walk then decides every step with exact 64-bit
 * integer arithmetic: it visits the start voxel and applies each voxel-face
 * crossing of the segment in increasing order of its ray parameter,
 * simultaneous crossings taking the lower axis (x, y, z) first.  A ray is
 * clipped at the first key outside [key_min, key_max) and then carries no hit.
 * A ray longer than max_range is shortened to max_range and carries no hit;
 * every voxel it visits, the last included, takes a miss.
 */
#ifndef OHM_H
#define OHM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ohm_map_s* ohm_map;

typedef enum {
  OHM_OK = 0,
  OHM_E_INVALID_ARG = -1,
  OHM_E_NO_DEVICE = -2,
  OHM_E_HIP = -3,
  OHM_E_WORKSPACE_TOO_SMALL = -4,
  OHM_E_UNSUPPORTED = -5
} ohm_status;

/* Batch semantics.
 * OHM_MODE_PER_UPDATE: every hit and miss is applied as l <- clamp(l + delta)
 *   with an atomic compare-and-swap, in whatever order the GPU produces
 *   (the paper's CAS update, Sec. III-B).  Where clamping never engages the
 *   result equals the plain sum; elsewhere it lies between "all hits first"
 *   and "all misses first".
 * OHM_MODE_COUNT_CLAMP: per scan, each voxel's hit and miss weights are
 *   accumulated and applied once, l <- clamp((l + H*l_hit) + M*l_miss) in
 *   fp32 without contraction.  Deterministic; bit-exact for unit weights. */
enum { OHM_MODE_PER_UPDATE = 0, OHM_MODE_COUNT_CLAMP = 1 };

/* Optional layers requested at map creation (bit mask). */
enum {
  OHM_LAYER_OCC = 1,         /* always present */
  OHM_LAYER_NDT = 2,         /* NDT-OM sample count, mean and covariance */
  OHM_LAYER_ADJOINT = 4,     /* last scan at which the clamp was active */
  OHM_LAYER_SCAN_GROUPS = 8, /* G accumulator slots (default 8): in count mode, ohm_integrate_rays
                                walks up to G consecutive scans of a call in one launch (each
                                into its own slot, finalized in scan order: the same result).
                                Each slot costs 256 KiB per region of capacity; a weighted scan
                                uses two slots.  Every map has at least two slots' memory. */
  OHM_LAYER_MEAN = 16,       /* voxel mean (paper Sec. III-A): per voxel a 32-bit word packing the
                                10-bit sub-voxel position code of each axis (x bits 0-9, y 10-19,
                                z 20-29) and a 32-bit sample count.  A sample's code is its
                                position inside its voxel in 1/1024 voxel, rounded down, from the
                                quantised sample; merging k samples (code sum S) into (n, c) gives
                                floor((2 (n c + S) + n + k) / (2 (n + k))) per axis and n + k.
                                Per-update mode merges each sample by 64-bit compare-and-swap;
                                count mode merges each scan's samples in one step, in scan order
                                (exact).  Updated by ohm_integrate_rays; 8 B per voxel plus 16 B
                                per voxel and accumulator slot, and 8 B per voxel of slot mask. */
  OHM_LAYER_DECAY = 32,      /* decay rate (paper Sec. II-E): per voxel the summed distance rays
                                travel through it, measured along the quantised segment the walk
                                traverses (Q32.32 metres, exact integer sums), and the samples
                                that fell in it; the rate is their quotient.  Updated by
                                ohm_integrate_rays in both modes (plain sums).  12 B per voxel. */
  OHM_LAYER_NDT_TM = 64,     /* NDT-TM (paper Sec. II-D, III-C; requires OHM_LAYER_NDT): per voxel the
                                misses M behind the permeability H / (H + M) (H = the NDT sample
                                count) and a 1D Gaussian (mean, population variance) of the
                                intensity of the samples that fell in it.  A miss counts toward M
                                when the voxel held >= ndt_min_samples samples before the scan and
                                the squared Mahalanobis distance q = D^T S^-1 D of the ray's closest
                                point (as in the NDT-OM weighting) is <= ndt_tm_gate.  Updated by
                                ohm_ndt_tm_integrate; cleared with the NDT statistics.  12 B per
                                voxel plus 16 B of per-scan intensity moments. */
  OHM_LAYER_TSDF = 128       /* truncated signed distance (paper Sec. II-F): per voxel a distance D
                                and a weight W (float, packed in one 64-bit word), updated by
                                ohm_tsdf_integrate.  8 B per voxel plus 16 B of per-scan sums. */
};
/* OHM_LAYER_MEAN and OHM_LAYER_DECAY are not available together with
 * OHM_LAYER_NDT (OHM_E_UNSUPPORTED at creation), nor in batched plans;
 * OHM_LAYER_NDT_TM needs OHM_LAYER_NDT (OHM_E_INVALID_ARG without it). */

/* Slot count of OHM_LAYER_SCAN_GROUPS, or-ed into the layer mask: n in [1, 64]
 * (0: the default 8).  Only valid together with OHM_LAYER_SCAN_GROUPS. */
#define OHM_SCAN_GROUP_SLOTS(n) ((uint32_t)(n) << 8)

/* Quantities readable with ohm_map_read_dense (output element type). */
enum {
  OHM_READ_OCC = 0,        /* float   log-odds (l_init where never touched) */
  OHM_READ_HITS = 1,       /* float   hit weight of the last scan (count mode) */
  OHM_READ_MISSES = 2,     /* float   miss weight of the last scan (count mode; NDT: summed miss delta) */
  OHM_READ_NDT_COUNT = 3,  /* uint32  NDT sample count */
  OHM_READ_NDT_MEAN = 4,   /* float[3] NDT mean, metres, relative to the voxel centre */
  OHM_READ_NDT_COV = 5,    /* float[6] NDT covariance xx, xy, xz, yy, yz, zz (m^2) */
  OHM_READ_CLAMP_SCAN = 6, /* uint32  1 + last scan index whose pre-clamp value left [l_min, l_max], 0 = never */
  OHM_READ_MEAN_PACKED = 7,  /* uint32  packed 10-bit mean codes (OHM_LAYER_MEAN) */
  OHM_READ_MEAN_COUNT = 8,   /* uint32  samples behind the mean */
  OHM_READ_MEAN = 9,         /* float[3] mean position, metres from the voxel centre (code cell centres;
                                0 where no sample) */
  OHM_READ_DECAY_LENGTH = 10,/* float   summed distance through the voxel, metres (OHM_LAYER_DECAY) */
  OHM_READ_DECAY_HITS = 11,  /* uint32  samples that fell in the voxel */
  OHM_READ_DECAY_RATE = 12,  /* float   hits / distance (per metre; 0 where no distance) */
  OHM_READ_TM_MISSES = 13,   /* uint32  NDT-TM checked misses M (OHM_LAYER_NDT_TM) */
  OHM_READ_TM_PERMEABILITY = 14, /* float H / (H + M), H the NDT sample count; 0 where H + M = 0 */
  OHM_READ_INTENSITY_MEAN = 15,  /* float NDT-TM intensity mean (0 where no sample) */
  OHM_READ_INTENSITY_VAR = 16,   /* float NDT-TM intensity population variance */
  OHM_READ_TSDF_DISTANCE = 17,   /* float TSDF distance D, metres (0 where never observed) */
  OHM_READ_TSDF_WEIGHT = 18      /* float TSDF weight W (0 where never observed) */
};

typedef struct {
  double voxel_size;       /* metres, > 0 */
  double map_origin[3];    /* world position of key (0,0,0)'s min corner */
  int32_t key_min[3];      /* map bounds in keys, half-open [key_min, key_max) */
  int32_t key_max[3];
  int32_t region_log2;     /* region edge = 2^region_log2 voxels; must be 5 */
  int32_t fixed_bits;      /* F in [8, 20]; 16 gives 1/65536-voxel resolution */
  float l_hit;             /* > 0 (paper's example values: +0.847) */
  float l_miss;            /* < 0 (-0.405) */
  float l_min, l_max;      /* clamp bounds, l_min < l_max */
  float l_init;            /* value of never-touched voxels, in [l_min, l_max] */
  double max_range;        /* metres; <= 0 disables truncation */
  int32_t mode;            /* OHM_MODE_* */
  float sensor_noise;      /* NDT: sensor noise sigma in metres (> 0) */
  float adaptation_rate;   /* NDT: lambda in [0, 1] */
  uint32_t ndt_min_samples;/* NDT: samples needed before a voxel's Gaussian is used (>= 2) */
  float ndt_clear_below;   /* NDT: clear sample data where l < this after a scan's
                              misses; -INFINITY disables */
  double ndt_tm_gate;      /* NDT-TM: largest squared Mahalanobis distance of a miss that
                              counts toward M (> 0; 9 = three standard deviations) */
  double tsdf_truncation;  /* TSDF: band half-width tau along the ray, metres (> 0) */
  double tsdf_max_weight;  /* TSDF: weight cap (>= 1) */
} ohm_params;

typedef struct {
  uint64_t rays_in;             /* rays submitted */
  uint64_t rays_invalid;        /* non-finite or unrepresentable (skipped) */
  uint64_t rays_origin_oob;     /* origin outside the map (skipped) */
  uint64_t rays_truncated;      /* shortened to max_range */
  uint64_t rays_clipped;        /* left the map before their sample */
  uint64_t rays_hit;            /* applied a hit */
  uint64_t voxel_updates;       /* hits + misses applied (dropped ones excluded) */
  uint64_t updates_dropped_pool;/* updates lost to a full region pool */
  uint32_t regions_used;
  uint32_t region_capacity;
  int32_t sticky_error;         /* bit 0: region pool exhausted; bit 1: a region slot being
                                   published by another block never appeared (updates dropped);
                                   bit 2: a ray weight was negative or not finite (ray skipped,
                                   counted in rays_invalid) */
  int32_t reserved;
} ohm_map_stats;

/* Bytes of device workspace a map needs.  region_capacity is the number of
 * 32^3 regions the map can hold; layers is an OHM_LAYER_* mask, optionally
 * with OHM_SCAN_GROUP_SLOTS(n). */
ohm_status ohm_map_workspace_size(const ohm_params* params, uint32_t region_capacity, uint32_t layers,
                                  size_t* bytes);

/* Create a map in d_workspace (>= ohm_map_workspace_size bytes, 256-byte
 * aligned, owned by the caller and untouched by ohm_map_destroy).  Enqueues
 * the map's initialisation on `stream`. */
ohm_status ohm_map_create(const ohm_params* params, uint32_t region_capacity, uint32_t layers, void* d_workspace,
                          size_t workspace_bytes, void* stream, ohm_map* out);

ohm_status ohm_map_destroy(ohm_map map);

/* Return every voxel to l_init (and NDT/adjoint layers to zero), free all
 * regions and clear the statistics. */
ohm_status ohm_map_reset(ohm_map map, void* stream);

/* Update parameters that do not change the map layout (l_*, max_range, mode,
 * NDT parameters).  Frame, bounds, region size and fixed_bits must match. */
ohm_status ohm_map_set_params(ohm_map map, const ohm_params* params);

/*
 * Integrate n_scans scans of rays (occupancy update, paper Sec. III-B).
 *   d_origins       float[n_scans][3]   sensor position of each scan
 *   d_samples       float[N][3]         sample points, N = h_scan_offsets[n_scans]
 *   h_scan_offsets  uint32[n_scans+1]   HOST array; scan s owns rays
 *                                       [h_scan_offsets[s], h_scan_offsets[s+1])
 *   d_weights       float[N] or NULL    per-ray weight scaling that ray's hit and
 *                                       miss increments (NULL = 1); each must be
 *                                       finite and >= 0: a ray with any other
 *                                       weight is skipped whole, counted in
 *                                       rays_invalid, and sets sticky_error bit 2
 * Scan offsets are a host array, not device memory: the host sizes every
 * launch from the scans' sizes and cuts scan groups from them, which device
 * offsets would make a synchronising copy per call.
 * Scans are applied in order; in count mode each scan is one batch with one
 * clamp per voxel.  In count mode the last scan's hit/miss weights remain
 * readable (OHM_READ_HITS / OHM_READ_MISSES) until the next call.  On a map
 * with OHM_LAYER_SCAN_GROUPS, count mode walks up to G consecutive scans of
 * the call in one launch (unless ray-order scratch is attached) and applies
 * them per voxel in scan order: the result is the same.
 */
ohm_status ohm_integrate_rays(ohm_map map, const float* d_origins, const float* d_samples,
                              const uint32_t* h_scan_offsets, uint32_t n_scans, const float* d_weights,
                              void* stream);


/*
 * Integrate scans into an NDT-OM map (created with OHM_LAYER_NDT; paper
 * Sec. II-D and III-C).  Per scan: phase 1 walks every ray and applies its
 * misses, each weighted by the voxel's Gaussian: for a voxel holding at least
 * ndt_min_samples samples with mean mu and covariance Sigma, with x* the point
 * of the ray segment closest to mu, S = Sigma + sensor_noise^2 I and
 * g = exp(-0.5 (x*-mu)^T S^-1 (x*-mu)), the miss is
 *   delta = logit(0.5 - lambda * g * (0.5 - sigmoid(l_miss)))
 * (plain l_miss for voxels with fewer samples).  Phase 2 folds every sample
 * of the scan into its voxel's count, mean and covariance (population
 * covariance, mean relative to the voxel centre) and applies the hits.
 * Arguments as for ohm_integrate_rays.
 */
ohm_status ohm_ndt_integrate(ohm_map map, const float* d_origins, const float* d_samples,
                             const uint32_t* h_scan_offsets, uint32_t n_scans, const float* d_weights,
                             void* stream);

/*
 * NDT-TM integration (map created with OHM_LAYER_NDT | OHM_LAYER_NDT_TM;
 * paper Sec. II-D and III-C): everything ohm_ndt_integrate does, plus, per
 * scan, the checked misses M (see OHM_LAYER_NDT_TM; decided on the voxel's
 * statistics from before the scan, like the NDT-OM weight, and counted
 * whatever the ray's weight) and, in the second phase, the intensities of
 * the scan's samples merged into each voxel's intensity mean and population
 * variance (pairwise merge of the scan's moments, in fp64).
 *   d_intensities  float[N]: one intensity per ray (required)
 * Other arguments as for ohm_ndt_integrate.  ohm_ndt_integrate itself
 * returns OHM_E_INVALID_ARG on an NDT-TM map (it has no intensities).
 */
ohm_status ohm_ndt_tm_integrate(ohm_map map, const float* d_origins, const float* d_samples,
                                const float* d_intensities, const uint32_t* h_scan_offsets, uint32_t n_scans,
                                const float* d_weights, void* stream);

/*
 * TSDF integration (map created with OHM_LAYER_TSDF; paper Sec. II-F).  Only
 * a ray with a surface takes part: valid, origin in the map, not truncated
 * by max_range, sample voxel in the map and of non-zero length.  With
 * r = |e - o| and u = (e - o) / r (fp64), its band is the segment from
 * o + max(r - tau, 0) u to o + (r + tau) u, tau = tsdf_truncation; both
 * ends are quantised like ray ends and the band is walked exactly (clipped
 * at the map's bounds; a band whose first voxel is outside the map is
 * skipped).  Each band voxel with centre c takes the projective distance
 * sd = clamp(r - (c - o).u, -tau, tau) (positive in front of the surface).
 * A voxel keeps (D, W), both 0 until observed; n updates of summed distance
 * S give D <- (W D + S) / (W + n), W <- min(W + n, tsdf_max_weight), in fp64,
 * stored as float.  Count mode sums each scan's distances per voxel (Q32.32
 * integers: exact and order-free) and applies them once per scan;
 * per-update mode applies every update at once by 64-bit compare-and-swap on
 * the packed (D, W) word, in whatever order the GPU produces.  Statistics:
 * rays_hit counts rays with a band, voxel_updates the band voxels inside the
 * map.  The occupancy layer is not touched.  Arguments as for
 * ohm_integrate_rays without weights.
 */
ohm_status ohm_tsdf_integrate(ohm_map map, const float* d_origins, const float* d_samples,
                              const uint32_t* h_scan_offsets, uint32_t n_scans, void* stream);

/*
 * Adjoint of count-mode integration (the gradient of a loss on the final
 * log-odds; forward per scan k and voxel v: s = (l + H l_hit) + U,
 * l <- clamp(s), with H the summed hit weight and U the summed weighted miss
 * increments).  Requirements: the map was created with OHM_LAYER_ADJOINT,
 * mode OHM_MODE_COUNT_CLAMP, and since its last create / reset has integrated
 * exactly these scans (same arguments) with ohm_ndt_integrate (ndt != 0,
 * NDT clearing disabled) or ohm_integrate_rays (ndt == 0).
 *   d_grad          float[box_dim z][y][x]: dL/dl (final log-odds) over the box
 *                   at h_box_min; voxels outside the box have zero gradient
 *   d_grad_weights  float[N] or NULL: receives dL/dw_r for every ray
 *                   (0 for skipped rays)
 *   d_grad_scalars  double[3]: receives dL/d(l_hit, l_miss, sensor_noise)
 *                   (overwritten, not accumulated)
 * `ndt` says which forward to differentiate: a map with the NDT layer can also
 * be integrated with ohm_integrate_rays (occupancy only), so the layer mask
 * alone cannot tell.
 * The traversals are recomputed, not stored.  For NDT maps the sample
 * statistics are rebuilt in place scan by scan and hold the same values
 * afterwards.  Returns OHM_E_UNSUPPORTED for per-update mode or enabled NDT
 * clearing (neither is differentiable here).
 */
ohm_status ohm_backward(ohm_map map, int32_t ndt, const float* d_grad, const int32_t h_box_min[3],
                        const int32_t h_box_dim[3], const float* d_origins, const float* d_samples,
                        const uint32_t* h_scan_offsets, uint32_t n_scans, const float* d_weights,
                        float* d_grad_weights, double* d_grad_scalars, void* stream);

/*
 * Copy a dense box of one quantity to d_out, laid out [box_dim z][y][x]
 * (x fastest) with the element type listed for `what`.  Voxels outside the
 * map or in unallocated regions read as never touched.
 */
ohm_status ohm_map_read_dense(ohm_map map, int32_t what, const int32_t h_box_min[3], const int32_t h_box_dim[3],
                              void* d_out, void* stream);

/*
 * Debug / verification: the update list of every ray, produced by the same
 * walk the integration kernels run.  Two passes:
 *   pass 1 (d_updates == NULL): writes d_ray_counts[i] (uint32, updates of
 *     ray i) and d_ray_flags[i] (bit 0 truncated, 1 clipped, 2 hit,
 *     3 invalid, 4 origin outside the map);
 *   pass 2: with d_ray_offsets[i] (int64, exclusive prefix sum of the counts)
 *     writes ray i's updates to d_updates[d_ray_offsets[i] + j] as int32
 *     (kx, ky, kz, kind), kind 0 = miss, 1 = hit, in walk order.
 * The map is not modified.
 */
ohm_status ohm_debug_trace_rays(ohm_map map, const float* d_origins, const float* d_samples,
                                const uint32_t* h_scan_offsets, uint32_t n_scans, uint32_t* d_ray_counts,
                                int32_t* d_ray_flags, const int64_t* d_ray_offsets, int32_t* d_updates,
                                void* stream);

/*
 * Batched integration (many scans of uneven size from several sensors into
 * several maps, one graph launch).  Each set names a map (count mode, one set
 * per map) and its scans in application order, with the same conventions as
 * ohm_integrate_rays.  A plan copies the sets' pointers, the maps' parameters
 * and the scan layout, so the buffers must stay valid and unchanged (contents
 * may change) for the plan's life.  Running a plan integrates every set's
 * scans into its map with exactly the per-scan count-then-clamp result of
 * calling ohm_integrate_rays scan by scan; scans of different maps run
 * concurrently.  tuning->group_scans (G, 1..64) scans per map share one walk
 * launch and one finalize; each group needs G per-scan accumulators of
 * capacity x 32^3 x 8 bytes per map in the plan workspace.
 *
 * This plan API stands in for a single "integrate batched" call: the
 * library allocates no device memory, so the plan's accumulators live in a
 * caller workspace sized by ohm_batch_workspace_size; the graph is captured
 * once and replayed per run instead of being rebuilt by every call; and a
 * set per map replaces a per-scan map index.  The schedule search (group
 * size, walk tile, ray order) and its on-disk cache are in the Python
 * binding (batch.autotune): it builds and times candidate plans, each of
 * which needs its own workspace, and allocation belongs to the caller.  C
 * callers pass an ohm_batch_tuning directly.
 */
typedef struct {
  ohm_map map;
  const float* d_origins;          /* float[n_scans][3] */
  const float* d_samples;          /* float[N][3] */
  const float* d_weights;          /* float[N] or NULL (all sets alike) */
  const uint32_t* h_scan_offsets;  /* uint32[n_scans + 1], host */
  uint32_t n_scans;
} ohm_scan_set;

typedef struct {
  uint32_t group_scans;      /* G: scans per map per launch group, 1..64 */
  uint32_t seg_major_steps;  /* walk segment length, as in ohm_walk_tuning (0: 16) */
  uint32_t tile_threads;     /* threads per 256-ray tile: 256, 512 or 1024 (0: 512) */
  uint32_t keep_ray_order;   /* 0: each run walks every scan's rays in direction order
                                (azimuth strips of about 2,048 rays, then elevation: a
                                tile covers a patch of directions about as wide as it is
                                tall), which keeps a tile's
                                rays together when a scan's directions arrive unordered;
                                nonzero: walk them in the given order (scans already in
                                sensor order).  Never changes results. */
} ohm_batch_tuning;

typedef struct ohm_batch_s* ohm_batch;

ohm_status ohm_batch_workspace_size(const ohm_scan_set* sets, uint32_t n_sets, const ohm_batch_tuning* tuning,
                                    size_t* bytes);
/* Build the plan in d_workspace (256-byte aligned, caller-owned) and capture
 * it as a graph; synchronises `stream` once. */
ohm_status ohm_batch_create(const ohm_scan_set* sets, uint32_t n_sets, const ohm_batch_tuning* tuning,
                            void* d_workspace, size_t workspace_bytes, void* stream, ohm_batch* out);
/* Launch the captured plan on `stream` (asynchronous). */
ohm_status ohm_batch_run(ohm_batch plan, void* stream);
ohm_status ohm_batch_destroy(ohm_batch plan);

/* Walk launch shape.  Each ray's walk is cut into segments of
 * seg_major_steps crossings of its major axis (the axis it travels furthest
 * along); a block of tile_threads threads (256, 512 or 1024) processes the
 * segments of 256 consecutive rays.  Affects speed only, never results.
 * Defaults: 16 and 512. */
typedef struct {
  uint32_t seg_major_steps;
  uint32_t tile_threads;
} ohm_walk_tuning;

ohm_status ohm_map_set_tuning(ohm_map map, const ohm_walk_tuning* tuning);

/* Direction ordering of the per-scan path (ohm_integrate_rays).  A walk
 * tile works best when its 256 rays point close together, as a spinning
 * lidar's scan order gives; a scan whose ray directions arrive unordered can
 * instead be walked in direction order (azimuth strips of about 256 rays,
 * then elevation: tiles of about equal work, which one scan's launch needs;
 * the batched plan's strips are eight tiles wide).  Attaching a scratch buffer turns this on for every scan
 * of at most max_rays rays (longer scans walk in their given order); it
 * costs three small kernels per scan and never changes results.
 * ohm_ray_order_scratch_size gives the bytes for max_rays (> 0).
 * d_scratch: caller-owned device memory, 256-byte aligned, at least that
 * size, valid until detached (d_scratch = NULL) or the map is destroyed;
 * calls on one map must not overlap while it is attached. */
ohm_status ohm_ray_order_scratch_size(uint32_t max_rays, size_t* bytes);
ohm_status ohm_map_set_ray_order(ohm_map map, void* d_scratch, size_t bytes, uint32_t max_rays);

/* Column layout of the map's scans, for the walk order of the grouped walk
 * (OHM_LAYER_SCAN_GROUPS, count mode).  column_rays = R > 0 declares that
 * every scan arrives as a column-major range image of R rays per column
 * (ray = column * R + beam), as a spinning multi-beam lidar (Table I)
 * emits it: each full chunk of 32 columns is then walked as R / 8 tiles of
 * 8 beams by 32 columns instead of 256 consecutive rays (4 columns of a
 * 64-beam sensor), patches about square in angle whose rays share about
 * twice as many voxels (a partial last chunk keeps the given order).  Only
 * the order of the walk changes, never the result; a scan not laid out so
 * is still integrated correctly, only without the gain.  The per-scan path
 * keeps the given order: one scan's launch has too few tiles to even out
 * the patches' unequal lengths.  R: 0 (the given order, the default) or a
 * multiple of 8 up to 65536; anything else is OHM_E_INVALID_ARG. */
ohm_status ohm_map_set_scan_layout(ohm_map map, uint32_t column_rays);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): ohm_integrate_rays with
 * direction ordering (as with ohm_map_set_ray_order) whose ordering scratch
 * is a fixed buffer inside the library instead of caller memory.  It
 * allocates nothing: no hipMalloc, no events (map profiling records nothing
 * for it).  Every scan is walked in direction order; a scan of more than
 * OHM_NO_ALLOC_MAX_RAYS rays is an argument error (nothing enqueued), and so
 * is a current device other than the map's.  The buffer (about 2 MiB) is
 * one per GPU, held until the process ends, and shared by every call on
 * that GPU: calls that overlap on one GPU (other streams, other threads)
 * race on it and must be serialised by the caller.  The result equals
 * ohm_integrate_rays on a map with ray ordering attached.
 */
#define OHM_NO_ALLOC_MAX_RAYS 262144u
ohm_status ohm_integrate_rays_no_alloc(ohm_map map, const float* d_origins, const float* d_samples,
                                       const uint32_t* h_scan_offsets, uint32_t n_scans, const float* d_weights,
                                       void* stream);

/* Kernel kinds reported by ohm_map_kernel_times. */
enum {
  OHM_KERNEL_PREPASS = 0,   /* region pass: allocation and touched list */
  OHM_KERNEL_WALK = 1,      /* per-ray voxel walk with its updates */
  OHM_KERNEL_FINALIZE = 2,  /* per-scan clamp / accumulator clear */
  OHM_KERNEL_NDT_HIT = 3,   /* NDT sample fold (phase 2) */
  OHM_KERNEL_WALK_GROUP = 4,      /* voxel walk over a group of scans (OHM_LAYER_SCAN_GROUPS) */
  OHM_KERNEL_FINALIZE_GROUP = 5,  /* in-order apply of a group's scans */
  OHM_KERNEL_NDT_SAMPLES = 6,     /* NDT hit samples into the per-scan moments */
  OHM_KERNEL_OTHER = 7,
  OHM_KERNEL_KINDS = 8
};

/* Profiling.  While enabled, each kernel the map launches is bracketed by a
 * pair of HIP events recorded on the launch stream.  ohm_map_kernel_times
 * waits for the recorded events, writes per kernel kind the number of
 * launches (h_launches[OHM_KERNEL_KINDS]) and their summed duration in
 * milliseconds (h_ms[OHM_KERNEL_KINDS]), and clears the record. */
ohm_status ohm_map_set_profiling(ohm_map map, int enable);
ohm_status ohm_map_kernel_times(ohm_map map, uint32_t* h_launches, double* h_ms);

/* Measurement helper (not part of integration): times 2^27 independent
 * atomic updates into the caller's device buffer d_buffer (bytes long, at
 * least one word; contents are overwritten), at pseudo-random word addresses
 * or, with OHM_PROBE_SEQUENTIAL in flags, at consecutive addresses across
 * each wave.  The update is an f32 atomic add of 1.0f (default), an f32
 * clamp-add by compare-and-swap retried until it lands (OHM_PROBE_F32_CAS;
 * the per-update walk's operation) or a u64 atomic add (OHM_PROBE_U64_ADD).
 * Writes the rate in operations per second to *h_ops_per_s; synchronises
 * `stream`.  These are the ceilings that the walks' per-voxel atomic
 * updates are compared with at the footprint of the layer they update. */
enum { OHM_PROBE_SEQUENTIAL = 1, OHM_PROBE_F32_CAS = 2, OHM_PROBE_U64_ADD = 4, OHM_PROBE_READ_ONLY = 8 };
ohm_status ohm_probe_atomic_rate(void* d_buffer, size_t bytes, int flags, double* h_ops_per_s, void* stream);

/* Measurement helper (not part of integration): the device's streaming
 * bandwidth at a footprint.  Times a copy of `bytes` from d_src to d_dst
 * (both device buffers of at least `bytes`, 16-byte aligned; d_dst is
 * overwritten) or, with OHM_PROBE_READ_ONLY in flags, a read of d_src alone
 * (d_dst then receives at most a few 16-byte words).  bytes must be a
 * multiple of 16 and at least 16 MiB; flags other than OHM_PROBE_READ_ONLY
 * are rejected (OHM_E_INVALID_ARG).  Writes the bytes moved per second
 * (read plus written) to *h_bytes_per_s; synchronises `stream`.  The HBM
 * rooflines of the walks quote the published peak with this measured rate
 * beside it. */
ohm_status ohm_probe_stream_rate(const void* d_src, void* d_dst, size_t bytes, int flags, double* h_bytes_per_s,
                                 void* stream);

/* Synchronise `stream` and read the map's statistics. */
ohm_status ohm_map_sync_status(ohm_map map, void* stream, ohm_map_stats* out);

const char* ohm_status_string(ohm_status status);

/* Build identification: the sha256 (64 hex digits) of the kernel sources,
 * their headers and this header that the library was compiled from, so that
 * a caller can refuse a library built from other sources. */
const char* ohm_build_source_digest(void);

#ifdef __cplusplus
}
#endif

#endif /* OHM_H */
