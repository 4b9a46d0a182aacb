"""Synthetic lidar workloads with the shapes of the paper's evaluation.

The paper evaluates on recorded VLP-16 data sets (Section IV, Table III) that
are not available here; these seeded generators stand in for them:

* ``config0`` -- 32,768 rays from the centre of a 20 m cube of 0.1 m voxels,
  directions uniform on the sphere, ranges U[1, 15] m (seed 0).
* ``config1`` -- a 64-beam x 2048-column spinning lidar (elevation -22.5 to
  +22.5 deg) driven 100 x 0.1 m along a 4 x 3 m box tunnel holding 200 random
  axis-aligned boxes (0.2-1 m sides), range noise N(0, 0.02 m), no-return rays
  emitted at 50 m, 0.1 m voxels over a 200 x 200 x 40 m map, 30 m max range.
* ``config2`` -- the config-1 scans with NDT-OM parameters (sensor noise 0.05 m).
* ``config3`` -- 16 sensor streams, 1,000 scans of log-uniform size in
  [8,192, 262,144] rays, streams 0-7 into a 0.1 m map and 8-15 into a 0.05 m map.
* ``config4`` -- the first 20 config-1 scans on 0.2 m voxels with per-ray
  weights U[0.5, 1] and an occupied/free label grid rasterised from the scene.

Everything is plain numpy (float64 geometry, float32 outputs) and fully
determined by the seeds, so the same arrays are produced on any host.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import List, Optional

import numpy as np

# Map-parameter modes (mirrors the C-ABI enum values).
MODE_PER_UPDATE = 0
MODE_COUNT_CLAMP = 1

TUNNEL_Y = 2.0          # tunnel interior |y| < 2 m
TUNNEL_Z = 1.5          # tunnel interior |z| < 1.5 m
TUNNEL_X = (-45.0, 55.0)  # tunnel length along x; both ends open
NO_RETURN_RANGE = 50.0  # rays that hit nothing are emitted at this range


@dataclasses.dataclass
class MapParams:
    """Map frame and update parameters (field names match ``ohm_params``)."""

    voxel_size: float = 0.1
    map_origin: tuple = (0.0, 0.0, 0.0)
    key_min: tuple = (0, 0, 0)
    key_max: tuple = (1, 1, 1)
    fixed_bits: int = 16
    l_hit: float = 0.847
    l_miss: float = -0.405
    l_min: float = -2.0
    l_max: float = 3.5
    l_init: float = 0.0
    max_range: float = 0.0            # <= 0: unlimited
    mode: int = MODE_COUNT_CLAMP
    sensor_noise: float = 0.05        # NDT
    adaptation_rate: float = 1.0      # NDT
    ndt_min_samples: int = 4          # NDT
    ndt_clear_below: float = -math.inf  # NDT sample clearing threshold (disabled)
    ndt_tm_gate: float = 9.0          # NDT-TM: squared Mahalanobis distance of a checked miss (3 sigma)
    tsdf_truncation: float = 0.3      # TSDF: band half-width along the ray (metres)
    tsdf_max_weight: float = 10000.0  # TSDF: weight cap

    def replace(self, **kw) -> "MapParams":
        return dataclasses.replace(self, **kw)

    @property
    def dims(self):
        return tuple(int(b - a) for a, b in zip(self.key_min, self.key_max))


@dataclasses.dataclass
class RayBatch:
    """Rays grouped into scans: scan ``s`` owns rays ``offsets[s]:offsets[s+1]``
    and shares the sensor position ``origins[s]``."""

    origins: np.ndarray   # float32 [S, 3]
    samples: np.ndarray   # float32 [N, 3]
    offsets: np.ndarray   # uint32  [S + 1]
    weights: Optional[np.ndarray] = None  # float32 [N] or None

    @property
    def n_scans(self) -> int:
        return int(self.origins.shape[0])

    @property
    def n_rays(self) -> int:
        return int(self.samples.shape[0])

    def scans(self, first: int, count: int) -> "RayBatch":
        """The contiguous sub-batch of ``count`` scans starting at ``first``."""
        lo, hi = int(self.offsets[first]), int(self.offsets[first + count])
        w = None if self.weights is None else self.weights[lo:hi].copy()
        return RayBatch(self.origins[first:first + count].copy(),
                        self.samples[lo:hi].copy(),
                        (self.offsets[first:first + count + 1] - lo).astype(np.uint32),
                        w)


def grid_map(lo, hi, voxel_size, **kw) -> MapParams:
    """A map whose key (0,0,0) min corner is at ``lo`` spanning up to ``hi``."""
    lo = tuple(float(v) for v in lo)
    dims = tuple(int(round((h - l) / voxel_size)) for l, h in zip(lo, hi))
    return MapParams(voxel_size=float(voxel_size), map_origin=lo,
                     key_min=(0, 0, 0), key_max=dims, **kw)


# --------------------------------------------------------------------------
# config 0: uniform rays from the cube centre
# --------------------------------------------------------------------------

def config0(n_rays: int = 32768, seed: int = 0, mode: int = MODE_COUNT_CLAMP):
    params = grid_map((-10.0, -10.0, -10.0), (10.0, 10.0, 10.0), 0.1, mode=mode)
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n_rays, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.uniform(1.0, 15.0, size=n_rays)
    samples = (d * r[:, None]).astype(np.float32)
    batch = RayBatch(np.zeros((1, 3), np.float32), samples,
                     np.array([0, n_rays], np.uint32))
    return params, batch


def random_rays(n_rays: int, seed: int, lo, hi, origin, r_lo=0.0, r_hi=1.0):
    """Small randomised ray sets for parity tests: one origin, uniform
    directions, ranges U[r_lo, r_hi] (world units)."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n_rays, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.uniform(r_lo, r_hi, size=n_rays)
    o = np.asarray(origin, np.float64)
    samples = (o[None, :] + d * r[:, None]).astype(np.float32)
    return RayBatch(np.asarray(origin, np.float32).reshape(1, 3), samples,
                    np.array([0, n_rays], np.uint32))


# --------------------------------------------------------------------------
# config 1 scene: box tunnel with random boxes
# --------------------------------------------------------------------------

@functools.lru_cache(maxsize=8)
def _tunnel_scene_cached(n_boxes, seed, path_len, clearance):
    return _make_tunnel_scene(n_boxes, seed, path_len, clearance)


def tunnel_scene(n_boxes: int = 200, seed: int = 1, path_len: float = 9.9, clearance: float = 0.5):
    """Axis-aligned boxes ``[n, 2, 3]`` (min, max): see _make_tunnel_scene."""
    return _tunnel_scene_cached(n_boxes, seed, path_len, clearance).copy()


def _make_tunnel_scene(n_boxes, seed, path_len, clearance):
    """Axis-aligned boxes ``[n, 2, 3]`` (min, max) with centres uniform in the
    tunnel, sides U[0.2, 1] m, none within ``clearance`` of the sensor path
    (the x axis from 0 to ``path_len``)."""
    rng = np.random.default_rng(seed)
    boxes = []
    while len(boxes) < n_boxes:
        c = np.array([rng.uniform(*TUNNEL_X), rng.uniform(-TUNNEL_Y, TUNNEL_Y),
                      rng.uniform(-TUNNEL_Z, TUNNEL_Z)])
        half = rng.uniform(0.2, 1.0, size=3) / 2.0
        bmin, bmax = c - half, c + half
        dx = max(0.0, bmin[0] - path_len, 0.0 - bmax[0])
        dy = max(0.0, bmin[1], -bmax[1])
        dz = max(0.0, bmin[2], -bmax[2])
        if math.sqrt(dx * dx + dy * dy + dz * dz) < clearance:
            continue
        boxes.append(np.stack([bmin, bmax]))
    return np.asarray(boxes, np.float64)


def _first_hit(pos: np.ndarray, dirs: np.ndarray, boxes: np.ndarray) -> np.ndarray:
    """Distance along unit ``dirs`` from ``pos`` to the first tunnel wall or box
    surface (inf when the ray leaves through an open tunnel end)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dirs
        # tunnel side walls (the sensor is inside the tube)
        ty = np.where(dirs[:, 1] > 0, (TUNNEL_Y - pos[1]) * inv[:, 1],
                      np.where(dirs[:, 1] < 0, (-TUNNEL_Y - pos[1]) * inv[:, 1], np.inf))
        tz = np.where(dirs[:, 2] > 0, (TUNNEL_Z - pos[2]) * inv[:, 2],
                      np.where(dirs[:, 2] < 0, (-TUNNEL_Z - pos[2]) * inv[:, 2], np.inf))
        t = np.minimum(ty, tz)
        xw = pos[0] + t * dirs[:, 0]
        t = np.where((xw >= TUNNEL_X[0]) & (xw <= TUNNEL_X[1]), t, np.inf)
        for bmin, bmax in boxes:
            # cull with the box's bounding sphere: only rays inside the cone it
            # subtends from the sensor can reach it
            c = 0.5 * (bmin + bmax)
            rho = 0.5 * float(np.linalg.norm(bmax - bmin))
            v = c - pos
            dist = float(np.linalg.norm(v))
            if dist - rho > 31.0 and np.all(np.isfinite(t)):
                continue
            if dist > rho:
                cos_a = math.sqrt(max(0.0, 1.0 - (rho / dist) ** 2)) - 1e-9
                idx = np.nonzero(dirs @ (v / dist) >= cos_a)[0]
            else:
                idx = np.arange(dirs.shape[0])
            if idx.size == 0:
                continue
            iv = inv[idx]
            t0 = (bmin[None, :] - pos[None, :]) * iv
            t1 = (bmax[None, :] - pos[None, :]) * iv
            tn = np.nanmax(np.minimum(t0, t1), axis=1)
            tf = np.nanmin(np.maximum(t0, t1), axis=1)
            hit = tf >= np.maximum(tn, 0.0)
            # a sensor inside a box sees the box's far walls
            th = np.where(tn >= 0.0, tn, tf)
            cur = t[idx]
            t[idx] = np.where(hit & (th < cur), th, cur)
    return t


def spinning_directions(beams: int = 64, cols: int = 2048,
                        elev_deg=(-22.5, 22.5)) -> np.ndarray:
    """Unit directions of one spinning-lidar revolution, column-major
    (ray = column * beams + beam), as a real sensor emits them."""
    e = np.deg2rad(elev_deg[0] + (elev_deg[1] - elev_deg[0]) * np.arange(beams) / (beams - 1))
    az = 2.0 * np.pi * np.arange(cols) / cols
    ce, se = np.cos(e), np.sin(e)
    d = np.empty((cols, beams, 3))
    d[:, :, 0] = np.cos(az)[:, None] * ce[None, :]
    d[:, :, 1] = np.sin(az)[:, None] * ce[None, :]
    d[:, :, 2] = se[None, :]
    return d.reshape(-1, 3)


def lidar_scan(pos, dirs, boxes, noise_seed, noise_sigma=0.02):
    pos = np.asarray(pos, np.float64)
    t = _first_hit(pos, dirs, boxes)
    rng = np.random.default_rng(noise_seed)
    noise = rng.normal(0.0, noise_sigma, size=t.shape[0])
    r = np.where(np.isfinite(t), t + noise, NO_RETURN_RANGE)
    return (pos[None, :] + dirs * r[:, None]).astype(np.float32)


def config1_params(voxel_size: float = 0.1, mode: int = MODE_COUNT_CLAMP) -> MapParams:
    return grid_map((-100.0, -100.0, -20.0), (100.0, 100.0, 20.0), voxel_size,
                    max_range=30.0, mode=mode)


def config1(n_scans: int = 100, first_scan: int = 0, beams: int = 64, cols: int = 2048,
            voxel_size: float = 0.1, mode: int = MODE_COUNT_CLAMP):
    """Spinning-lidar scans along the tunnel.  Scan ``k`` sits at (0.1 k, 0, 0)
    and draws its range noise from seed (2, k)."""
    params = config1_params(voxel_size, mode)
    boxes = tunnel_scene()
    dirs = spinning_directions(beams, cols)
    n = dirs.shape[0]
    origins = np.zeros((n_scans, 3), np.float32)
    samples = np.empty((n_scans * n, 3), np.float32)
    for i in range(n_scans):
        k = first_scan + i
        pos = np.array([0.1 * k, 0.0, 0.0])
        origins[i] = pos
        samples[i * n:(i + 1) * n] = lidar_scan(pos, dirs, boxes, noise_seed=[2, k])
    offsets = (np.arange(n_scans + 1) * n).astype(np.uint32)
    return params, RayBatch(origins, samples, offsets)


def lidar_intensities(batch: RayBatch, seed: int = 7) -> np.ndarray:
    """Synthetic return intensities for the NDT-TM workload (the recorded data
    sets' intensities are not available): a smooth field over the sample
    positions, 100 +- 60, plus per-ray noise N(0, 5), seeded; float32 per ray."""
    rng = np.random.default_rng(seed)
    p = batch.samples.astype(np.float64)
    field = 100.0 + 60.0 * np.sin(0.7 * p[:, 0]) * np.cos(1.3 * p[:, 2])
    return (field + rng.normal(0.0, 5.0, size=p.shape[0])).astype(np.float32)


def config2(n_scans: int = 100, first_scan: int = 0, mode: int = MODE_COUNT_CLAMP, **kw):
    params, batch = config1(n_scans, first_scan, mode=mode, **kw)
    return params.replace(sensor_noise=0.05, adaptation_rate=1.0, ndt_min_samples=4), batch


# --------------------------------------------------------------------------
# config 3: many uneven scans from 16 sensor streams into two maps
# --------------------------------------------------------------------------

@dataclasses.dataclass
class StreamScan:
    stream: int
    index: int      # scan index within its stream
    map_id: int     # 0: 0.1 m map, 1: 0.05 m map
    n_rays: int


def config3_schedule(n_streams: int = 16, n_scans: int = 1000, seed: int = 3,
                     lo: int = 8192, hi: int = 262144) -> (List[StreamScan], np.ndarray):
    """Scan sizes (log-uniform) and per-stream mount offsets U[-0.5, 0.5]^3."""
    rng = np.random.default_rng(seed)
    mounts = rng.uniform(-0.5, 0.5, size=(n_streams, 3))
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_scans))).astype(np.int64)
    per_stream = [n_scans // n_streams + (1 if s < n_scans % n_streams else 0)
                  for s in range(n_streams)]
    scans, c = [], 0
    for s in range(n_streams):
        for j in range(per_stream[s]):
            scans.append(StreamScan(s, j, 0 if s < n_streams // 2 else 1, int(sizes[c])))
            c += 1
    return scans, mounts


def _config3_scan(args):
    stream, index, n, mount = args
    rng = np.random.default_rng(1000 * stream + index)
    az = rng.uniform(0.0, 2.0 * np.pi, size=n)
    el = np.deg2rad(rng.uniform(-22.5, 22.5, size=n))
    dirs = np.stack([np.cos(az) * np.cos(el), np.sin(az) * np.cos(el), np.sin(el)], 1)
    pos = np.array([0.1 * (index % 100), 0.0, 0.0]) + mount
    return pos.astype(np.float32), lidar_scan(pos, dirs, tunnel_scene(), noise_seed=[2, 1000 * stream + index])


def config3(n_streams: int = 16, n_scans: int = 1000, size_scale: float = 1.0, jobs: int = 1):
    """Returns the two maps' params and, per map, a RayBatch whose scans are in
    the per-map application order (scan index within stream, then stream id).
    ``size_scale`` < 1 shrinks every scan (for quick tests); ``jobs`` > 1
    generates scans in a process pool (every scan is seeded on its own, so
    the output does not depend on it)."""
    scans, mounts = config3_schedule(n_streams, n_scans)
    params = [config1_params(0.1), config1_params(0.05)]
    out = []
    for map_id in (0, 1):
        mine = sorted((s for s in scans if s.map_id == map_id), key=lambda s: (s.index, s.stream))
        work = [(sc.stream, sc.index, max(1, int(round(sc.n_rays * size_scale))), mounts[sc.stream]) for sc in mine]
        if jobs > 1:
            # fresh interpreters (spawn), ended with close/join rather than a
            # terminate: the workers never inherit a parent's GPU state
            import multiprocessing as mp
            pool = mp.get_context("spawn").Pool(jobs)
            try:
                res = pool.map(_config3_scan, work, chunksize=4)
                pool.close()
            except BaseException:
                pool.terminate()
                raise
            finally:
                pool.join()
        else:
            res = [_config3_scan(w) for w in work]
        offsets = np.zeros(len(res) + 1, np.int64)
        offsets[1:] = np.cumsum([r[1].shape[0] for r in res])
        out.append(RayBatch(np.asarray([r[0] for r in res], np.float32), np.concatenate([r[1] for r in res]),
                            offsets.astype(np.uint32)))
    return params, out


# --------------------------------------------------------------------------
# config 4: differentiation workload
# --------------------------------------------------------------------------

def label_grid(params: MapParams, box_min, box_dim, boxes=None) -> np.ndarray:
    """1 where the voxel centre is solid (outside the tunnel interior or inside
    a box), else 0; float32 ``[dz, dy, dx]``."""
    if boxes is None:
        boxes = tunnel_scene()
    s = params.voxel_size
    axes = [params.map_origin[a] + (box_min[a] + np.arange(box_dim[a]) + 0.5) * s for a in range(3)]
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    free = (np.abs(y) < TUNNEL_Y) & (np.abs(z) < TUNNEL_Z) & (x > TUNNEL_X[0]) & (x < TUNNEL_X[1])
    solid = ~free
    for bmin, bmax in boxes:
        solid |= ((x >= bmin[0]) & (x <= bmax[0]) & (y >= bmin[1]) & (y <= bmax[1])
                  & (z >= bmin[2]) & (z <= bmax[2]))
    return solid.astype(np.float32)


def config4(n_scans: int = 20, beams: int = 64, cols: int = 2048, weight_seed: int = 4):
    params, batch = config2(n_scans, voxel_size=0.2, beams=beams, cols=cols)
    rng = np.random.default_rng(weight_seed)
    batch.weights = rng.uniform(0.5, 1.0, size=batch.n_rays).astype(np.float32)
    # 64^3 loss box (12.8 m cube) centred on the sensor path
    box_min = (493, 468, 68)
    box_dim = (64, 64, 64)
    labels = label_grid(params, box_min, box_dim)
    return params, batch, box_min, box_dim, labels
