"""CPU oracle for the OHM ray-integration path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, single-threaded reference implementations (C in
``ohm_oracle.c``, loaded with ctypes) of what the HIP library computes.  Only
``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package; the product path never does, and this package never
imports the product package.

Functions follow the paper (Stepanas et al., "OHM: GPU Based Occupancy Map
Generation"): Sec. II-B Eq. (2)-(3) and the clamping paragraph for the
log-odds update, Sec. III-B for the per-ray line walk with misses along the
ray and a hit at the sample, Sec. IV-A for max-range truncation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libohm_oracle.so")
_lib = None

# per-ray flag bits (orc_trace)
F_TRUNCATED = 1
F_CLIPPED = 2
F_HAS_HIT = 4
F_INVALID = 8
F_ORIGIN_OOB = 16

STATS_FIELDS = ("rays", "invalid", "origin_oob", "truncated", "clipped", "hits", "updates")


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("voxel_size", ctypes.c_double),
        ("map_origin", ctypes.c_double * 3),
        ("key_min", ctypes.c_int32 * 3),
        ("key_max", ctypes.c_int32 * 3),
        ("fixed_bits", ctypes.c_int32),
        ("l_hit", ctypes.c_float),
        ("l_miss", ctypes.c_float),
        ("l_min", ctypes.c_float),
        ("l_max", ctypes.c_float),
        ("l_init", ctypes.c_float),
        ("max_range", ctypes.c_double),
        ("sensor_noise", ctypes.c_double),
        ("adaptation_rate", ctypes.c_double),
        ("ndt_min_samples", ctypes.c_int32),
        ("ndt_clear_below", ctypes.c_double),
        ("ndt_tm_gate", ctypes.c_double),
        ("tsdf_truncation", ctypes.c_double),
        ("tsdf_max_weight", ctypes.c_double),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    from . import build as _b
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"oracle library {_LIB_PATH} is missing: build it with `python -m oracle.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_source_digest.argtypes = []
    lib.orc_source_digest.restype = ctypes.c_char_p
    if lib.orc_source_digest().decode() != _b.source_digest():
        raise RuntimeError(f"oracle library {_LIB_PATH} was built from another source: rebuild it with "
                           "`python -m oracle.build`")
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.orc_trace.restype = ctypes.c_int64
    lib.orc_trace.argtypes = [P(OrcParams), ctypes.c_int32, vp, vp, vp, vp, vp, vp]
    lib.orc_integrate_count.restype = ctypes.c_int
    lib.orc_integrate_count.argtypes = [P(OrcParams), ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.orc_integrate_envelope.restype = ctypes.c_int
    lib.orc_integrate_envelope.argtypes = [P(OrcParams), ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.orc_ndt_integrate.restype = ctypes.c_int
    lib.orc_ndt_integrate.argtypes = [P(OrcParams), ctypes.c_int32, ctypes.c_int32] + [vp] * 12
    lib.orc_adjoint.restype = ctypes.c_int
    lib.orc_adjoint.argtypes = [P(OrcParams), ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp,
                                ctypes.c_double, ctypes.c_int32, vp, vp, vp, vp, vp, vp]
    lib.orc_mean_integrate.restype = ctypes.c_int
    lib.orc_mean_integrate.argtypes = [P(OrcParams), ctypes.c_int32, ctypes.c_int32] + [vp] * 8
    lib.orc_decay_integrate.restype = ctypes.c_int
    lib.orc_decay_integrate.argtypes = [P(OrcParams), ctypes.c_int32] + [vp] * 8
    lib.orc_ndt_miss_delta.restype = ctypes.c_double
    lib.orc_ndt_miss_delta.argtypes = [P(OrcParams), vp, vp, vp, vp, ctypes.c_uint32]
    lib.orc_ndt_closest_q.restype = ctypes.c_double
    lib.orc_ndt_closest_q.argtypes = [P(OrcParams), vp, vp, vp, vp]
    lib.orc_tsdf_integrate.restype = ctypes.c_int
    lib.orc_tsdf_integrate.argtypes = [P(OrcParams), ctypes.c_int32, ctypes.c_int32] + [vp] * 8
    lib.orc_ndt_tm_integrate.restype = ctypes.c_int
    lib.orc_ndt_tm_integrate.argtypes = [P(OrcParams), ctypes.c_int32, ctypes.c_int32] + [vp] * 16
    _lib = lib
    return lib


def make_params(mp) -> OrcParams:
    """Build the oracle's parameter struct from a ``workloads.MapParams``."""
    p = OrcParams()
    p.voxel_size = float(mp.voxel_size)
    for a in range(3):
        p.map_origin[a] = float(mp.map_origin[a])
        p.key_min[a] = int(mp.key_min[a])
        p.key_max[a] = int(mp.key_max[a])
    p.fixed_bits = int(mp.fixed_bits)
    p.l_hit, p.l_miss = float(mp.l_hit), float(mp.l_miss)
    p.l_min, p.l_max, p.l_init = float(mp.l_min), float(mp.l_max), float(mp.l_init)
    p.max_range = float(mp.max_range)
    p.sensor_noise = float(mp.sensor_noise)
    p.adaptation_rate = float(mp.adaptation_rate)
    p.ndt_min_samples = int(mp.ndt_min_samples)
    p.ndt_clear_below = float(mp.ndt_clear_below)
    p.ndt_tm_gate = float(mp.ndt_tm_gate)
    p.tsdf_truncation = float(mp.tsdf_truncation)
    p.tsdf_max_weight = float(mp.tsdf_max_weight)
    return p


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _batch_arrays(batch):
    o = np.ascontiguousarray(batch.origins, np.float32)
    s = np.ascontiguousarray(batch.samples, np.float32)
    off = np.ascontiguousarray(batch.offsets, np.uint32)
    w = None if batch.weights is None else np.ascontiguousarray(batch.weights, np.float32)
    return o, s, off, w


def trace(mp, batch) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """Per-ray update lists.

    Returns ``(counts int64[N], flags int32[N], offsets int64[N+1],
    updates int32[total, 4])`` where each update row is (kx, ky, kz, kind),
    kind 0 = miss, 1 = hit, in walk order from the sensor."""
    lib = _load()
    p = make_params(mp)
    o, s, off, _ = _batch_arrays(batch)
    n = s.shape[0]
    counts = np.zeros(n, np.int64)
    flags = np.zeros(n, np.int32)
    total = lib.orc_trace(ctypes.byref(p), batch.n_scans, _ptr(off), _ptr(o), _ptr(s),
                          _ptr(counts), _ptr(flags), None)
    keys = np.zeros((max(total, 1), 4), np.int32)
    lib.orc_trace(ctypes.byref(p), batch.n_scans, _ptr(off), _ptr(o), _ptr(s), None, None, _ptr(keys))
    offs = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=offs[1:])
    return counts, flags, offs, keys[:total]


def integrate_count(mp, batch, box_min=None, box_dim=None, occ=None):
    """Count-then-clamp integration into a dense box window (default: the
    whole map).  Returns ``(occ [dz,dy,dx] float32, last_hit, last_miss,
    stats dict)``; ``last_*`` are the last scan's per-voxel hit and miss
    weights (counts without weights)."""
    lib = _load()
    p = make_params(mp)
    if box_min is None:
        box_min = tuple(mp.key_min)
        box_dim = tuple(b - a for a, b in zip(mp.key_min, mp.key_max))
    bmin = np.asarray(box_min, np.int32)
    bdim = np.asarray(box_dim, np.int32)
    shape = (int(bdim[2]), int(bdim[1]), int(bdim[0]))
    if occ is None:
        occ = np.full(shape, np.float32(mp.l_init), np.float32)
    else:
        occ = np.ascontiguousarray(occ, np.float32).copy()
    last_hit = np.zeros(shape, np.float32)
    last_miss = np.zeros(shape, np.float32)
    stats = np.zeros(len(STATS_FIELDS), np.uint64)
    o, s, off, w = _batch_arrays(batch)
    rc = lib.orc_integrate_count(ctypes.byref(p), batch.n_scans, _ptr(off), _ptr(o), _ptr(s), _ptr(w),
                                 _ptr(bmin), _ptr(bdim), _ptr(occ), _ptr(last_hit), _ptr(last_miss),
                                 _ptr(stats))
    if rc != 0:
        raise MemoryError("oracle box allocation failed")
    return occ, last_hit, last_miss, dict(zip(STATS_FIELDS, (int(v) for v in stats)))


def integrate_envelope(mp, batch, box_min=None, box_dim=None, lo=None, hi=None):
    """Per-update (any-order CAS) semantics: returns ``(lo, hi, n_updates,
    stats)``, the fp64 bracket of every reachable result per voxel and the
    number of updates each voxel received."""
    lib = _load()
    p = make_params(mp)
    if box_min is None:
        box_min = tuple(mp.key_min)
        box_dim = tuple(b - a for a, b in zip(mp.key_min, mp.key_max))
    bmin = np.asarray(box_min, np.int32)
    bdim = np.asarray(box_dim, np.int32)
    shape = (int(bdim[2]), int(bdim[1]), int(bdim[0]))
    lo = np.full(shape, float(np.float32(mp.l_init)), np.float64) if lo is None else lo.astype(np.float64).copy()
    hi = np.full(shape, float(np.float32(mp.l_init)), np.float64) if hi is None else hi.astype(np.float64).copy()
    nupd = np.zeros(shape, np.uint32)
    stats = np.zeros(len(STATS_FIELDS), np.uint64)
    o, s, off, w = _batch_arrays(batch)
    rc = lib.orc_integrate_envelope(ctypes.byref(p), batch.n_scans, _ptr(off), _ptr(o), _ptr(s), _ptr(w),
                                    _ptr(bmin), _ptr(bdim), _ptr(lo), _ptr(hi), _ptr(nupd), _ptr(stats))
    if rc != 0:
        raise MemoryError("oracle box allocation failed")
    return lo, hi, nupd, dict(zip(STATS_FIELDS, (int(v) for v in stats)))


class NdtState:
    """NDT-OM voxel statistics over a box window (fp64, voxel-centred)."""

    def __init__(self, shape):
        self.n = np.zeros(shape, np.uint32)
        self.mu = np.zeros(shape + (3,), np.float64)
        self.cov = np.zeros(shape + (6,), np.float64)


def ndt_miss_delta(mp, o, e, mu_w, cov6, n) -> float:
    """The NDT-weighted miss increment of one voxel (paper Sec. II-D)."""
    lib = _load()
    p = make_params(mp)
    a = [np.ascontiguousarray(np.asarray(x, np.float64)) for x in (o, e, mu_w, cov6)]
    return float(lib.orc_ndt_miss_delta(ctypes.byref(p), *[_ptr(x) for x in a], int(n)))


def ndt_integrate(mp, batch, box_min=None, box_dim=None, occ=None, state=None, mode=1):
    """NDT-OM integration (paper Sec. II-D, III-C) into a box window.
    Returns ``(occ, state, last_miss_sum, stats)``."""
    lib = _load()
    p = make_params(mp)
    if box_min is None:
        box_min = tuple(mp.key_min)
        box_dim = tuple(b - a for a, b in zip(mp.key_min, mp.key_max))
    bmin = np.asarray(box_min, np.int32)
    bdim = np.asarray(box_dim, np.int32)
    shape = (int(bdim[2]), int(bdim[1]), int(bdim[0]))
    occ = np.full(shape, np.float32(mp.l_init), np.float32) if occ is None else np.ascontiguousarray(occ, np.float32).copy()
    if state is None:
        state = NdtState(shape)
    miss = np.zeros(shape, np.float64)
    stats = np.zeros(len(STATS_FIELDS), np.uint64)
    o, s, off, w = _batch_arrays(batch)
    rc = lib.orc_ndt_integrate(ctypes.byref(p), int(mode), batch.n_scans, _ptr(off), _ptr(o), _ptr(s), _ptr(w),
                               _ptr(bmin), _ptr(bdim), _ptr(occ), _ptr(state.n), _ptr(state.mu),
                               _ptr(state.cov), _ptr(miss), _ptr(stats))
    if rc != 0:
        raise MemoryError("oracle box allocation failed")
    return occ, state, miss, dict(zip(STATS_FIELDS, (int(v) for v in stats)))


def ndt_closest_q(mp, o, e, mu_w, cov6) -> float:
    """Squared Mahalanobis distance of the ray's closest point to a voxel's
    Gaussian (the NDT-TM miss check, paper Sec. II-D)."""
    lib = _load()
    p = make_params(mp)
    a = [np.ascontiguousarray(np.asarray(x, np.float64)) for x in (o, e, mu_w, cov6)]
    return float(lib.orc_ndt_closest_q(ctypes.byref(p), *[_ptr(x) for x in a]))


class NdtTmState(NdtState):
    """NDT-TM voxel state over a box window: the NDT-OM statistics plus the
    checked miss count M (permeability n / (n + M)), the count of misses whose
    check sat within a relative 1e-9 of the gate, and the intensity mean and
    population variance."""

    def __init__(self, shape):
        super().__init__(shape)
        self.miss = np.zeros(shape, np.uint32)
        self.near = np.zeros(shape, np.uint32)
        self.in_mean = np.zeros(shape, np.float64)
        self.in_var = np.zeros(shape, np.float64)

    def permeability(self):
        tot = self.n.astype(np.float64) + self.miss
        return np.divide(self.n.astype(np.float64), tot, out=np.zeros_like(tot), where=tot > 0)


def ndt_tm_integrate(mp, batch, intensities, box_min=None, box_dim=None, occ=None, state=None, mode=1):
    """NDT-TM integration (paper Sec. II-D, III-C) into a box window: NDT-OM
    plus permeability counts and the intensity Gaussian.  ``intensities``:
    float32 per ray.  Returns ``(occ, state, stats)``."""
    lib = _load()
    p = make_params(mp)
    if box_min is None:
        box_min = tuple(mp.key_min)
        box_dim = tuple(b - a for a, b in zip(mp.key_min, mp.key_max))
    bmin = np.asarray(box_min, np.int32)
    bdim = np.asarray(box_dim, np.int32)
    shape = (int(bdim[2]), int(bdim[1]), int(bdim[0]))
    occ = np.full(shape, np.float32(mp.l_init), np.float32) if occ is None else np.ascontiguousarray(occ, np.float32).copy()
    if state is None:
        state = NdtTmState(shape)
    inten = np.ascontiguousarray(intensities, np.float32)
    if inten.shape[0] < batch.n_rays:
        raise ValueError("one intensity per ray")
    stats = np.zeros(len(STATS_FIELDS), np.uint64)
    o, s, off, w = _batch_arrays(batch)
    rc = lib.orc_ndt_tm_integrate(ctypes.byref(p), int(mode), batch.n_scans, _ptr(off), _ptr(o), _ptr(s),
                                  _ptr(inten), _ptr(w), _ptr(bmin), _ptr(bdim), _ptr(occ), _ptr(state.n),
                                  _ptr(state.mu), _ptr(state.cov), _ptr(state.miss), _ptr(state.near),
                                  _ptr(state.in_mean), _ptr(state.in_var), _ptr(stats))
    if rc != 0:
        raise MemoryError("oracle box allocation failed")
    return occ, state, dict(zip(STATS_FIELDS, (int(v) for v in stats)))


def adjoint(mp, batch, box_min, box_dim, labels, mask=None, ndt=True, grads=True, near_eps=1e-3):
    """fp64 differentiable forward over the loss box and, with ``grads``, the
    analytic gradients (paper's count-mode update, BCE loss on sigmoid(l)).
    Returns a dict with loss, occ, clamp_last, near, grad_w [N], grad_scalars
    (d/d l_hit, l_miss, sensor_noise)."""
    lib = _load()
    p = make_params(mp)
    bmin = np.asarray(box_min, np.int32)
    bdim = np.asarray(box_dim, np.int32)
    shape = (int(bdim[2]), int(bdim[1]), int(bdim[0]))
    y = np.ascontiguousarray(labels, np.float64).reshape(shape)
    m = np.ones(shape, np.float64) if mask is None else np.ascontiguousarray(mask, np.float64).reshape(shape)
    loss = ctypes.c_double(0.0)
    occ = np.zeros(shape, np.float64)
    cl = np.zeros(shape, np.uint32)
    near = np.zeros(shape, np.uint8)
    gw = np.zeros(batch.n_rays, np.float64) if grads else None
    gs = np.zeros(3, np.float64) if grads else None
    o, s, off, w = _batch_arrays(batch)
    rc = lib.orc_adjoint(ctypes.byref(p), 1 if ndt else 0, batch.n_scans, _ptr(off), _ptr(o), _ptr(s), _ptr(w),
                         _ptr(bmin), _ptr(bdim), _ptr(y), _ptr(m), float(near_eps), 1 if grads else 0,
                         ctypes.byref(loss), _ptr(occ), _ptr(cl), _ptr(near), _ptr(gw), _ptr(gs))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return dict(loss=loss.value, occ=occ, clamp_last=cl, near=near, grad_w=gw, grad_scalars=gs)


def mean_integrate(mp, batch, box_min=None, box_dim=None, packed=None, count=None, mode=1):
    """Voxel mean layer (paper Sec. III-A, 10-bit sub-voxel codes per axis in
    one word plus a sample count) over a box window.  mode 1 merges each
    scan's samples of a voxel at once, mode 0 one sample at a time in ray
    order.  Returns ``(packed uint32 [dz,dy,dx], count uint32 [dz,dy,dx])``."""
    lib = _load()
    p = make_params(mp)
    if box_min is None:
        box_min = tuple(mp.key_min)
        box_dim = tuple(b - a for a, b in zip(mp.key_min, mp.key_max))
    bmin = np.asarray(box_min, np.int32)
    bdim = np.asarray(box_dim, np.int32)
    shape = (int(bdim[2]), int(bdim[1]), int(bdim[0]))
    packed = np.zeros(shape, np.uint32) if packed is None else np.ascontiguousarray(packed, np.uint32).copy()
    count = np.zeros(shape, np.uint32) if count is None else np.ascontiguousarray(count, np.uint32).copy()
    o, s, off, w = _batch_arrays(batch)
    rc = lib.orc_mean_integrate(ctypes.byref(p), int(mode), batch.n_scans, _ptr(off), _ptr(o), _ptr(s), _ptr(w),
                                _ptr(bmin), _ptr(bdim), _ptr(packed), _ptr(count))
    if rc != 0:
        raise MemoryError("oracle box allocation failed")
    return packed, count


def unpack_mean(packed):
    """Per-axis 10-bit codes of packed mean words: int array [..., 3]."""
    packed = np.asarray(packed, np.uint32)
    return np.stack([(packed >> (10 * a)) & 1023 for a in range(3)], axis=-1).astype(np.int64)


def decay_integrate(mp, batch, box_min=None, box_dim=None, length=None, hits=None):
    """Decay-rate layer (paper Sec. II-E) over a box window: per voxel the
    summed distance rays travel through it (metres, fp64) and the samples
    that fell in it.  Returns ``(length [dz,dy,dx] float64, hits uint32)``;
    the rate is hits / length."""
    lib = _load()
    p = make_params(mp)
    if box_min is None:
        box_min = tuple(mp.key_min)
        box_dim = tuple(b - a for a, b in zip(mp.key_min, mp.key_max))
    bmin = np.asarray(box_min, np.int32)
    bdim = np.asarray(box_dim, np.int32)
    shape = (int(bdim[2]), int(bdim[1]), int(bdim[0]))
    length = np.zeros(shape, np.float64) if length is None else np.ascontiguousarray(length, np.float64).copy()
    hits = np.zeros(shape, np.uint32) if hits is None else np.ascontiguousarray(hits, np.uint32).copy()
    o, s, off, w = _batch_arrays(batch)
    rc = lib.orc_decay_integrate(ctypes.byref(p), batch.n_scans, _ptr(off), _ptr(o), _ptr(s), _ptr(w),
                                 _ptr(bmin), _ptr(bdim), _ptr(length), _ptr(hits))
    if rc != 0:
        raise MemoryError("oracle box allocation failed")
    return length, hits


def tsdf_integrate(mp, batch, box_min=None, box_dim=None, dist=None, weight=None, mode=1):
    """TSDF integration (paper Sec. II-F) into a box window: per voxel the
    weighted mean projective distance D and its weight W.  mode 1 = per-scan
    sums, 0 = per update in ray order.  Returns ``(dist, weight, stats)``."""
    lib = _load()
    p = make_params(mp)
    if box_min is None:
        box_min = tuple(mp.key_min)
        box_dim = tuple(b - a for a, b in zip(mp.key_min, mp.key_max))
    bmin = np.asarray(box_min, np.int32)
    bdim = np.asarray(box_dim, np.int32)
    shape = (int(bdim[2]), int(bdim[1]), int(bdim[0]))
    dist = np.zeros(shape, np.float32) if dist is None else np.ascontiguousarray(dist, np.float32).copy()
    weight = np.zeros(shape, np.float32) if weight is None else np.ascontiguousarray(weight, np.float32).copy()
    stats = np.zeros(len(STATS_FIELDS), np.uint64)
    o, s, off, _ = _batch_arrays(batch)
    rc = lib.orc_tsdf_integrate(ctypes.byref(p), int(mode), batch.n_scans, _ptr(off), _ptr(o), _ptr(s), _ptr(bmin),
                                _ptr(bdim), _ptr(dist), _ptr(weight), _ptr(stats))
    if rc != 0:
        raise MemoryError("oracle box allocation failed")
    return dist, weight, dict(zip(STATS_FIELDS, (int(v) for v in stats)))
