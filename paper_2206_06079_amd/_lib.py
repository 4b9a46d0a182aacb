"""ctypes declarations of the C ABI in include/ohm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libohm_hip.so")

OHM_OK = 0
OHM_E_INVALID_ARG = -1
OHM_E_NO_DEVICE = -2
OHM_E_HIP = -3
OHM_E_WORKSPACE_TOO_SMALL = -4
OHM_E_UNSUPPORTED = -5

MODE_PER_UPDATE = 0
MODE_COUNT_CLAMP = 1

LAYER_OCC = 1
LAYER_NDT = 2
LAYER_ADJOINT = 4
LAYER_SCAN_GROUPS = 8
LAYER_MEAN = 16
LAYER_DECAY = 32
LAYER_NDT_TM = 64
LAYER_TSDF = 128


def scan_group_slots(n: int) -> int:
    """Layer-mask bits asking for n accumulator slots (OHM_SCAN_GROUP_SLOTS)."""
    return (int(n) & 0xFF) << 8


READ_OCC = 0
READ_HITS = 1
READ_MISSES = 2
READ_NDT_COUNT = 3
READ_NDT_MEAN = 4
READ_NDT_COV = 5
READ_CLAMP_SCAN = 6
READ_MEAN_PACKED = 7
READ_MEAN_COUNT = 8
READ_MEAN = 9
READ_DECAY_LENGTH = 10
READ_DECAY_HITS = 11
READ_DECAY_RATE = 12
READ_TM_MISSES = 13
READ_TM_PERMEABILITY = 14
READ_INTENSITY_MEAN = 15
READ_INTENSITY_VAR = 16
READ_TSDF_DISTANCE = 17
READ_TSDF_WEIGHT = 18
PROBE_SEQUENTIAL, PROBE_F32_CAS, PROBE_U64_ADD, PROBE_READ_ONLY = 1, 2, 4, 8

# Every symbol include/ohm.h declares.
EXPORTS = (
    "ohm_map_workspace_size", "ohm_map_create", "ohm_map_destroy", "ohm_map_reset",
    "ohm_map_set_params", "ohm_integrate_rays", "ohm_ndt_integrate", "ohm_map_read_dense",
    "ohm_debug_trace_rays", "ohm_map_sync_status", "ohm_status_string",
    "ohm_map_set_profiling", "ohm_map_kernel_times", "ohm_backward",
    "ohm_batch_workspace_size", "ohm_batch_create", "ohm_batch_run", "ohm_batch_destroy",
    "ohm_map_set_tuning", "ohm_probe_atomic_rate", "ohm_probe_stream_rate", "ohm_ray_order_scratch_size",
    "ohm_map_set_ray_order", "ohm_map_set_scan_layout",
    "ohm_build_source_digest", "ohm_ndt_tm_integrate", "ohm_tsdf_integrate", "ohm_integrate_rays_no_alloc",
)

NO_ALLOC_MAX_RAYS = 262144


class WalkTuning(ctypes.Structure):
    _fields_ = [("seg_major_steps", ctypes.c_uint32), ("tile_threads", ctypes.c_uint32)]


class ScanSet(ctypes.Structure):
    _fields_ = [
        ("map", ctypes.c_void_p),
        ("d_origins", ctypes.c_void_p),
        ("d_samples", ctypes.c_void_p),
        ("d_weights", ctypes.c_void_p),
        ("h_scan_offsets", ctypes.c_void_p),
        ("n_scans", ctypes.c_uint32),
    ]


class BatchTuning(ctypes.Structure):
    _fields_ = [("group_scans", ctypes.c_uint32), ("seg_major_steps", ctypes.c_uint32),
                ("tile_threads", ctypes.c_uint32), ("keep_ray_order", ctypes.c_uint32)]

KERNEL_KINDS = 8
KERNEL_NAMES = {0: "prepass", 1: "walk", 2: "finalize", 3: "ndt_hit", 4: "walk_group", 5: "finalize_group",
                6: "ndt_samples", 7: "other"}


class OhmParams(ctypes.Structure):
    _fields_ = [
        ("voxel_size", ctypes.c_double),
        ("map_origin", ctypes.c_double * 3),
        ("key_min", ctypes.c_int32 * 3),
        ("key_max", ctypes.c_int32 * 3),
        ("region_log2", ctypes.c_int32),
        ("fixed_bits", ctypes.c_int32),
        ("l_hit", ctypes.c_float),
        ("l_miss", ctypes.c_float),
        ("l_min", ctypes.c_float),
        ("l_max", ctypes.c_float),
        ("l_init", ctypes.c_float),
        ("max_range", ctypes.c_double),
        ("mode", ctypes.c_int32),
        ("sensor_noise", ctypes.c_float),
        ("adaptation_rate", ctypes.c_float),
        ("ndt_min_samples", ctypes.c_uint32),
        ("ndt_clear_below", ctypes.c_float),
        ("ndt_tm_gate", ctypes.c_double),
        ("tsdf_truncation", ctypes.c_double),
        ("tsdf_max_weight", ctypes.c_double),
    ]


class OhmStats(ctypes.Structure):
    _fields_ = [
        ("rays_in", ctypes.c_uint64),
        ("rays_invalid", ctypes.c_uint64),
        ("rays_origin_oob", ctypes.c_uint64),
        ("rays_truncated", ctypes.c_uint64),
        ("rays_clipped", ctypes.c_uint64),
        ("rays_hit", ctypes.c_uint64),
        ("voxel_updates", ctypes.c_uint64),
        ("updates_dropped_pool", ctypes.c_uint64),
        ("regions_used", ctypes.c_uint32),
        ("region_capacity", ctypes.c_uint32),
        ("sticky_error", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_ if name != "reserved"}


_lib = None


class OhmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


def load() -> ctypes.CDLL:
    """Load the HIP library; raises when it has not been built (there is no
    fallback implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it with "
                           "`python -m paper_2206_06079_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.ohm_build_source_digest.argtypes = []
    lib.ohm_build_source_digest.restype = ctypes.c_char_p
    built = lib.ohm_build_source_digest().decode()
    from . import build as _build
    if os.path.isdir(_build.CSRC):
        want = _build.source_digest()
        if built != want:
            raise RuntimeError(f"HIP library {LIB_PATH} was built from other sources (digest {built[:12]}, "
                               f"sources {want[:12]}): rebuild it with `python -m paper_2206_06079_amd.build`")
    vp, P = ctypes.c_void_p, ctypes.POINTER
    st = ctypes.c_int
    sig = {
        "ohm_map_workspace_size": [P(OhmParams), ctypes.c_uint32, ctypes.c_uint32, P(ctypes.c_size_t)],
        "ohm_map_create": [P(OhmParams), ctypes.c_uint32, ctypes.c_uint32, vp, ctypes.c_size_t, vp, P(vp)],
        "ohm_map_destroy": [vp],
        "ohm_map_reset": [vp, vp],
        "ohm_map_set_params": [vp, P(OhmParams)],
        "ohm_integrate_rays": [vp, vp, vp, vp, ctypes.c_uint32, vp, vp],
        "ohm_integrate_rays_no_alloc": [vp, vp, vp, vp, ctypes.c_uint32, vp, vp],
        "ohm_ndt_integrate": [vp, vp, vp, vp, ctypes.c_uint32, vp, vp],
        "ohm_ndt_tm_integrate": [vp, vp, vp, vp, vp, ctypes.c_uint32, vp, vp],
        "ohm_tsdf_integrate": [vp, vp, vp, vp, ctypes.c_uint32, vp],
        "ohm_map_read_dense": [vp, ctypes.c_int32, vp, vp, vp, vp],
        "ohm_debug_trace_rays": [vp, vp, vp, vp, ctypes.c_uint32, vp, vp, vp, vp, vp],
        "ohm_map_sync_status": [vp, vp, P(OhmStats)],
        "ohm_map_set_profiling": [vp, ctypes.c_int],
        "ohm_backward": [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, ctypes.c_uint32, vp, vp, vp, vp],
        "ohm_batch_workspace_size": [vp, ctypes.c_uint32, vp, P(ctypes.c_size_t)],
        "ohm_batch_create": [vp, ctypes.c_uint32, vp, vp, ctypes.c_size_t, vp, P(vp)],
        "ohm_batch_run": [vp, vp],
        "ohm_map_set_tuning": [vp, vp],
        "ohm_batch_destroy": [vp],
        "ohm_map_kernel_times": [vp, vp, vp],
        "ohm_probe_atomic_rate": [vp, ctypes.c_size_t, ctypes.c_int, P(ctypes.c_double), vp],
        "ohm_probe_stream_rate": [vp, vp, ctypes.c_size_t, ctypes.c_int, P(ctypes.c_double), vp],
        "ohm_ray_order_scratch_size": [ctypes.c_uint32, P(ctypes.c_size_t)],
        "ohm_map_set_ray_order": [vp, vp, ctypes.c_size_t, ctypes.c_uint32],
        "ohm_map_set_scan_layout": [vp, ctypes.c_uint32],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = st
    lib.ohm_status_string.argtypes = [ctypes.c_int]
    lib.ohm_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load().ohm_status_string(status).decode()
    except Exception:  # pragma: no cover - library missing
        return "status %d" % status


def check(status: int, where: str) -> None:
    if status != OHM_OK:
        raise OhmError(status, where)


def make_params(mp) -> OhmParams:
    """Marshal any object with the ohm_params field names (for instance
    ``workloads.MapParams``) into the C struct."""
    p = OhmParams()
    p.voxel_size = float(mp.voxel_size)
    for a in range(3):
        p.map_origin[a] = float(mp.map_origin[a])
        p.key_min[a] = int(mp.key_min[a])
        p.key_max[a] = int(mp.key_max[a])
    p.region_log2 = int(getattr(mp, "region_log2", 5))
    p.fixed_bits = int(mp.fixed_bits)
    p.l_hit, p.l_miss = float(mp.l_hit), float(mp.l_miss)
    p.l_min, p.l_max, p.l_init = float(mp.l_min), float(mp.l_max), float(mp.l_init)
    p.max_range = float(mp.max_range)
    p.mode = int(mp.mode)
    p.sensor_noise = float(mp.sensor_noise)
    p.adaptation_rate = float(mp.adaptation_rate)
    p.ndt_min_samples = int(mp.ndt_min_samples)
    p.ndt_clear_below = float(mp.ndt_clear_below)
    p.ndt_tm_gate = float(getattr(mp, "ndt_tm_gate", 9.0))
    p.tsdf_truncation = float(getattr(mp, "tsdf_truncation", 0.3))
    p.tsdf_max_weight = float(getattr(mp, "tsdf_max_weight", 10000.0))
    return p
