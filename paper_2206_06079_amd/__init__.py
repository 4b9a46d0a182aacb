"""MI355X (gfx950) lidar ray integration into region-chunked 3D log-odds
occupancy maps: a HIP C-ABI library (include/ohm.h) with a thin torch binding.

Follows Stepanas et al., "OHM: GPU Based Occupancy Map Generation": exact
per-ray voxel walks (Sec. III-B) updating log-odds occupancy (Sec. II-B) and
NDT-OM statistics (Sec. II-D, III-C) in dense 32^3 regions (Sec. III-A), with
the voxel-mean, decay-rate (Sec. II-E), NDT-TM (Sec. II-D) and TSDF (Sec. II-F)
layers.
"""
from . import _lib  # noqa: F401
from ._lib import (  # noqa: F401
    LAYER_ADJOINT, LAYER_DECAY, LAYER_MEAN, LAYER_NDT, LAYER_NDT_TM, LAYER_OCC, LAYER_SCAN_GROUPS, LAYER_TSDF,
    MODE_COUNT_CLAMP, READ_INTENSITY_MEAN, READ_INTENSITY_VAR, READ_TM_MISSES, READ_TM_PERMEABILITY,
    READ_TSDF_DISTANCE, READ_TSDF_WEIGHT,
    MODE_PER_UPDATE, READ_CLAMP_SCAN, READ_DECAY_HITS, READ_DECAY_LENGTH, READ_DECAY_RATE, READ_HITS, READ_MEAN,
    READ_MEAN_COUNT, READ_MEAN_PACKED, READ_MISSES, READ_NDT_COUNT, READ_NDT_COV, READ_NDT_MEAN, READ_OCC,
    OHM_E_HIP, OHM_E_INVALID_ARG, OHM_E_NO_DEVICE, OHM_E_UNSUPPORTED, OHM_E_WORKSPACE_TOO_SMALL, OHM_OK,
    OhmError, scan_group_slots,
)
from .ohm import OhmIntegrate, OhmMap, probe_atomic_rate, probe_stream_rate, regions_needed  # noqa: F401
from .batch import OhmBatch, ScanSetArgs, autotune  # noqa: F401
