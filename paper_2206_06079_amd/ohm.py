"""Python binding over the C ABI: torch supplies device memory and streams,
every step of the integration runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check, load, make_params


def _stream_ptr(stream: Optional[torch.cuda.Stream] = None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t: Optional[torch.Tensor], dtype, name: str, device) -> Optional[ctypes.c_void_p]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, map is on {device}")
    return ctypes.c_void_p(t.data_ptr())


def _host_offsets(offsets) -> np.ndarray:
    if isinstance(offsets, torch.Tensor):
        offsets = offsets.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(offsets, dtype=np.uint32))


class OhmMap:
    """A region-chunked occupancy map living in a torch-allocated workspace."""

    def __init__(self, params, region_capacity: int, layers: int = _lib.LAYER_OCC,
                 device: Optional[torch.device] = None, stream: Optional[torch.cuda.Stream] = None):
        lib = load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.params = params
        self.layers = layers | _lib.LAYER_OCC
        self.capacity = int(region_capacity)
        self._cparams = make_params(params)
        size = ctypes.c_size_t(0)
        check(lib.ohm_map_workspace_size(ctypes.byref(self._cparams), self.capacity, self.layers,
                                         ctypes.byref(size)), "ohm_map_workspace_size")
        self.workspace_bytes = int(size.value)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        handle = ctypes.c_void_p()
        check(lib.ohm_map_create(ctypes.byref(self._cparams), self.capacity, self.layers,
                                 ctypes.c_void_p(self.workspace.data_ptr()), self.workspace_bytes,
                                 _stream_ptr(stream), ctypes.byref(handle)), "ohm_map_create")
        self._handle = handle

    # -- lifetime -----------------------------------------------------------------
    def close(self):
        if getattr(self, "_handle", None):
            load().ohm_map_destroy(self._handle)
            self._handle = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._handle:
            raise RuntimeError("map is closed")
        return self._handle

    def reset(self, stream=None):
        check(load().ohm_map_reset(self.handle, _stream_ptr(stream)), "ohm_map_reset")

    def set_params(self, params):
        cp = make_params(params)
        check(load().ohm_map_set_params(self.handle, ctypes.byref(cp)), "ohm_map_set_params")
        self.params, self._cparams = params, cp

    # -- integration ----------------------------------------------------------------
    def _scan_args(self, origins, samples, offsets, weights):
        h_off = _host_offsets(offsets)
        n_scans = h_off.shape[0] - 1
        if n_scans < 0:
            raise ValueError("offsets needs at least one entry")
        if origins.dim() != 2 or origins.shape[1] != 3 or origins.shape[0] < n_scans:
            raise ValueError("origins must be [n_scans, 3]")
        if samples.dim() != 2 or samples.shape[1] != 3 or samples.shape[0] < int(h_off[-1]):
            raise ValueError("samples must be [N, 3] with N >= offsets[-1]")
        if weights is not None and weights.shape[0] < int(h_off[-1]):
            raise ValueError("weights must have one entry per ray")
        return (_dev_ptr(origins, torch.float32, "origins", self.device),
                _dev_ptr(samples, torch.float32, "samples", self.device),
                h_off, n_scans, _dev_ptr(weights, torch.float32, "weights", self.device))

    def integrate(self, origins: torch.Tensor, samples: torch.Tensor, offsets, weights=None, stream=None):
        """Occupancy integration of scans (ohm_integrate_rays)."""
        o, s, h_off, n_scans, w = self._scan_args(origins, samples, offsets, weights)
        check(load().ohm_integrate_rays(self.handle, o, s, h_off.ctypes.data_as(ctypes.c_void_p), n_scans, w,
                                        _stream_ptr(stream)), "ohm_integrate_rays")

    def integrate_no_alloc(self, origins: torch.Tensor, samples: torch.Tensor, offsets, weights=None, stream=None):
        """Occupancy integration in direction order with the library's own
        fixed scratch (ohm_integrate_rays_no_alloc)."""
        o, s, h_off, n_scans, w = self._scan_args(origins, samples, offsets, weights)
        check(load().ohm_integrate_rays_no_alloc(self.handle, o, s, h_off.ctypes.data_as(ctypes.c_void_p), n_scans,
                                                 w, _stream_ptr(stream)), "ohm_integrate_rays_no_alloc")

    def ndt_integrate(self, origins: torch.Tensor, samples: torch.Tensor, offsets, weights=None, stream=None):
        """NDT-OM integration of scans (ohm_ndt_integrate)."""
        o, s, h_off, n_scans, w = self._scan_args(origins, samples, offsets, weights)
        check(load().ohm_ndt_integrate(self.handle, o, s, h_off.ctypes.data_as(ctypes.c_void_p), n_scans, w,
                                       _stream_ptr(stream)), "ohm_ndt_integrate")

    def ndt_tm_integrate(self, origins: torch.Tensor, samples: torch.Tensor, intensities: torch.Tensor, offsets,
                         weights=None, stream=None):
        """NDT-TM integration of scans (ohm_ndt_tm_integrate): NDT-OM plus
        checked misses and the intensity Gaussian; one intensity per ray."""
        o, s, h_off, n_scans, w = self._scan_args(origins, samples, offsets, weights)
        if intensities.shape[0] < int(h_off[-1]):
            raise ValueError("intensities must have one entry per ray")
        i = _dev_ptr(intensities, torch.float32, "intensities", self.device)
        check(load().ohm_ndt_tm_integrate(self.handle, o, s, i, h_off.ctypes.data_as(ctypes.c_void_p), n_scans, w,
                                          _stream_ptr(stream)), "ohm_ndt_tm_integrate")

    def tsdf_integrate(self, origins: torch.Tensor, samples: torch.Tensor, offsets, stream=None):
        """TSDF integration of scans (ohm_tsdf_integrate)."""
        o, s, h_off, n_scans, _ = self._scan_args(origins, samples, offsets, None)
        check(load().ohm_tsdf_integrate(self.handle, o, s, h_off.ctypes.data_as(ctypes.c_void_p), n_scans,
                                        _stream_ptr(stream)), "ohm_tsdf_integrate")

    # -- read-back ------------------------------------------------------------------
    _READ_SHAPES = {
        _lib.READ_OCC: (torch.float32, ()), _lib.READ_HITS: (torch.float32, ()),
        _lib.READ_MISSES: (torch.float32, ()), _lib.READ_NDT_COUNT: (torch.int32, ()),
        _lib.READ_NDT_MEAN: (torch.float32, (3,)), _lib.READ_NDT_COV: (torch.float32, (6,)),
        _lib.READ_CLAMP_SCAN: (torch.int32, ()),
        _lib.READ_MEAN_PACKED: (torch.int32, ()), _lib.READ_MEAN_COUNT: (torch.int32, ()),
        _lib.READ_MEAN: (torch.float32, (3,)), _lib.READ_DECAY_LENGTH: (torch.float32, ()),
        _lib.READ_DECAY_HITS: (torch.int32, ()), _lib.READ_DECAY_RATE: (torch.float32, ()),
        _lib.READ_TM_MISSES: (torch.int32, ()), _lib.READ_TM_PERMEABILITY: (torch.float32, ()),
        _lib.READ_INTENSITY_MEAN: (torch.float32, ()), _lib.READ_INTENSITY_VAR: (torch.float32, ()),
        _lib.READ_TSDF_DISTANCE: (torch.float32, ()), _lib.READ_TSDF_WEIGHT: (torch.float32, ()),
    }

    def read_dense(self, what: int, box_min: Sequence[int], box_dim: Sequence[int], out=None, stream=None):
        dtype, tail = self._READ_SHAPES[what]
        shape = (int(box_dim[2]), int(box_dim[1]), int(box_dim[0])) + tail
        if out is None:
            out = torch.empty(shape, dtype=dtype, device=self.device)
        bmin = (ctypes.c_int32 * 3)(*[int(v) for v in box_min])
        bdim = (ctypes.c_int32 * 3)(*[int(v) for v in box_dim])
        check(load().ohm_map_read_dense(self.handle, what, bmin, bdim, _dev_ptr(out, dtype, "out", self.device),
                                        _stream_ptr(stream)), "ohm_map_read_dense")
        return out

    def occupancy(self, box_min=None, box_dim=None):
        if box_min is None:
            box_min = self.params.key_min
            box_dim = [b - a for a, b in zip(self.params.key_min, self.params.key_max)]
        return self.read_dense(_lib.READ_OCC, box_min, box_dim)

    def trace(self, origins: torch.Tensor, samples: torch.Tensor, offsets, stream=None):
        """Per-ray update lists from the library's walk: returns
        (counts int64[N], flags int32[N], offsets int64[N+1], updates int32[T,4])."""
        o, s, h_off, n_scans, _ = self._scan_args(origins, samples, offsets, None)
        n = int(h_off[-1])
        lib = load()
        counts = torch.zeros(n, dtype=torch.int32, device=self.device)
        flags = torch.zeros(n, dtype=torch.int32, device=self.device)
        hp = h_off.ctypes.data_as(ctypes.c_void_p)
        check(lib.ohm_debug_trace_rays(self.handle, o, s, hp, n_scans, ctypes.c_void_p(counts.data_ptr()),
                                       ctypes.c_void_p(flags.data_ptr()), None, None, _stream_ptr(stream)),
              "ohm_debug_trace_rays(count)")
        offs = torch.zeros(n + 1, dtype=torch.int64, device=self.device)
        offs[1:] = torch.cumsum(counts.to(torch.int64), 0)
        total = int(offs[-1].item())
        upd = torch.zeros((max(total, 1), 4), dtype=torch.int32, device=self.device)
        check(lib.ohm_debug_trace_rays(self.handle, o, s, hp, n_scans, None, None,
                                       ctypes.c_void_p(offs.data_ptr()), ctypes.c_void_p(upd.data_ptr()),
                                       _stream_ptr(stream)), "ohm_debug_trace_rays(write)")
        return counts.to(torch.int64), flags, offs, upd[:total]

    def backward(self, grad_box: torch.Tensor, box_min, box_dim, origins, samples, offsets, weights=None,
                 ndt: bool = True, grad_weights: Optional[torch.Tensor] = None, stream=None):
        """ohm_backward: returns (dL/dw float32 [N] or None, dL/d(l_hit, l_miss,
        sensor_noise) float64 [3])."""
        o, s, h_off, n_scans, w = self._scan_args(origins, samples, offsets, weights)
        if grad_box.shape != (int(box_dim[2]), int(box_dim[1]), int(box_dim[0])):
            raise ValueError("grad_box must be [dz, dy, dx]")
        gs = torch.zeros(3, dtype=torch.float64, device=self.device)
        bmin = (ctypes.c_int32 * 3)(*[int(v) for v in box_min])
        bdim = (ctypes.c_int32 * 3)(*[int(v) for v in box_dim])
        gw_ptr = _dev_ptr(grad_weights, torch.float32, "grad_weights", self.device)
        check(load().ohm_backward(self.handle, 1 if ndt else 0,
                                  _dev_ptr(grad_box.contiguous(), torch.float32, "grad_box", self.device),
                                  bmin, bdim, o, s, h_off.ctypes.data_as(ctypes.c_void_p), n_scans, w, gw_ptr,
                                  _dev_ptr(gs, torch.float64, "grad_scalars", self.device), _stream_ptr(stream)),
              "ohm_backward")
        return grad_weights, gs

    def set_tuning(self, seg_major_steps: int = 16, tile_threads: int = 512):
        t = _lib.WalkTuning(int(seg_major_steps), int(tile_threads))
        check(load().ohm_map_set_tuning(self.handle, ctypes.byref(t)), "ohm_map_set_tuning")

    def set_scan_layout(self, column_rays: int):
        """Declare the scans column-major range images of ``column_rays``
        rays per column (ohm_map_set_scan_layout): the grouped walk then
        takes 8-beam by 32-column patches as tiles; 0 restores the given
        order."""
        check(load().ohm_map_set_scan_layout(self.handle, int(column_rays)), "ohm_map_set_scan_layout")

    def set_ray_order(self, max_rays: int):
        """Walk every scan of at most ``max_rays`` rays in direction order
        (ohm_map_set_ray_order); 0 turns it off.  The scratch buffer is held
        by this object."""
        lib = load()
        if max_rays <= 0:
            check(lib.ohm_map_set_ray_order(self.handle, None, 0, 0), "ohm_map_set_ray_order")
            self._order_scratch = None
            return
        size = ctypes.c_size_t(0)
        check(lib.ohm_ray_order_scratch_size(int(max_rays), ctypes.byref(size)), "ohm_ray_order_scratch_size")
        buf = torch.empty(int(size.value), dtype=torch.uint8, device=self.device)
        check(lib.ohm_map_set_ray_order(self.handle, ctypes.c_void_p(buf.data_ptr()), int(size.value), int(max_rays)),
              "ohm_map_set_ray_order")
        self._order_scratch = buf

    def set_profiling(self, enable: bool):
        check(load().ohm_map_set_profiling(self.handle, 1 if enable else 0), "ohm_map_set_profiling")

    def kernel_times(self) -> dict:
        """{kind: (launches, total_ms)} of the kernels recorded since the last
        call while profiling was enabled (synchronises)."""
        launches = (ctypes.c_uint32 * _lib.KERNEL_KINDS)()
        ms = (ctypes.c_double * _lib.KERNEL_KINDS)()
        check(load().ohm_map_kernel_times(self.handle, launches, ms), "ohm_map_kernel_times")
        return {_lib.KERNEL_NAMES.get(k, str(k)): (int(launches[k]), float(ms[k]))
                for k in range(_lib.KERNEL_KINDS) if launches[k]}

    def stats(self, stream=None) -> dict:
        st = _lib.OhmStats()
        check(load().ohm_map_sync_status(self.handle, _stream_ptr(stream), ctypes.byref(st)), "ohm_map_sync_status")
        return st.as_dict()


_PROBE_OPS = {"f32_add": 0, "f32_cas": 2, "u64_add": 4}


def probe_atomic_rate(footprint_bytes: int, sequential: bool = False, op: str = "f32_add", device=None,
                      stream=None) -> float:
    """Independent atomic updates per second at the given footprint (see
    ohm_probe_atomic_rate): op is "f32_add", "f32_cas" (clamp-add by
    compare-and-swap) or "u64_add"."""
    dev = torch.device("cuda", 0) if device is None else torch.device(device)
    buf = torch.zeros(max(2, int(footprint_bytes) // 4), dtype=torch.float32, device=dev)
    rate = ctypes.c_double(0.0)
    flags = _PROBE_OPS[op] | (1 if sequential else 0)
    check(load().ohm_probe_atomic_rate(ctypes.c_void_p(buf.data_ptr()), buf.numel() * 4, flags,
                                       ctypes.byref(rate), _stream_ptr(stream)), "ohm_probe_atomic_rate")
    return float(rate.value)


def probe_stream_rate(footprint_bytes: int, read_only: bool = False, device=None, stream=None) -> float:
    """Streaming bandwidth in bytes per second (read plus written) of a copy
    of footprint_bytes between two device buffers, or of a read alone (see
    ohm_probe_stream_rate)."""
    dev = torch.device("cuda", 0) if device is None else torch.device(device)
    n = max(16 << 20, int(footprint_bytes)) // 16 * 16
    src = torch.zeros(n, dtype=torch.uint8, device=dev)
    dst = torch.empty(n, dtype=torch.uint8, device=dev)
    rate = ctypes.c_double(0.0)
    check(load().ohm_probe_stream_rate(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n,
                                       _lib.PROBE_READ_ONLY if read_only else 0, ctypes.byref(rate),
                                       _stream_ptr(stream)), "ohm_probe_stream_rate")
    return float(rate.value)


def regions_needed(params, margin: float = 1.25) -> int:
    """Upper bound on regions for a map whose whole extent may be touched
    (used for small maps where reserving every region is cheap)."""
    n = 1
    for a in range(3):
        lo = params.key_min[a] >> 5
        hi = (params.key_max[a] - 1) >> 5
        n *= hi - lo + 1
    return n


class OhmIntegrate(torch.autograd.Function):
    """Differentiable count-mode integration: maps (per-ray weights, l_hit,
    l_miss, sensor_noise) to the final log-odds over a dense box.  The forward
    integrates every scan into a fresh map; the backward runs the library's
    adjoint kernel (traversals recomputed, NDT statistics replayed)."""

    @staticmethod
    def forward(ctx, weights, l_hit, l_miss, sensor_noise, params, origins, samples, offsets, box_min, box_dim,
                ndt=True, capacity=1024):
        p = params.replace(l_hit=float(l_hit), l_miss=float(l_miss), sensor_noise=float(sensor_noise),
                           mode=_lib.MODE_COUNT_CLAMP)
        layers = _lib.LAYER_OCC | _lib.LAYER_ADJOINT | (_lib.LAYER_NDT if ndt else 0)
        m = OhmMap(p, capacity, layers=layers, device=samples.device)
        w = weights.detach().contiguous()
        if ndt:
            m.ndt_integrate(origins, samples, offsets, w)
        else:
            m.integrate(origins, samples, offsets, w)
        out = m.read_dense(_lib.READ_OCC, box_min, box_dim)
        ctx.map = m
        ctx.args = (origins, samples, offsets, w, tuple(box_min), tuple(box_dim), ndt)
        ctx.dtypes = (l_hit.dtype, l_miss.dtype, sensor_noise.dtype)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        origins, samples, offsets, w, box_min, box_dim, ndt = ctx.args
        m = ctx.map
        gw = torch.empty_like(w)
        gw, gs = m.backward(grad_out.float().contiguous(), box_min, box_dim, origins, samples, offsets, w, ndt=ndt,
                            grad_weights=gw)
        m.close()
        ctx.map = None
        d_hit, d_miss, d_sig = (gs[i].to(dt) for i, dt in enumerate(ctx.dtypes))
        return gw, d_hit, d_miss, d_sig, None, None, None, None, None, None, None, None
