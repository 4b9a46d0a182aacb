"""Batched multi-sensor integration (ohm_batch_*) and its autotuner.

A plan integrates, per map, that map's scans in order -- the same result as
calling ``OhmMap.integrate`` scan by scan -- with the scans of all maps cut
into groups of G per map, each group one walk launch, and the whole sequence
captured as one graph.  ``autotune`` picks G and the walk tile by timing
candidate plans on throwaway maps with the same parameters, and caches the
choice."""
from __future__ import annotations

import ctypes
import json
import os
import time
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check, load
from .ohm import OhmMap, _dev_ptr, _host_offsets, _stream_ptr

DEFAULT_CANDIDATES = (1, 2, 4, 8, 16)
DEFAULT_TILES = ((32, 512), (16, 512), (32, 1024))  # (segment major steps, threads per tile)


class ScanSetArgs:
    """One map and its scans (device tensors, host offsets)."""

    def __init__(self, m: OhmMap, origins: torch.Tensor, samples: torch.Tensor, offsets, weights=None):
        self.map = m
        self.origins = origins.contiguous()
        self.samples = samples.contiguous()
        self.weights = None if weights is None else weights.contiguous()
        self.offsets = _host_offsets(offsets)
        n_scans = self.offsets.shape[0] - 1
        if n_scans < 0 or np.any(np.diff(self.offsets.astype(np.int64)) < 0):
            raise ValueError("offsets must be non-decreasing with at least one entry")
        if self.origins.dim() != 2 or self.origins.shape[1] != 3 or self.origins.shape[0] < n_scans:
            raise ValueError("origins must be [n_scans, 3]")
        if self.samples.dim() != 2 or self.samples.shape[1] != 3 or self.samples.shape[0] < int(self.offsets[-1]):
            raise ValueError("samples must be [N, 3] with N >= offsets[-1]")
        if self.weights is not None and self.weights.shape[0] < int(self.offsets[-1]):
            raise ValueError("weights must have one entry per ray")

    @property
    def n_scans(self):
        return int(self.offsets.shape[0] - 1)

    def struct(self) -> _lib.ScanSet:
        d = self.map.device
        s = _lib.ScanSet()
        s.map = self.map.handle
        s.d_origins = _dev_ptr(self.origins, torch.float32, "origins", d)
        s.d_samples = _dev_ptr(self.samples, torch.float32, "samples", d)
        s.d_weights = _dev_ptr(self.weights, torch.float32, "weights", d)
        s.h_scan_offsets = self.offsets.ctypes.data_as(ctypes.c_void_p)
        s.n_scans = self.n_scans
        return s


class OhmBatch:
    """A captured batched-integration plan over several maps.

    ``group_scans`` scans per map share one walk launch; ``seg_major_steps``
    and ``tile_threads`` set the walk's segment length and threads per
    256-ray tile (0 keeps the library defaults); ``keep_ray_order`` walks
    each scan's rays in the given order instead of direction order.  None of
    them changes the result."""

    def __init__(self, sets: Sequence[ScanSetArgs], group_scans: int, stream=None, seg_major_steps: int = 0,
                 tile_threads: int = 0, keep_ray_order: int = 0):
        lib = load()
        self.sets = list(sets)
        arr = (_lib.ScanSet * len(self.sets))(*[s.struct() for s in self.sets])
        self._arr = arr
        tun = _lib.BatchTuning(int(group_scans), int(seg_major_steps), int(tile_threads), int(keep_ray_order))
        size = ctypes.c_size_t(0)
        check(lib.ohm_batch_workspace_size(arr, len(self.sets), ctypes.byref(tun), ctypes.byref(size)),
              "ohm_batch_workspace_size")
        dev = self.sets[0].map.device
        self.workspace = torch.empty(int(size.value), dtype=torch.uint8, device=dev)
        h = ctypes.c_void_p()
        check(lib.ohm_batch_create(arr, len(self.sets), ctypes.byref(tun), ctypes.c_void_p(self.workspace.data_ptr()),
                                   int(size.value), _stream_ptr(stream), ctypes.byref(h)), "ohm_batch_create")
        self._handle = h
        self.group_scans = int(group_scans)
        self.seg_major_steps = int(seg_major_steps)
        self.tile_threads = int(tile_threads)
        self.keep_ray_order = int(keep_ray_order)

    def run(self, stream=None):
        check(load().ohm_batch_run(self._handle, _stream_ptr(stream)), "ohm_batch_run")

    def close(self):
        if getattr(self, "_handle", None):
            load().ohm_batch_destroy(self._handle)
            self._handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def _signature(sets: Sequence[ScanSetArgs]) -> str:
    dev = torch.cuda.get_device_name(sets[0].map.device)
    parts = []
    for s in sets:
        n = np.diff(s.offsets.astype(np.int64))
        parts.append("%.4g:%d:%d" % (s.map.params.voxel_size, s.n_scans, int(np.log2(max(1, n.mean())) * 4)))
    return dev + "|" + "|".join(parts) + "|w%d" % int(sets[0].weights is not None)


def autotune(sets: Sequence[ScanSetArgs], groups=DEFAULT_CANDIDATES, tiles=DEFAULT_TILES, orders=(0,),
             cache_path: Optional[str] = None, reps: int = 2, log=None) -> dict:
    """Pick the schedule -- group size G, walk tile (segment length K,
    threads per tile) and ray order (0: direction order, 1: as given) -- with
    the shortest plan run, timing every combination on fresh maps with the
    sets' parameters and capacities (the caller's maps are not touched).
    Returns the keyword arguments of ``OhmBatch``.  With ``cache_path`` the
    choice is read from / written to a JSON cache keyed by device and
    workload signature."""
    key = _signature(sets)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            c = cache[key]
            return {"group_scans": int(c["group_scans"]), "seg_major_steps": int(c["seg_major_steps"]),
                    "tile_threads": int(c["tile_threads"]), "keep_ray_order": int(c.get("keep_ray_order", 0))}
    timings = {}
    for g in groups:
        for k, t in tiles:
            for o in orders:
                maps = [OhmMap(s.map.params, s.map.capacity, device=s.map.device) for s in sets]
                trial = [ScanSetArgs(m, s.origins, s.samples, s.offsets, s.weights) for m, s in zip(maps, sets)]
                plan = OhmBatch(trial, g, seg_major_steps=k, tile_threads=t, keep_ray_order=o)
                plan.run()
                torch.cuda.synchronize()
                best = float("inf")
                for _ in range(reps):
                    t0 = time.perf_counter()
                    plan.run()
                    torch.cuda.synchronize()
                    best = min(best, time.perf_counter() - t0)
                timings[(g, k, t, o)] = best
                plan.close()
                for m in maps:
                    m.close()
                if log:
                    log(f"autotune G={g} K={k} T={t} keep_order={o}: {best * 1e3:.2f} ms")
    g, k, t, o = min(timings, key=timings.get)
    choice = {"group_scans": int(g), "seg_major_steps": int(k), "tile_threads": int(t), "keep_ray_order": int(o)}
    if cache_path:
        cache[key] = dict(choice, ms={"%d/%d/%d/%d" % c: v * 1e3 for c, v in timings.items()})
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return choice
