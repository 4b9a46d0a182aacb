"""GPU check of the allocation-free entry point (ohm_integrate_rays_no_alloc),
called through the C ABI, against the entry point it varies:
ohm_integrate_rays on a map with direction-ordering scratch attached
(ohm_map_set_ray_order).  Count mode is exact, so occupancy, the last scan's
hit and miss counts and the statistics must be identical.  Two calls in a
row, the second with smaller scans, so the shared scratch must be reused
correctly; a scan above the size limit is rejected with nothing enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2206_06079_amd as ohm
from paper_2206_06079_amd import _lib
from gpu_helpers import device, full_box, to_dev
from workloads import scenes
from workloads.scenes import RayBatch

pytestmark = pytest.mark.gpu


def unordered_scans(sizes, seed):
    """Scans from slightly different origins with unordered directions."""
    rng = np.random.default_rng(seed)
    origins, samples = [], []
    for k, n in enumerate(sizes):
        o = np.array([0.013 + 0.1 * k, -0.021, 0.0305])
        b = scenes.random_rays(n, seed * 100 + k, None, None, o, 0.2, 3.0)
        origins.append(b.origins[0])
        samples.append(b.samples)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    return RayBatch(np.asarray(origins, np.float32), np.concatenate(samples), off)


def call_no_alloc(m, batch):
    o, s, off, w = to_dev(batch)
    st = _lib.load().ohm_integrate_rays_no_alloc(
        m.handle, ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(s.data_ptr()),
        off.ctypes.data_as(ctypes.c_void_p), batch.n_scans,
        ctypes.c_void_p(w.data_ptr()) if w is not None else None,
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st


def read_all(m, mp):
    bmin, bdim = full_box(mp)
    return (m.read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy(),
            m.read_dense(ohm.READ_HITS, bmin, bdim).cpu().numpy(),
            m.read_dense(ohm.READ_MISSES, bmin, bdim).cpu().numpy(), m.stats())


@pytest.mark.parametrize("weighted", [False, True])
def test_no_alloc_equals_ordered_integrate(weighted):
    mp = scenes.grid_map((-3.2, -3.2, -3.2), (3.2, 3.2, 3.2), 0.1, max_range=2.5)
    first = unordered_scans([200000, 60000, 262144], seed=1)
    second = unordered_scans([20000, 9000], seed=2)
    if weighted:
        for b, sd in ((first, 3), (second, 4)):
            b.weights = np.random.default_rng(sd).uniform(0.5, 1.0, b.n_rays).astype(np.float32)
    a = ohm.OhmMap(mp, 8, device=device())
    r = ohm.OhmMap(mp, 8, device=device())
    r.set_ray_order(_lib.NO_ALLOC_MAX_RAYS)
    for batch in (first, second):
        assert call_no_alloc(a, batch) == _lib.OHM_OK
        o, s, off, w = to_dev(batch)
        r.integrate(o, s, off, w)
        got, ref = read_all(a, mp), read_all(r, mp)
        for x, y in zip(got[:3], ref[:3]):
            assert np.array_equal(x, y)
        assert got[3] == ref[3]
    assert got[3]["voxel_updates"] > 1_000_000
    a.close()
    r.close()


def test_no_alloc_rejects_oversized_scans():
    mp = scenes.grid_map((-3.2, -3.2, -3.2), (3.2, 3.2, 3.2), 0.1)
    m = ohm.OhmMap(mp, 8, device=device())
    big = unordered_scans([_lib.NO_ALLOC_MAX_RAYS + 1], seed=5)
    assert call_no_alloc(m, big) == _lib.OHM_E_INVALID_ARG
    st = m.stats()
    assert st["rays_in"] == 0  # nothing was enqueued
    m.close()
