"""The per-ray weight contract in the oracle: a ray whose weight is negative
or not finite is skipped whole and counted as invalid, in every integrator
(count, envelope, NDT, adjoint); a zero weight is a valid ray."""
import numpy as np

import oracle
from workloads import scenes
from workloads.scenes import RayBatch

MP = scenes.grid_map((-1.6, -1.6, -1.6), (1.6, 1.6, 1.6), 0.1, max_range=1.2)


def _batches():
    b = scenes.random_rays(400, 31, None, None, (0.02, -0.01, 0.03), 0.2, 1.5)
    w = np.random.default_rng(5).uniform(0.5, 1.0, 400).astype(np.float32)
    bad = np.array([3, 77, 150, 299], np.int64)
    w[bad] = [-0.25, np.nan, np.inf, -np.inf]
    w[10] = 0.0
    keep = np.setdiff1d(np.arange(400), bad)
    full = RayBatch(b.origins, b.samples, b.offsets, w)
    kept = RayBatch(b.origins, b.samples[keep], np.array([0, keep.size], np.uint32), w[keep])
    return full, kept, bad.size


def test_count_skips_bad_weights():
    full, kept, nbad = _batches()
    occ_f, _, _, st_f = oracle.integrate_count(MP, full)
    occ_k, _, _, st_k = oracle.integrate_count(MP, kept)
    assert np.array_equal(occ_f, occ_k)
    assert st_f["invalid"] == nbad and st_f["rays"] == st_k["rays"] + nbad
    assert st_f["updates"] == st_k["updates"]


def test_envelope_skips_bad_weights():
    full, kept, _ = _batches()
    lo_f, hi_f, n_f, _ = oracle.integrate_envelope(MP, full)
    lo_k, hi_k, n_k, _ = oracle.integrate_envelope(MP, kept)
    assert np.array_equal(lo_f, lo_k) and np.array_equal(hi_f, hi_k) and np.array_equal(n_f, n_k)


def test_ndt_and_adjoint_skip_bad_weights():
    full, kept, nbad = _batches()
    occ_f, st_f, _, s_f = oracle.ndt_integrate(MP, full)
    occ_k, st_k, _, s_k = oracle.ndt_integrate(MP, kept)
    assert np.array_equal(occ_f, occ_k) and np.array_equal(st_f.n, st_k.n)
    assert s_f["invalid"] == nbad
    box_min, box_dim = (4, 4, 4), (24, 24, 24)
    lab = np.zeros(box_dim[::-1])
    a_f = oracle.adjoint(MP, full, box_min, box_dim, lab, ndt=True)
    a_k = oracle.adjoint(MP, kept, box_min, box_dim, lab, ndt=True)
    assert a_f["loss"] == a_k["loss"]
    keep = np.setdiff1d(np.arange(full.n_rays), [3, 77, 150, 299])
    assert np.array_equal(a_f["grad_w"][keep], a_k["grad_w"])
    assert np.all(a_f["grad_w"][[3, 77, 150, 299]] == 0.0)
