"""GPU parity of the NDT-OM path (ohm_ndt_integrate) against the CPU oracle.

Sample counts must match exactly; means and covariances within 1e-5 (m, m^2);
occupancy within 1e-5 plus the fixed-point quantisation of the summed
increments (2^-33 per update)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2206_06079_amd as ohm
from gpu_helpers import device, per_update_tolerance, to_dev
from workloads import scenes

pytestmark = pytest.mark.gpu

CFG1_BOX_MIN = (690, 978, 183)
CFG1_BOX_DIM = (720, 44, 34)


def gpu_ndt(mp, batch, box_min, box_dim, capacity=1024, scans_per_call=None):
    m = ohm.OhmMap(mp, capacity, layers=ohm.LAYER_NDT, device=device())
    if scans_per_call is None:
        o, s, off, w = to_dev(batch)
        m.ndt_integrate(o, s, off, w)
    else:
        for first in range(0, batch.n_scans, scans_per_call):
            sub = batch.scans(first, min(scans_per_call, batch.n_scans - first))
            o, s, off, w = to_dev(sub)
            m.ndt_integrate(o, s, off, w)
    out = dict(
        occ=m.read_dense(ohm.READ_OCC, box_min, box_dim).cpu().numpy(),
        n=m.read_dense(ohm.READ_NDT_COUNT, box_min, box_dim).cpu().numpy().astype(np.uint32),
        mu=m.read_dense(ohm.READ_NDT_MEAN, box_min, box_dim).cpu().numpy(),
        cov=m.read_dense(ohm.READ_NDT_COV, box_min, box_dim).cpu().numpy(),
        stats=m.stats(),
    )
    m.close()
    return out


def update_counts(mp, batch, box_min, box_dim):
    """Per-voxel number of updates over all scans (unit-weight count oracle)."""
    total = np.zeros((box_dim[2], box_dim[1], box_dim[0]), np.int64)
    for s in range(batch.n_scans):
        _, h, mm, _ = oracle.integrate_count(mp.replace(max_range=mp.max_range), batch.scans(s, 1), box_min, box_dim)
        total += (h + mm).astype(np.int64)
    return total


def check_stats(g, o_occ, o_state, k, tol_occ=None):
    assert np.array_equal(g["n"], o_state.n), "sample counts differ"
    has = o_state.n > 0
    assert has.sum() > 100
    np.testing.assert_allclose(g["mu"][has], o_state.mu[has], atol=1e-5, rtol=0)
    np.testing.assert_allclose(g["cov"][has], o_state.cov[has], atol=1e-5, rtol=1e-4)
    if tol_occ is None:
        tol_occ = 1e-5 + k * 2.0 ** -33
    err = np.abs(g["occ"].astype(np.float64) - o_occ.astype(np.float64))
    assert np.all(err <= tol_occ), f"max occupancy error {err.max()}"


def test_ndt_count_mode_config2_scans():
    mp, batch = scenes.config2(n_scans=4, first_scan=20)
    g = gpu_ndt(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM)
    o_occ, o_state, _, o_st = oracle.ndt_integrate(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM, mode=1)
    k = update_counts(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM)
    check_stats(g, o_occ, o_state, k)
    assert g["stats"]["voxel_updates"] == o_st["updates"]
    # the Gaussian weighting was exercised: some voxels held >= 4 samples
    assert (o_state.n >= 4).sum() > 1000


def test_ndt_count_mode_split_calls():
    mp, batch = scenes.config2(n_scans=3, first_scan=40)
    g = gpu_ndt(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM, scans_per_call=1)
    o_occ, o_state, _, _ = oracle.ndt_integrate(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM, mode=1)
    check_stats(g, o_occ, o_state, update_counts(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM))


def test_ndt_per_update_mode():
    mp, batch = scenes.config2(n_scans=3, first_scan=60, mode=scenes.MODE_PER_UPDATE)
    g = gpu_ndt(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM)
    o_occ, o_state, _, _ = oracle.ndt_integrate(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM, mode=0)
    k = update_counts(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM)
    check_stats(g, o_occ, o_state, k, tol_occ=1e-5 + per_update_tolerance(k.astype(np.uint32)) + k * 2.0 ** -33)


def test_ndt_weighted_and_clearing():
    mp, batch = scenes.config2(n_scans=3, first_scan=5)
    mp = mp.replace(ndt_clear_below=-1.0)
    batch.weights = np.random.default_rng(4).uniform(0.5, 1.0, batch.n_rays).astype(np.float32)
    g = gpu_ndt(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM)
    o_occ, o_state, _, _ = oracle.ndt_integrate(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM, mode=1)
    k = update_counts(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM)
    check_stats(g, o_occ, o_state, k)


def test_ndt_small_map_first_scan_equals_plain():
    """First scan of an empty NDT map: same occupancy as the plain path."""
    mp = scenes.grid_map((-3.2, -3.2, -3.2), (3.2, 3.2, 3.2), 0.1, max_range=2.5)
    batch = scenes.random_rays(5000, 12, None, None, (0.01, 0.02, -0.03), 0.3, 3.5)
    box_min, box_dim = (0, 0, 0), mp.dims
    g = gpu_ndt(mp, batch, box_min, box_dim, capacity=16)
    o_occ, _, _, _ = oracle.integrate_count(mp, batch)
    k = update_counts(mp, batch, box_min, box_dim)
    assert np.all(np.abs(g["occ"] - o_occ) <= 1e-5 + k * 2.0 ** -33)


def test_ndt_threshold_change_between_calls():
    """Changing ndt_min_samples between calls (ohm_map_set_params) applies the
    new threshold to every voxel's existing samples in the next call."""
    mp, batch = scenes.config2(n_scans=4, first_scan=50)
    m = ohm.OhmMap(mp, 1024, layers=ohm.LAYER_NDT, device=device())
    o, s, off, w = to_dev(batch.scans(0, 2))
    m.ndt_integrate(o, s, off, w)
    mp3 = mp.replace(ndt_min_samples=3)
    m.set_params(mp3)
    o, s, off, w = to_dev(batch.scans(2, 2))
    m.ndt_integrate(o, s, off, w)
    occ = m.read_dense(ohm.READ_OCC, CFG1_BOX_MIN, CFG1_BOX_DIM).cpu().numpy()
    n = m.read_dense(ohm.READ_NDT_COUNT, CFG1_BOX_MIN, CFG1_BOX_DIM).cpu().numpy().astype(np.uint32)
    m.close()
    o_occ, o_state, _, _ = oracle.ndt_integrate(mp, batch.scans(0, 2), CFG1_BOX_MIN, CFG1_BOX_DIM, mode=1)
    o_occ, o_state, _, _ = oracle.ndt_integrate(mp3, batch.scans(2, 2), CFG1_BOX_MIN, CFG1_BOX_DIM, occ=o_occ,
                                                state=o_state, mode=1)
    assert np.array_equal(n, o_state.n)
    k = update_counts(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM)
    assert np.all(np.abs(occ.astype(np.float64) - o_occ) <= 1e-5 + k * 2.0 ** -33)
    # voxels holding exactly 3 samples after the first two scans take weighted misses now
    assert (o_state.n == 3).sum() > 100


def hit_block_batch(seed=11):
    """Scans of ragged sizes around the 512-ray hit blocks (1, 511, 512, 513,
    1500, 3000 rays), half of each scan's rays ending within 1 cm of one of
    three points (many hits in one voxel), the rest in random directions,
    some beyond the 2.5 m range (truncated: no hit); a few NaN samples; 5 % of
    the weights zero (a hit that adds its sample but no occupancy)."""
    rng = np.random.default_rng(seed)
    sizes = [1, 511, 512, 513, 1500, 3000]
    targets = np.array([[1.23, 0.47, -0.66], [-0.91, 1.58, 0.35], [0.12, -1.74, 1.05]])
    origins, samples = [], []
    for s, n in enumerate(sizes):
        o = np.array([0.01 * s, -0.02 * s, 0.015 * s])
        d = rng.normal(size=(n, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        pts = o + d * rng.uniform(0.3, 3.5, size=(n, 1))
        near = rng.random(n) < 0.5
        pts[near] = targets[rng.integers(0, 3, near.sum())] + rng.uniform(-0.01, 0.01, (near.sum(), 3))
        origins.append(o)
        samples.append(pts)
    samples = np.concatenate(samples).astype(np.float32)
    samples[rng.choice(samples.shape[0], 4, replace=False), 1] = np.nan
    weights = rng.uniform(0.5, 1.0, samples.shape[0]).astype(np.float32)
    weights[rng.random(samples.shape[0]) < 0.05] = 0.0
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    return scenes.RayBatch(np.array(origins, np.float32), samples, offsets, weights)


@pytest.mark.parametrize("weighted", [False, True])
def test_ndt_hit_blocks_ragged_and_crowded(weighted):
    """The hit samples are summed per voxel in 512-ray blocks of the walk's
    launch: scans shorter than a block, a ragged last block, hundreds of
    samples landing in one voxel, zero weights and invalid rays all give the
    oracle's sample counts and statistics."""
    mp = scenes.grid_map((-3.2, -3.2, -3.2), (3.2, 3.2, 3.2), 0.1, max_range=2.5)
    batch = hit_block_batch()
    if not weighted:
        batch.weights = None
    box_min, box_dim = (0, 0, 0), mp.dims
    g = gpu_ndt(mp, batch, box_min, box_dim, capacity=16)
    o_occ, o_state, _, _ = oracle.ndt_integrate(mp, batch, box_min, box_dim, mode=1)
    assert o_state.n.max() > 200  # one voxel took hundreds of samples
    k = update_counts(mp, batch, box_min, box_dim)
    check_stats(g, o_occ, o_state, k)
