"""GPU parity of the optional occupancy-walk layers against the oracle:

* voxel mean (OHM_LAYER_MEAN): count mode is exact, so packed codes and
  counts must equal the oracle bit for bit, per scan, through scan groups,
  with weights; per-update mode (compare-and-swap, any order) equals the
  oracle exactly where each voxel takes at most one sample per scan, and
  elsewhere keeps exact counts and codes within the samples' range;
* decay rate (OHM_LAYER_DECAY): hit counts exact; distances within the
  Q32.32 rounding of each visit (2^-33 m) and the fp64 rounding of the
  crossing parameters, plus the float read-back (2^-23 relative).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2206_06079_amd as ohm
from gpu_helpers import device, full_box, to_dev
from workloads import scenes
from workloads.scenes import RayBatch

pytestmark = pytest.mark.gpu

CFG1_BOX_MIN = (690, 978, 183)
CFG1_BOX_DIM = (720, 44, 34)


def run_layers(mp, batch, layers, box_min, box_dim, capacity=1024, calls=None):
    m = ohm.OhmMap(mp, capacity, layers=ohm.LAYER_OCC | layers, device=device())
    if calls is None:
        o, s, off, w = to_dev(batch)
        m.integrate(o, s, off, w)
    else:
        first = 0
        for cnt in calls:
            o, s, off, w = to_dev(batch.scans(first, cnt))
            m.integrate(o, s, off, w)
            first += cnt
    out = {"occ": m.read_dense(ohm.READ_OCC, box_min, box_dim).cpu().numpy(), "stats": m.stats()}
    if layers & ohm.LAYER_MEAN:
        out["packed"] = m.read_dense(ohm.READ_MEAN_PACKED, box_min, box_dim).cpu().numpy().view(np.uint32)
        out["count"] = m.read_dense(ohm.READ_MEAN_COUNT, box_min, box_dim).cpu().numpy().view(np.uint32)
        out["mean"] = m.read_dense(ohm.READ_MEAN, box_min, box_dim).cpu().numpy()
    if layers & ohm.LAYER_DECAY:
        out["length"] = m.read_dense(ohm.READ_DECAY_LENGTH, box_min, box_dim).cpu().numpy()
        out["hits"] = m.read_dense(ohm.READ_DECAY_HITS, box_min, box_dim).cpu().numpy().view(np.uint32)
        out["rate"] = m.read_dense(ohm.READ_DECAY_RATE, box_min, box_dim).cpu().numpy()
    m.close()
    return out


def groups(n):
    return ohm.LAYER_SCAN_GROUPS | ohm.scan_group_slots(n)


@pytest.mark.parametrize("variant", ["per_scan", "grouped", "grouped_weighted", "split_calls"])
def test_mean_count_mode_bit_exact(variant):
    mp, batch = scenes.config1(n_scans=4, first_scan=20)
    layers = ohm.LAYER_MEAN
    calls = None
    if variant.startswith("grouped"):
        layers |= groups(3)
    if variant == "grouped_weighted":
        batch.weights = np.random.default_rng(3).uniform(0.5, 1.0, batch.n_rays).astype(np.float32)
        layers = ohm.LAYER_MEAN | groups(6)
    if variant == "split_calls":
        calls = (1, 3)
    g = run_layers(mp, batch, layers, CFG1_BOX_MIN, CFG1_BOX_DIM, calls=calls)
    packed, count = oracle.mean_integrate(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM, mode=1)
    assert int(count.sum()) == g["stats"]["rays_hit"]
    assert np.array_equal(g["count"], count)
    assert np.array_equal(g["packed"], packed)
    # the float read-back is the code cell centre, relative to the voxel centre
    codes = oracle.unpack_mean(packed)
    has = count > 0
    exp = ((codes + 0.5) / 1024.0 - 0.5) * mp.voxel_size
    np.testing.assert_allclose(g["mean"][has], exp[has], atol=1e-7)
    assert np.all(g["mean"][~has] == 0)
    # the occupancy is untouched by the layer
    occ, _, _, _ = oracle.integrate_count(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM)
    if batch.weights is None:
        assert np.array_equal(g["occ"], occ)


def test_mean_per_update_one_sample_per_voxel_and_scan():
    """Each scan's rays end in distinct voxels, so every order of the
    compare-and-swap merges gives the oracle's result exactly."""
    mp = scenes.grid_map((-1.6, -1.6, -1.6), (1.6, 1.6, 1.6), 0.1, mode=scenes.MODE_PER_UPDATE)
    rng = np.random.default_rng(5)
    scans, origins = [], []
    for k in range(6):
        keys = rng.choice(32 ** 3, size=900, replace=False)
        kz, ky, kx = np.unravel_index(keys, (32, 32, 32))
        pts = np.stack([kx, ky, kz], 1) * 0.1 - 1.6 + rng.uniform(0.001, 0.099, size=(900, 3))
        scans.append(pts.astype(np.float32))
        origins.append([0.01 * k, 0.02, -0.03])
    batch = RayBatch(np.asarray(origins, np.float32), np.concatenate(scans),
                     (np.arange(7) * 900).astype(np.uint32))
    bmin, bdim = full_box(mp)
    g = run_layers(mp, batch, ohm.LAYER_MEAN, bmin, bdim, capacity=8)
    packed, count = oracle.mean_integrate(mp, batch, mode=0)
    assert np.array_equal(g["count"], count)
    assert np.array_equal(g["packed"], packed)


def test_mean_per_update_any_order_invariants():
    """Many samples per voxel and scan (config 0 ends near the sensor as
    well as far): counts exact, every code between the smallest and largest
    code of the voxel's samples."""
    mp, batch = scenes.config0(n_rays=20000, mode=scenes.MODE_PER_UPDATE)
    mp = mp.replace(max_range=0.0)
    rng = np.random.default_rng(11)
    # pull half the samples into a few voxels so they collide
    batch.samples[::2] = (np.array([2.05, -1.05, 0.55]) + rng.uniform(0, 0.09, size=(10000, 3))).astype(np.float32)
    bmin, bdim = full_box(mp)
    g = run_layers(mp, batch, ohm.LAYER_MEAN, bmin, bdim, capacity=343)
    packed, count = oracle.mean_integrate(mp, batch, mode=1)
    assert np.array_equal(g["count"], count)
    # per-voxel code range of the samples (codes from the quantised samples)
    q = np.rint((batch.samples.astype(np.float64) - np.asarray(mp.map_origin)) * (2.0 ** 16) / mp.voxel_size)
    q = q.astype(np.int64)
    keys = q >> 16
    codes = (q & 0xFFFF) >> 6
    inside = np.all((keys >= 0) & (keys < 200), axis=1)
    lin = (keys[:, 2] * 200 + keys[:, 1]) * 200 + keys[:, 0]
    lo = np.full((200 ** 3, 3), 1 << 20, np.int64)
    hi = np.full((200 ** 3, 3), -1, np.int64)
    for a in range(3):
        np.minimum.at(lo[:, a], lin[inside], codes[inside, a])
        np.maximum.at(hi[:, a], lin[inside], codes[inside, a])
    got = oracle.unpack_mean(g["packed"]).reshape(-1, 3)
    has = g["count"].reshape(-1) > 0
    assert has.sum() > 1000
    assert np.all(got[has] >= lo[has]) and np.all(got[has] <= hi[has])
    assert g["count"].max() > 100          # the collisions happened


def decay_tolerance(k, length):
    return k * 2.0 ** -32 + 2.0 ** -22 * length + 1e-9


@pytest.mark.parametrize("mode", [scenes.MODE_COUNT_CLAMP, scenes.MODE_PER_UPDATE])
def test_decay_config1_scans(mode):
    mp, batch = scenes.config1(n_scans=3, first_scan=40, mode=mode)
    layers = ohm.LAYER_DECAY | (groups(2) if mode == scenes.MODE_COUNT_CLAMP else 0)
    g = run_layers(mp, batch, layers, CFG1_BOX_MIN, CFG1_BOX_DIM)
    length, hits = oracle.decay_integrate(mp, batch, CFG1_BOX_MIN, CFG1_BOX_DIM)
    assert np.array_equal(g["hits"], hits)
    k = np.zeros(length.shape)
    for s in range(batch.n_scans):
        _, h, m_, _ = oracle.integrate_count(mp, batch.scans(s, 1), CFG1_BOX_MIN, CFG1_BOX_DIM)
        k += h + m_
    err = np.abs(g["length"].astype(np.float64) - length)
    assert np.all(err <= decay_tolerance(k, length)), err.max()
    pos = length > 1e-6
    rate = hits[pos] / length[pos]
    np.testing.assert_allclose(g["rate"][pos], rate, rtol=1e-5)
    assert np.all(g["rate"][~pos & (g["length"] == 0)] == 0)


def test_decay_and_mean_together_with_clipping_and_truncation():
    mp = scenes.grid_map((-1.6, -1.6, -1.6), (1.6, 1.6, 1.6), 0.1, max_range=1.4)
    batch = scenes.random_rays(30000, 44, None, None, (0.013, -0.021, 0.0305), 0.05, 3.0)
    bmin, bdim = full_box(mp)
    g = run_layers(mp, batch, ohm.LAYER_MEAN | ohm.LAYER_DECAY, bmin, bdim, capacity=8)
    length, hits = oracle.decay_integrate(mp, batch)
    packed, count = oracle.mean_integrate(mp, batch, mode=1)
    assert np.array_equal(g["hits"], hits) and np.array_equal(g["count"], count)
    assert np.array_equal(g["packed"], packed)
    _, h, m_, _ = oracle.integrate_count(mp, batch)
    err = np.abs(g["length"].astype(np.float64) - length)
    assert np.all(err <= decay_tolerance(h + m_, length)), err.max()
    assert g["stats"]["rays_truncated"] > 1000


def test_layer_combinations_rejected():
    mp = scenes.grid_map((-1.6, -1.6, -1.6), (1.6, 1.6, 1.6), 0.1)
    for layers in (ohm.LAYER_NDT | ohm.LAYER_MEAN, ohm.LAYER_NDT | ohm.LAYER_DECAY):
        with pytest.raises(ohm.OhmError) as e:
            ohm.OhmMap(mp, 8, layers=layers, device=device())
        assert e.value.status == ohm.OHM_E_UNSUPPORTED
    m = ohm.OhmMap(mp, 8, layers=ohm.LAYER_MEAN, device=device())
    batch = scenes.random_rays(100, 1, None, None, (0.0, 0.0, 0.0), 0.1, 1.0)
    o, s, off, w = to_dev(batch)
    with pytest.raises(ohm.OhmError) as e:
        ohm.OhmBatch([ohm.ScanSetArgs(m, o, s, off)], 1)
    assert e.value.status == ohm.OHM_E_UNSUPPORTED
    with pytest.raises(ohm.OhmError):
        ohm.OhmMap(mp, 8, device=device()).read_dense(ohm.READ_DECAY_RATE, (0, 0, 0), (2, 2, 2))
    m.close()
