"""GPU coverage of the weighted kernel instances and of call sequences that
mix the per-scan, grouped and batched paths on one map:

* weighted count mode through scan groups and through a batched plan, bit-
  identical to weighted per-scan calls (the Q32.32 sums are exact integers);
* weighted per-update mode (plain and NDT) inside the oracle's bounds;
* rays with negative or non-finite weights skipped whole, like the oracle;
* per-scan and NDT calls after a batched plan on the same map;
* the adjoint refusing a map that a batched plan has integrated into;
* the NDT sample threshold and the truncated segment end, on the device.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2206_06079_amd as ohm
from gpu_helpers import device, full_box, gpu_integrate, per_update_tolerance, to_dev
from workloads import scenes
from workloads.scenes import RayBatch

pytestmark = pytest.mark.gpu

WINDOWS = [((690, 978, 183), (720, 44, 34)), ((1380, 1956, 366), (1440, 88, 68))]
Q = 2.0 ** -33


def small_map(n=48, voxel=0.1, **kw):
    return scenes.grid_map((-n * voxel / 2,) * 3, (n * voxel / 2,) * 3, voxel, **kw)


def weighted_scans(n_scans=5, n_rays=3000, seed=40):
    parts = [scenes.random_rays(n_rays, seed + k, None, None, (0.01 * k, -0.02, 0.03), 0.2, 2.2)
             for k in range(n_scans)]
    w = np.random.default_rng(seed).uniform(0.5, 1.0, n_scans * n_rays).astype(np.float32)
    return RayBatch(np.concatenate([b.origins for b in parts]), np.concatenate([b.samples for b in parts]),
                    (np.arange(n_scans + 1) * n_rays).astype(np.uint32), w)


def update_counts(mp, batch, bmin, bdim):
    k = np.zeros((bdim[2], bdim[1], bdim[0]), np.float64)
    for s in range(batch.n_scans):
        b = batch.scans(s, 1)
        b.weights = None
        _, h, m, _ = oracle.integrate_count(mp, b, bmin, bdim)
        k += h + m
    return k


@pytest.mark.parametrize("slots", [2, 7, 8])
def test_weighted_groups_equal_weighted_per_scan(slots):
    """Scan groups with weights use wide slots (two f32 slots each): with 2,
    7 or 8 slots the groups hold 1, 3 or 4 scans.  Bit-identical to per-scan
    launches; within k 2^-33 + 1e-5 of the oracle."""
    mp = small_map(48, max_range=1.9)
    batch = weighted_scans(9)
    bmin, bdim = full_box(mp)
    per, hp, mp_, _ = gpu_integrate(mp, batch, 32, bmin, bdim)
    layers = ohm.LAYER_OCC | ohm.LAYER_SCAN_GROUPS | ohm.scan_group_slots(slots)
    grp, hg, mg, st = gpu_integrate(mp, batch, 32, bmin, bdim, layers=layers)
    assert np.array_equal(per, grp)
    assert np.array_equal(hp, hg) and np.array_equal(mp_, mg)
    exp, _, _, o_st = oracle.integrate_count(mp, batch)
    k = update_counts(mp, batch, bmin, bdim)
    assert np.all(np.abs(grp.astype(np.float64) - exp) <= 1e-5 + k * Q)
    assert st["voxel_updates"] == o_st["updates"]


def test_mixed_weighted_and_unit_calls():
    """Calls alternating unit and per-ray weights on one map (the kept slot
    switches between f32 counts and wide sums): the oracle's sequence."""
    mp = small_map(48)
    batch = weighted_scans(4, 2000, seed=70)
    bmin, bdim = full_box(mp)
    m = ohm.OhmMap(mp, 32, layers=ohm.LAYER_OCC | ohm.LAYER_SCAN_GROUPS | ohm.scan_group_slots(4),
                   device=device())
    occ = np.full((bdim[2], bdim[1], bdim[0]), np.float32(mp.l_init), np.float32)
    k = np.zeros(occ.shape)
    for s, weighted in enumerate((True, False, True, False)):
        sub = batch.scans(s, 1)
        if not weighted:
            sub.weights = None
        o, smp, off, w = to_dev(sub)
        m.integrate(o, smp, off, w)
        occ, _, _, _ = oracle.integrate_count(mp, sub, bmin, bdim, occ=occ)
        k += update_counts(mp, sub, bmin, bdim)
        got = m.read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy()
        assert np.all(np.abs(got.astype(np.float64) - occ) <= 1e-5 + k * Q), s
        hits = m.read_dense(ohm.READ_HITS, bmin, bdim).cpu().numpy()
        _, o_hit, _, _ = oracle.integrate_count(mp, sub, bmin, bdim)
        assert np.all(np.abs(hits - o_hit) <= 1e-5), s
    m.close()


def test_weighted_batched_equals_weighted_per_scan():
    params, batches = scenes.config3(n_streams=16, n_scans=48, size_scale=0.05)
    rng = np.random.default_rng(9)
    for b in batches:
        b.weights = rng.uniform(0.5, 1.0, b.n_rays).astype(np.float32)
    maps, sets = [], []
    for p, b, cap in zip(params, batches, (512, 1536)):
        m = ohm.OhmMap(p, cap, device=device())
        o, s, off, w = to_dev(b)
        maps.append(m)
        sets.append(ohm.ScanSetArgs(m, o, s, off, w))
    plan = ohm.OhmBatch(sets, 5)
    plan.run()
    torch.cuda.synchronize()
    for mi, (p, b, cap) in enumerate(zip(params, batches, (512, 1536))):
        bmin, bdim = WINDOWS[mi]
        ref = ohm.OhmMap(p, cap, device=device())
        o, s, off, w = to_dev(b)
        ref.integrate(o, s, off, w)
        per = ref.read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy()
        got = maps[mi].read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy()
        assert np.array_equal(got, per), f"map {mi}: weighted batched differs from weighted per-scan"
        exp, _, _, _ = oracle.integrate_count(p, b, bmin, bdim)
        k = update_counts(p, b, bmin, bdim)
        assert np.all(np.abs(got.astype(np.float64) - exp) <= 1e-5 + k * Q)
        ref.close()
    plan.close()
    for m in maps:
        m.close()


def test_per_update_weighted_in_bracket():
    mp = small_map(48, mode=scenes.MODE_PER_UPDATE, l_min=-1.2, l_max=1.6)
    batch = weighted_scans(3, 4000, seed=90)
    bmin, bdim = full_box(mp)
    occ, _, _, st = gpu_integrate(mp, batch, 32, bmin, bdim)
    lo, hi, nupd, o_st = oracle.integrate_envelope(mp, batch)
    tol = per_update_tolerance(nupd)
    assert np.all(occ >= lo - tol) and np.all(occ <= hi + tol)
    free = (hi - lo) < 1e-12
    assert free.sum() > 1000
    assert np.all(np.abs(occ[free] - lo[free]) <= np.maximum(tol[free], 1e-5))
    assert st["voxel_updates"] == o_st["updates"]


def test_ndt_per_update_weighted():
    """Weighted per-update NDT: misses by compare-and-swap in any order (all
    of one sign), then the hits: the oracle's misses-then-hits value within
    the per-update rounding bound."""
    mp, batch = scenes.config2(n_scans=3, first_scan=30, mode=scenes.MODE_PER_UPDATE)
    batch.weights = np.random.default_rng(12).uniform(0.5, 1.0, batch.n_rays).astype(np.float32)
    bmin, bdim = WINDOWS[0]
    m = ohm.OhmMap(mp, 1024, layers=ohm.LAYER_NDT, device=device())
    o, s, off, w = to_dev(batch)
    m.ndt_integrate(o, s, off, w)
    occ = m.read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy()
    n = m.read_dense(ohm.READ_NDT_COUNT, bmin, bdim).cpu().numpy().astype(np.uint32)
    m.close()
    o_occ, o_state, _, _ = oracle.ndt_integrate(mp, batch, bmin, bdim, mode=0)
    k = update_counts(mp.replace(mode=scenes.MODE_COUNT_CLAMP), batch, bmin, bdim)
    assert np.array_equal(n, o_state.n)
    tol = 1e-5 + per_update_tolerance(k.astype(np.uint32)) + k * Q
    err = np.abs(occ.astype(np.float64) - o_occ.astype(np.float64))
    assert np.all(err <= tol), err.max()


@pytest.mark.parametrize("mode", [scenes.MODE_COUNT_CLAMP, scenes.MODE_PER_UPDATE])
def test_bad_weights_skip_the_ray(mode):
    mp = small_map(32, mode=mode)
    batch = scenes.random_rays(2000, 17, None, None, (0.02, 0.0, -0.01), 0.2, 1.5)
    w = np.random.default_rng(2).uniform(0.5, 1.0, 2000).astype(np.float32)
    bad = [5, 600, 1999, 1024]
    w[bad] = [-1.0, np.nan, np.inf, -0.0]      # -0.0 is a valid (zero) weight
    batch.weights = w
    bmin, bdim = full_box(mp)
    occ, _, _, st = gpu_integrate(mp, batch, 8, bmin, bdim)
    assert st["rays_invalid"] == 3 and (st["sticky_error"] & 4)
    if mode == scenes.MODE_COUNT_CLAMP:
        exp, _, _, o_st = oracle.integrate_count(mp, batch)
        assert np.abs(occ.astype(np.float64) - exp).max() <= 1e-5
    else:
        lo, hi, nupd, o_st = oracle.integrate_envelope(mp, batch)
        tol = per_update_tolerance(nupd)
        assert np.all(occ >= lo - tol) and np.all(occ <= hi + tol)
    assert st["voxel_updates"] == o_st["updates"] and o_st["invalid"] == 3


def test_bad_weights_ndt_and_unit_weights_unflagged():
    mp = small_map(32)
    batch = scenes.random_rays(1500, 18, None, None, (0.0, 0.01, 0.0), 0.2, 1.5)
    batch.weights = np.ones(1500, np.float32)
    batch.weights[[7, 8]] = [np.nan, -2.0]
    m = ohm.OhmMap(mp, 8, layers=ohm.LAYER_NDT, device=device())
    o, s, off, w = to_dev(batch)
    m.ndt_integrate(o, s, off, w)
    bmin, bdim = full_box(mp)
    n = m.read_dense(ohm.READ_NDT_COUNT, bmin, bdim).cpu().numpy().astype(np.uint32)
    st = m.stats()
    m.close()
    _, o_state, _, o_st = oracle.ndt_integrate(mp, batch)
    assert np.array_equal(n, o_state.n) and st["rays_invalid"] == o_st["invalid"] == 2
    assert st["sticky_error"] & 4
    m = ohm.OhmMap(mp, 8, device=device())
    m.integrate(o, s, off, None)
    assert m.stats()["sticky_error"] == 0
    m.close()


def test_per_scan_and_ndt_calls_after_a_batched_plan():
    """A plan run leaves both touched lists empty, so later per-scan and NDT
    calls on the same map list their regions from zero (an NDT map used
    as a plain count-mode map by the plan)."""
    p0, b0 = scenes.config3(n_streams=2, n_scans=6, size_scale=0.1)
    mp = p0[0].replace(sensor_noise=0.05, adaptation_rate=1.0, ndt_min_samples=4)
    batch = b0[0]
    bmin, bdim = WINDOWS[0]
    for reps in (1, 2):
        m = ohm.OhmMap(mp, 512, layers=ohm.LAYER_NDT, device=device())
        o, s, off, w = to_dev(batch)
        plan = ohm.OhmBatch([ohm.ScanSetArgs(m, o, s, off)], 2)
        for _ in range(reps):
            plan.run()
        plan.close()
        # then a plain call and an NDT call on the same map
        extra = scenes.config1(n_scans=2, first_scan=3)[1]
        eo, es, eoff, _ = to_dev(extra.scans(0, 1))
        m.integrate(eo, es, eoff)
        no, ns, noff, _ = to_dev(extra.scans(1, 1))
        m.ndt_integrate(no, ns, noff)
        got = m.read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy()
        n = m.read_dense(ohm.READ_NDT_COUNT, bmin, bdim).cpu().numpy().astype(np.uint32)
        m.close()
        seq = RayBatch(np.concatenate([batch.origins] * reps), np.concatenate([batch.samples] * reps),
                       np.concatenate([batch.offsets[:-1] + i * batch.offsets[-1] for i in range(reps)]
                                      + [[reps * batch.offsets[-1]]]).astype(np.uint32))
        occ, _, _, _ = oracle.integrate_count(mp, seq, bmin, bdim)
        occ, _, _, _ = oracle.integrate_count(mp, extra.scans(0, 1), bmin, bdim, occ=occ)
        occ, state, _, _ = oracle.ndt_integrate(mp, extra.scans(1, 1), bmin, bdim, occ=occ)
        k = update_counts(mp, extra.scans(1, 1), bmin, bdim)
        assert np.all(np.abs(got.astype(np.float64) - occ) <= 1e-5 + k * Q), reps
        assert np.array_equal(n, state.n)


def test_backward_refuses_a_batched_map():
    p0, b0 = scenes.config3(n_streams=2, n_scans=4, size_scale=0.05)
    m = ohm.OhmMap(p0[0], 512, layers=ohm.LAYER_ADJOINT, device=device())
    o, s, off, w = to_dev(b0[0])
    plan = ohm.OhmBatch([ohm.ScanSetArgs(m, o, s, off)], 2)
    plan.run()
    plan.close()
    g = torch.zeros((4, 4, 4), device=device())
    with pytest.raises(ohm.OhmError) as e:
        m.backward(g, (0, 0, 0), (4, 4, 4), o, s, off, None, ndt=False)
    assert e.value.status == ohm.OHM_E_UNSUPPORTED
    m.reset()
    m.integrate(o, s, off)
    m.backward(g, (0, 0, 0), (4, 4, 4), o, s, off, None, ndt=False)   # accepted after a reset
    m.close()


# --- the NDT readings pinned in the oracle, on the device -------------------

@pytest.mark.parametrize("case", ["threshold_3", "threshold_4", "truncated"])
def test_ndt_pins_on_device(case):
    import test_oracle_ndt_pins as pins
    if case == "truncated":
        mp, batch, _ = pins.two_scans(4, (2.05, pins.MU[1] + pins.OFF, pins.MU[2]), max_range=0.97)
    else:
        mp, batch, _ = pins.two_scans(int(case[-1]), (1.05, pins.MU[1] + pins.OFF, pins.MU[2]))
    m = ohm.OhmMap(mp, 8, layers=ohm.LAYER_NDT, device=device())
    o, s, off, w = to_dev(batch)
    m.ndt_integrate(o, s, off, w)
    got = float(m.read_dense(ohm.READ_OCC, pins.KEY, (1, 1, 1)).cpu().numpy()[0, 0, 0])
    m.close()
    exp, _ = pins.ndt_occ(mp, batch)
    assert abs(got - exp) <= 1e-6
