"""Batched multi-sensor integration (one graph launch over many uneven scans
into two maps) against the oracle and against per-scan launches: occupancy
and last-touched results must be bit-identical (count mode, unit weights)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2206_06079_amd as ohm
from gpu_helpers import device, per_update_tolerance, to_dev
from workloads import scenes

pytestmark = pytest.mark.gpu

# windows covering everything the scans touch (x -31..41 m, |y| <= 2.2, |z| <= 1.7)
WINDOWS = [((690, 978, 183), (720, 44, 34)), ((1380, 1956, 366), (1440, 88, 68))]


def make_sets(params, batches, capacities=(512, 1536)):
    maps, sets = [], []
    for p, b, cap in zip(params, batches, capacities):
        m = ohm.OhmMap(p, cap, device=device())
        o, s, off, w = to_dev(b)
        maps.append(m)
        sets.append(ohm.ScanSetArgs(m, o, s, off, w))
    return maps, sets


@pytest.fixture(scope="module")
def cfg3_small():
    # 16 streams, 96 scans, scan sizes scaled by 0.1 (819 .. 26,214 rays)
    return scenes.config3(n_streams=16, n_scans=96, size_scale=0.1)


@pytest.mark.parametrize("group", [1, 3, 8, 13])
def test_batched_equals_oracle_and_per_scan(cfg3_small, group):
    params, batches = cfg3_small
    maps, sets = make_sets(params, batches)
    plan = ohm.OhmBatch(sets, group)
    plan.run()
    torch.cuda.synchronize()
    # per-scan launches on fresh maps
    ref_maps, _ = make_sets(params, batches)
    for m, b in zip(ref_maps, batches):
        o, s, off, w = to_dev(b)
        m.integrate(o, s, off, w)
    for mi, (p, b) in enumerate(zip(params, batches)):
        bmin, bdim = WINDOWS[mi]
        got = maps[mi].read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy()
        per = ref_maps[mi].read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy()
        exp, _, _, st = oracle.integrate_count(p, b, bmin, bdim)
        assert np.array_equal(got, exp), f"map {mi}: batched differs from the oracle"
        assert np.array_equal(per, exp), f"map {mi}: per-scan differs from the oracle"
        assert maps[mi].stats()["voxel_updates"] == st["updates"]
    plan.close()


def test_batched_graph_replays_continue(cfg3_small):
    """Replaying the graph integrates the scans again, exactly like a second
    per-scan pass (tags survive replays)."""
    params, batches = cfg3_small
    maps, sets = make_sets(params, batches)
    plan = ohm.OhmBatch(sets, 4)
    plan.run()
    plan.run()
    torch.cuda.synchronize()
    for mi, (p, b) in enumerate(zip(params, batches)):
        bmin, bdim = WINDOWS[mi]
        twice = scenes.RayBatch(np.concatenate([b.origins, b.origins]), np.concatenate([b.samples, b.samples]),
                                np.concatenate([b.offsets, b.offsets[1:] + b.offsets[-1]]).astype(np.uint32))
        exp, _, _, _ = oracle.integrate_count(p, twice, bmin, bdim)
        got = maps[mi].read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy()
        assert np.array_equal(got, exp)
    plan.close()


def test_autotuner_picks_and_caches(cfg3_small, tmp_path):
    params, batches = cfg3_small
    maps, sets = make_sets(params, batches)
    cache = str(tmp_path / "tune.json")
    tiles = ((8, 256), (32, 1024))
    choice = ohm.autotune(sets, groups=(1, 4, 16), tiles=tiles, orders=(0, 1), cache_path=cache, reps=1)
    assert choice["group_scans"] in (1, 4, 16)
    assert (choice["seg_major_steps"], choice["tile_threads"]) in tiles
    assert choice["keep_ray_order"] in (0, 1)
    # served from the cache (the candidates offered now are ignored)
    assert ohm.autotune(sets, groups=(2,), tiles=((4, 512),), cache_path=cache) == choice
    # the caller's maps were not touched
    assert all(m.stats()["rays_in"] == 0 for m in maps)


@pytest.mark.parametrize("tile", [(1, 256, 0), (5, 1024, 1), (4096, 512, 0), (32, 512, 1)])
def test_batched_walk_tiles_agree(cfg3_small, tile):
    """Any segment length, tile shape and ray order gives the oracle's maps."""
    params, batches = cfg3_small
    maps, sets = make_sets(params, batches)
    plan = ohm.OhmBatch(sets, 2, seg_major_steps=tile[0], tile_threads=tile[1], keep_ray_order=tile[2])
    plan.run()
    torch.cuda.synchronize()
    for mi, (p, b) in enumerate(zip(params, batches)):
        bmin, bdim = WINDOWS[mi]
        exp, _, _, _ = oracle.integrate_count(p, b, bmin, bdim)
        assert np.array_equal(maps[mi].read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy(), exp)
    plan.close()


def test_per_scan_direction_order(cfg3_small):
    """Per-scan integration of unordered scans walked in direction order
    (ohm_map_set_ray_order) gives the oracle's maps, in both modes; scans
    longer than the scratch allows walk in their given order."""
    params, batches = cfg3_small
    for mi, (p, b) in enumerate(zip(params, batches)):
        bmin, bdim = WINDOWS[mi]
        o, s, off, w = to_dev(b)
        m = ohm.OhmMap(p, (512, 1536)[mi], device=device())
        sizes = np.diff(b.offsets.astype(np.int64))
        m.set_ray_order(int(np.median(sizes)))   # about half the scans are ordered
        m.integrate(o, s, off, w)
        exp, _, _, st = oracle.integrate_count(p, b, bmin, bdim)
        assert np.array_equal(m.read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy(), exp)
        assert m.stats()["voxel_updates"] == st["updates"]
        m.close()
    p, b = params[0].replace(mode=ohm.MODE_PER_UPDATE), batches[0]
    bmin, bdim = WINDOWS[0]
    o, s, off, w = to_dev(b)
    m = ohm.OhmMap(p, 512, device=device())
    m.set_ray_order(300000)
    m.integrate(o, s, off, w)
    lo, hi, nupd, _ = oracle.integrate_envelope(p, b, bmin, bdim)
    got = m.read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy()
    tol = per_update_tolerance(nupd)
    assert np.all(got >= lo - tol) and np.all(got <= hi + tol)
    m.close()
