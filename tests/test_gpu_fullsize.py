"""The benchmark's workloads at full size, in the launch configurations it
times.

Headline: 100 spinning-lidar scans of 131,072 rays each (0.1 m voxels, 30 m
range) through
- one ohm_integrate_rays call on a map with 50-scan groups and the scans
  declared column-major, 64 rays per column (the benchmark's timed
  configuration: 8-beam by 32-column patch tiles), and without the layout;
- the same call on a map that launches once per scan;
- a batched plan of 50-scan groups over the same scans.
Count mode with unit weights is exact, so every voxel of a window holding
everything the scans reach (x 690..1409, y 978..1021, z 183..216; the
touched voxels lie at least one voxel inside each face) must equal the
oracle bit for bit, and so must the update and ray counts.

Per-update mode: the same 100 scans with each update applied and clamped
on its own (compare-and-swap), inside the oracle's bracket over every order
of a scan's updates (plus one ulp per update).

NDT-OM: the same 100 scans into an NDT map of 512 regions, within the NDT
tolerances (exact sample counts; mean and covariance within 1e-5; occupancy
within 1e-5 plus 2^-33 per update).

Adjoint: 20 weighted scans at 0.2 m into an NDT map, then the backward for
the masked BCE gradient, within 1e-4 of the oracle's fp64 gradients.

Batched streams: the first 128 of the 16-stream workload's 1,000 scans, at
full scan sizes (log-uniform 8,192..262,144 rays, 8.8 M rays, two maps at
0.1 m and 0.05 m), through the plan the benchmark's autotuner settles on
(64-scan groups, 32 major crossings per segment, 512 threads, direction
order); both maps bit-exact against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2206_06079_amd as ohm
from gpu_helpers import device, gpu_integrate, per_update_tolerance, to_dev
from test_gpu_adjoint import check, gpu_grads, in_box_counts, setup_case
from test_gpu_batch import WINDOWS, make_sets
from test_gpu_ndt import check_stats, gpu_ndt, update_counts
from workloads import scenes

pytestmark = pytest.mark.gpu

BOX_MIN = (690, 978, 183)
BOX_DIM = (720, 44, 34)
HEADLINE = ohm.LAYER_OCC | ohm.LAYER_SCAN_GROUPS | ohm.scan_group_slots(50)


@pytest.fixture(scope="module")
def headline():
    mp, batch = scenes.config1(n_scans=100)
    print(f"oracle: {batch.n_scans} scans, {batch.samples.shape[0]} rays", flush=True)
    exp = oracle.integrate_count(mp, batch, BOX_MIN, BOX_DIM)
    return mp, batch, exp


@pytest.mark.parametrize("layers,column_rays", [(HEADLINE, 64), (HEADLINE, 0), (ohm.LAYER_OCC, 0)],
                         ids=["groups50_layout64", "groups50", "per_scan"])
def test_headline_workload_equals_oracle(headline, layers, column_rays):
    mp, batch, (o_occ, o_hit, o_miss, o_st) = headline
    occ, hits, miss, st = gpu_integrate(mp, batch, 512, BOX_MIN, BOX_DIM, layers=layers, column_rays=column_rays)
    assert np.count_nonzero(o_occ) > 500_000
    assert np.array_equal(occ, o_occ)
    # the call's last scan keeps its counts readable
    assert np.array_equal(hits, o_hit) and np.array_equal(miss, o_miss)
    assert st["voxel_updates"] == o_st["updates"] == 677_555_021
    assert st["rays_in"] == o_st["rays"] and st["rays_truncated"] == o_st["truncated"]
    assert st["updates_dropped_pool"] == 0


@pytest.mark.parametrize("seg_major_steps,keep_ray_order", [(16, 0), (32, 1)])
def test_headline_workload_batched_equals_oracle(headline, seg_major_steps, keep_ray_order):
    """The benchmark's batched leg on the headline scans, in the launch
    configurations its autotuner chooses between (50 scans per group)."""
    mp, batch, (o_occ, _, _, o_st) = headline
    m = ohm.OhmMap(mp, 512, device=device())
    o, s, off, w = to_dev(batch)
    plan = ohm.OhmBatch([ohm.ScanSetArgs(m, o, s, off, w)], 50, seg_major_steps=seg_major_steps, tile_threads=512,
                        keep_ray_order=keep_ray_order)
    plan.run()
    torch.cuda.synchronize()
    occ = m.read_dense(ohm.READ_OCC, BOX_MIN, BOX_DIM).cpu().numpy()
    assert np.array_equal(occ, o_occ)
    assert m.stats()["voxel_updates"] == o_st["updates"]
    plan.close()
    m.close()


def test_per_update_headline_scans_within_envelope():
    mp, batch = scenes.config1(n_scans=100, mode=scenes.MODE_PER_UPDATE)
    occ, _, _, st = gpu_integrate(mp, batch, 512, BOX_MIN, BOX_DIM)
    lo, hi, nupd, o_st = oracle.integrate_envelope(mp, batch, BOX_MIN, BOX_DIM)
    tol = per_update_tolerance(nupd)
    assert np.all(occ >= lo - tol) and np.all(occ <= hi + tol)
    # voxels whose every order gives one value must take it
    free = (hi - lo) < 1e-12
    assert free.sum() > 100_000
    assert np.all(np.abs(occ[free] - lo[free]) <= np.maximum(tol[free], 1e-5))
    assert st["voxel_updates"] == o_st["updates"]
    assert st["updates_dropped_pool"] == 0


def test_ndt_headline_scans_equal_oracle():
    mp, batch = scenes.config2(n_scans=100)
    print(f"NDT: {batch.n_scans} scans, {batch.samples.shape[0]} rays", flush=True)
    g = gpu_ndt(mp, batch, BOX_MIN, BOX_DIM, capacity=512)
    o_occ, o_state, _, o_st = oracle.ndt_integrate(mp, batch, BOX_MIN, BOX_DIM, mode=1)
    k = update_counts(mp, batch, BOX_MIN, BOX_DIM)
    check_stats(g, o_occ, o_state, k)
    assert g["stats"]["voxel_updates"] == o_st["updates"]
    assert g["stats"]["updates_dropped_pool"] == 0
    assert (o_state.n >= 4).sum() > 50_000


def test_adjoint_twenty_weighted_scans():
    params, batch, box_min, box_dim, labels, mask, ref = setup_case(20)
    print(f"adjoint: {batch.n_scans} scans, {batch.samples.shape[0]} rays", flush=True)
    gw, gs, occ, n_after = gpu_grads(params, batch, box_min, box_dim, labels, mask)
    np.testing.assert_allclose(occ, ref["occ"], atol=1e-5, rtol=0)
    check(gw, gs, ref, in_box_counts(params, batch, box_min, box_dim), batch.n_scans)


def test_batched_streams_full_scan_sizes():
    params, batches = scenes.config3(n_streams=16, n_scans=128, jobs=16)
    print(f"batched: {[b.samples.shape[0] for b in batches]} rays per map", flush=True)
    maps, sets = make_sets(params, batches)
    plan = ohm.OhmBatch(sets, 64, seg_major_steps=16, tile_threads=512, keep_ray_order=0)
    plan.run()
    torch.cuda.synchronize()
    for mi, (p, b) in enumerate(zip(params, batches)):
        bmin, bdim = WINDOWS[mi]
        got = maps[mi].read_dense(ohm.READ_OCC, bmin, bdim).cpu().numpy()
        exp, _, _, st = oracle.integrate_count(p, b, bmin, bdim)
        assert np.count_nonzero(exp) > 500_000
        assert np.array_equal(got, exp), f"map {mi}: batched differs from the oracle"
        assert maps[mi].stats()["voxel_updates"] == st["updates"]
        assert maps[mi].stats()["updates_dropped_pool"] == 0
    plan.close()
    for m in maps:
        m.close()
