"""Pins for the oracle's decay-rate layer (paper Sec. II-E: the reflection
rate of a voxel is its hits over the summed distance rays travel through it):

* every voxel's distance equals the length of the quantised segment inside
  that voxel's closed box, from exact rational slab intersection (brute
  force, ``bruteforce.segment_box_interval``), times the segment length;
* the distances of one ray add up to its length (inside the map when it is
  clipped); an axis-aligned ray gives whole voxel sizes inside;
* hit counts equal the count oracle's; zero-length visits add nothing.
"""
import math

import numpy as np
import pytest

import oracle
from bruteforce import segment_box_interval
from workloads import scenes
from workloads.scenes import RayBatch

F = 16


def quantise(p, m, s):
    return [int(np.rint((float(p[a]) - m[a]) * (2.0 ** F) / s)) for a in range(3)]


def seg_length(q0, q1, s):
    return math.sqrt(sum(float(b - a) ** 2 for a, b in zip(q0, q1))) * s / 2.0 ** F


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_distances_equal_exact_box_intersections(seed):
    mp = scenes.grid_map((-0.8, -0.8, -0.8), (0.8, 0.8, 0.8), 0.1)
    batch = scenes.random_rays(25, seed, None, None, (0.013, -0.021, 0.0305), 0.05, 0.7)
    length, _ = oracle.decay_integrate(mp, batch)
    exp = np.zeros_like(length)
    o = batch.origins[0]
    for e in batch.samples:
        q0, q1 = quantise(o, mp.map_origin, 0.1), quantise(e, mp.map_origin, 0.1)
        L = seg_length(q0, q1, 0.1)
        k0 = [q >> F for q in q0]
        k1 = [q >> F for q in q1]
        for k in np.ndindex(*(abs(b - a) + 3 for a, b in zip(k0, k1))):
            key = [min(a, b) - 1 + k[i] for i, (a, b) in enumerate(zip(k0, k1))]
            iv = segment_box_interval(q0, q1, key, F)
            if iv is None or iv[1] == iv[0]:
                continue
            exp[key[2], key[1], key[0]] += float(iv[1] - iv[0]) * L
    np.testing.assert_allclose(length, exp, rtol=1e-12, atol=1e-15)


def test_ray_distances_sum_to_its_length():
    mp = scenes.grid_map((-1.6, -1.6, -1.6), (1.6, 1.6, 1.6), 0.1, max_range=1.3)
    batch = scenes.random_rays(200, 8, None, None, (0.02, 0.03, -0.01), 0.1, 4.0)
    o = batch.origins[0]
    for i in range(0, 200, 7):
        one = RayBatch(batch.origins, batch.samples[i:i + 1], np.array([0, 1], np.uint32))
        length, _ = oracle.decay_integrate(mp, one)
        _, flags, _, keys = oracle.trace(mp, one)
        e = batch.samples[i].astype(np.float64)
        d = e - o
        if np.linalg.norm(d) > 1.3:
            e = o + d * (1.3 / np.linalg.norm(d))
        q0, q1 = quantise(o, mp.map_origin, 0.1), quantise(e, mp.map_origin, 0.1)
        L = seg_length(q0, q1, 0.1)
        if flags[0] & oracle.F_CLIPPED:
            # distance inside the map: up to the face the walk leaves through
            inside = sum(float(iv[1] - iv[0]) for k in keys
                         for iv in [segment_box_interval(q0, q1, list(k[:3]), F)] if iv is not None)
            assert abs(length.sum() - inside * L) < 1e-12
            assert length.sum() < L
        else:
            assert abs(length.sum() - L) < 1e-12 * max(L, 1.0)


def test_axis_aligned_ray_whole_voxels():
    mp = scenes.grid_map((-1.6, -1.6, -1.6), (1.6, 1.6, 1.6), 0.1)
    b = RayBatch(np.array([[0.025, 0.05, 0.05]], np.float32), np.array([[0.675, 0.05, 0.05]], np.float32),
                 np.array([0, 1], np.uint32))
    length, hits = oracle.decay_integrate(mp, b)
    row = length[16, 16, :]
    np.testing.assert_allclose(row[17:22], 0.1, rtol=1e-6)         # whole voxels 17..21
    assert abs(row[16] - 0.075) < 1e-6 and abs(row[22] - 0.075) < 1e-6
    assert hits[16, 16, 22] == 1 and hits.sum() == 1
    assert np.count_nonzero(length) == 7


def test_hits_match_count_oracle_and_modes_agree():
    mp = scenes.grid_map((-3.2, -3.2, -3.2), (3.2, 3.2, 3.2), 0.1, max_range=2.5)
    batch = scenes.random_rays(3000, 12, None, None, (0.01, 0.02, -0.03), 0.3, 3.5)
    length, hits = oracle.decay_integrate(mp, batch)
    _, o_hits, o_miss, st = oracle.integrate_count(mp, batch)
    assert np.array_equal(hits, o_hits.astype(np.uint32))
    # every voxel with updates got some distance (no ray here starts on a face)
    assert np.all(length[(o_hits + o_miss) > 0] > 0)
    assert np.all(length[(o_hits + o_miss) == 0] == 0)
    # two scans: sums
    b2 = RayBatch(np.concatenate([batch.origins, batch.origins]), np.concatenate([batch.samples, batch.samples]),
                  np.array([0, 3000, 6000], np.uint32))
    l2, h2 = oracle.decay_integrate(mp, b2)
    np.testing.assert_allclose(l2, 2 * length, rtol=1e-13)
    assert np.array_equal(h2, 2 * hits)


def test_face_origin_moving_negative_visits_with_zero_length():
    """Origin exactly on a voxel face, moving negative: the first voxel is a
    zero-length visit (walk reading: it is traversed) and gets distance 0."""
    mp = scenes.grid_map((-1.6, -1.6, -1.6), (1.6, 1.6, 1.6), 0.1)
    b = RayBatch(np.array([[0.0, 0.05, 0.05]], np.float32), np.array([[-0.33, 0.05, 0.05]], np.float32),
                 np.array([0, 1], np.uint32))
    length, _ = oracle.decay_integrate(mp, b)
    _, _, _, keys = oracle.trace(mp, b)
    assert tuple(keys[0, :3]) == (16, 16, 16) and length[16, 16, 16] == 0.0
    assert abs(length.sum() - 0.33) < 1e-6


def test_clipped_rays_stop_at_the_map_face():
    """Rays leaving the map: the distances add up to the part of the segment
    inside the map's box (exact rational clipping against its faces)."""
    from fractions import Fraction
    mp = scenes.grid_map((-0.8, -0.8, -0.8), (0.8, 0.8, 0.8), 0.1)
    batch = scenes.random_rays(60, 21, None, None, (0.013, -0.021, 0.0305), 0.5, 2.0)
    o = batch.origins[0]
    n_clipped = 0
    for i in range(60):
        one = RayBatch(batch.origins, batch.samples[i:i + 1], np.array([0, 1], np.uint32))
        length, _ = oracle.decay_integrate(mp, one)
        q0, q1 = quantise(o, mp.map_origin, 0.1), quantise(batch.samples[i], mp.map_origin, 0.1)
        L = seg_length(q0, q1, 0.1)
        t_hi = Fraction(1)
        for a in range(3):
            d = q1[a] - q0[a]
            lim = (16 << F) if d > 0 else 0
            if d != 0:
                t_hi = min(t_hi, Fraction(lim - q0[a], d))
        n_clipped += t_hi < 1
        assert abs(length.sum() - float(t_hi) * L) < 1e-12
    assert n_clipped > 20
