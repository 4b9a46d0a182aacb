"""Pins for the oracle's voxel mean layer (paper Sec. III-A: a 32-bit
discretised mean position, 10 bits of sub-voxel position per axis, and a
32-bit sample count):

* a sample's 10-bit code equals floor(1024 x (position inside its voxel) /
  voxel size), computed here from the float64 position with numpy, away from
  code boundaries;
* one scan into an empty voxel gives the rational mean of the codes rounded
  half up (exact ``fractions.Fraction`` arithmetic), with the x, y, z codes
  in bits 0-9, 10-19 and 20-29;
* two scans whose first mean is an exact integer give the mean of all
  samples; a merge always stays between the smallest and largest code seen;
* counts are exact; truncated and clipped rays leave no sample; per-update
  mode with one sample per voxel and scan equals count mode.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
from workloads import scenes
from workloads.scenes import RayBatch

MP = scenes.grid_map((-1.6, -1.6, -1.6), (1.6, 1.6, 1.6), 0.1)
VOXEL = (21, 16, 16)                      # min corner (0.5, 0.0, 0.0)
VMIN = np.array([0.5, 0.0, 0.0])


def at_codes(codes, jitter=0.37):
    """Float32 points of voxel VOXEL whose code per axis is ``codes`` (the
    point sits `jitter` of a code step inside its code cell)."""
    c = np.asarray(codes, np.float64)
    pts = VMIN + (c + jitter) / 1024.0 * 0.1
    return pts.astype(np.float32)


def one_voxel(batch_samples, origins=None, offsets=None, mode=1, mp=MP):
    if origins is None:
        origins = np.array([[0.05, 0.05, 0.05]], np.float32)
        offsets = np.array([0, len(batch_samples)], np.uint32)
    b = RayBatch(origins, np.asarray(batch_samples, np.float32), offsets)
    packed, count = oracle.mean_integrate(mp, b, VOXEL, (1, 1, 1), mode=mode)
    return int(packed[0, 0, 0]), int(count[0, 0, 0])


def test_code_is_floor_of_subvoxel_position():
    rng = np.random.default_rng(1)
    pts = (VMIN + rng.uniform(0.0, 0.1, size=(400, 3))).astype(np.float32)
    frac = (pts.astype(np.float64) - VMIN) / 0.1 * 1024.0
    # the code comes from the quantised sample (1/64 code step at F = 16), so
    # points within half a quantum of a code boundary may round across it
    keep = np.all(np.abs(frac - np.round(frac)) > 0.02, axis=1)
    for p in pts[keep][:60]:
        packed, count = one_voxel([p])
        exp = np.floor((p.astype(np.float64) - VMIN) / 0.1 * 1024.0).astype(int)
        assert count == 1
        assert [(packed >> (10 * a)) & 1023 for a in range(3)] == list(exp)


@pytest.mark.parametrize("codes", [
    [[100, 7, 1000]],
    [[100, 7, 1000], [101, 8, 1001]],                      # means x.5: round half up
    [[0, 0, 0], [1, 1, 1], [1, 1, 1]],                     # 2/3 -> 1
    [[10, 500, 1023], [11, 501, 1023], [10, 500, 1022], [10, 503, 1020]],
    [[512, 3, 900]] * 9 + [[513, 4, 901]],
])
def test_single_scan_is_rounded_rational_mean(codes):
    packed, count = one_voxel(at_codes(codes))
    assert count == len(codes)
    for a in range(3):
        m = Fraction(sum(c[a] for c in codes), len(codes))
        exp = math.floor(m + Fraction(1, 2))
        assert (packed >> (10 * a)) & 1023 == exp, (a, m)
    assert packed >> 30 == 0


def test_two_scans_with_exact_first_mean():
    s1 = at_codes([[100, 20, 300], [102, 22, 306]])           # mean (101, 21, 303), exact
    s2 = at_codes([[104, 30, 301], [106, 10, 299], [98, 23, 306]])
    origins = np.array([[0.05, 0.05, 0.05], [0.06, -0.05, 0.02]], np.float32)
    packed, count = one_voxel(np.concatenate([s1, s2]), origins, np.array([0, 2, 5], np.uint32))
    allc = np.array([[100, 20, 300], [102, 22, 306], [104, 30, 301], [106, 10, 299], [98, 23, 306]])
    exp = [math.floor(Fraction(int(allc[:, a].sum()), 5) + Fraction(1, 2)) for a in range(3)]
    assert count == 5
    assert [(packed >> (10 * a)) & 1023 for a in range(3)] == exp


def test_merges_stay_within_the_codes_seen():
    rng = np.random.default_rng(7)
    n_scans, per = 12, 5
    codes = rng.integers(200, 260, size=(n_scans * per, 3))
    pts = at_codes(codes)
    origins = np.repeat(np.array([[0.05, 0.05, 0.05]], np.float32), n_scans, 0)
    offsets = (np.arange(n_scans + 1) * per).astype(np.uint32)
    for mode in (0, 1):
        packed, count = one_voxel(pts, origins, offsets, mode=mode)
        assert count == n_scans * per
        got = [(packed >> (10 * a)) & 1023 for a in range(3)]
        for a in range(3):
            assert codes[:, a].min() <= got[a] <= codes[:, a].max()
            # the rounded running mean stays near the exact mean of the codes
            assert abs(got[a] - codes[:, a].mean()) <= 3.0


def test_per_update_with_one_sample_per_scan_equals_count_mode():
    rng = np.random.default_rng(9)
    codes = rng.integers(0, 1024, size=(7, 3))
    pts = at_codes(codes)
    origins = np.repeat(np.array([[0.05, 0.05, 0.05]], np.float32), 7, 0)
    offsets = np.arange(8, dtype=np.uint32)
    assert one_voxel(pts, origins, offsets, mode=0) == one_voxel(pts, origins, offsets, mode=1)


def test_truncated_and_clipped_rays_leave_no_sample():
    p = at_codes([[500, 500, 500]])
    # truncated: max range shorter than the ray
    assert one_voxel(p, mp=MP.replace(max_range=0.3)) == (0, 0)
    # a ray whose sample lies outside the map leaves no sample anywhere
    b = RayBatch(np.array([[0.05, 0.05, 0.05]], np.float32), np.array([[3.0, 0.05, 0.05]], np.float32),
                 np.array([0, 1], np.uint32))
    packed, count = oracle.mean_integrate(MP, b)
    assert count.sum() == 0 and packed.sum() == 0


def test_whole_map_counts_equal_hits():
    mp = scenes.grid_map((-3.2, -3.2, -3.2), (3.2, 3.2, 3.2), 0.1, max_range=2.5)
    batch = scenes.random_rays(3000, 12, None, None, (0.01, 0.02, -0.03), 0.3, 3.5)
    packed, count = oracle.mean_integrate(mp, batch)
    _, hits, _, st = oracle.integrate_count(mp, batch)
    assert np.array_equal(count, hits.astype(np.uint32))
    assert int(count.sum()) == st["hits"]
    assert np.all(packed[count == 0] == 0)
