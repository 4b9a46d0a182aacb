"""Pins of the oracle's TSDF (paper Sec. II-F: a projective distance in a
band of one truncation distance in front of and behind the measured point,
along the sensor ray; Sec. III-B: per-update by 64-bit compare-and-swap).

Readings pinned: only rays with a surface (a hit under the occupancy rules)
update; the band is the segment from max(r - tau, 0) to r + tau along the
ray, walked exactly from its quantised ends; each band voxel takes
clamp(r - (c - o).u, -tau, tau); a voxel's distance is the running weighted
mean with unit weight per update, its weight capped at tsdf_max_weight.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from bruteforce import segment_voxels
from workloads import scenes
from workloads.scenes import RayBatch

TAU = 0.3
MP = scenes.grid_map((-3.2, -3.2, -3.2), (3.2, 3.2, 3.2), 0.1, tsdf_truncation=TAU, tsdf_max_weight=10000.0)


def one_ray(o, e):
    return RayBatch(np.asarray(o, np.float32).reshape(1, 3), np.asarray(e, np.float32).reshape(1, 3),
                    np.array([0, 1], np.uint32))


def test_axis_aligned_band_closed_form():
    """A ray along +x from a voxel corner to x = 1.23: band x in [0.93, 1.53],
    so keys 41..47 along x (map origin -3.2: key = floor((x + 3.2) / 0.1)),
    each with sdf = 1.23 - (centre - 0) clamped to 0.3."""
    o, e = (0.0, 0.05, 0.05), (1.23, 0.05, 0.05)
    d, w, st = oracle.tsdf_integrate(MP, one_ray(o, e))
    ky = kz = 32
    xs = np.nonzero(w[kz, ky])[0]
    x0 = math.floor((float(np.float32(1.23)) - TAU + 3.2) / 0.1)
    x1 = math.floor((float(np.float32(1.23)) + TAU + 3.2) / 0.1)
    assert list(xs) == list(range(x0, x1 + 1)) and (x0, x1) == (41, 47)
    assert int(w.sum()) == x1 - x0 + 1 == st["updates"]
    r = float(np.float32(1.23))
    for k in xs:
        c = -3.2 + (k + 0.5) * 0.1
        assert abs(d[kz, ky, k] - float(np.float32(min(max(r - c, -TAU), TAU)))) <= 1e-7


def test_short_ray_band_starts_at_origin():
    """r < tau: the band starts at the sensor."""
    o, e = (0.05, 0.05, 0.05), (0.25, 0.05, 0.05)
    d, w, _ = oracle.tsdf_integrate(MP, one_ray(o, e))
    xs = np.nonzero(w[32, 32])[0]
    assert xs[0] == 32 and xs[-1] == math.floor((0.25 + TAU + 3.2) / 0.1)


def test_rays_without_surface_do_not_update():
    """Truncated (max range), clipped (sample outside the map), zero-length
    and invalid rays leave the TSDF untouched."""
    rays = [((0.0, 0.0, 0.0), (2.5, 0.0, 0.0)),   # truncated by max range 2
            ((0.0, 0.0, 0.0), (0.0, 5.0, 0.0)),   # sample outside the map
            ((0.1, 0.1, 0.1), (0.1, 0.1, 0.1))]   # zero length
    for o, e in rays:
        d, w, st = oracle.tsdf_integrate(MP.replace(max_range=2.0), one_ray(o, e))
        assert not w.any() and not d.any() and st["updates"] == 0 and st["hits"] == 0


def _band_ends_fp64(o, e, tau, mp):
    """The band's quantised ends, computed here in numpy fp64 (the reading's
    formulas, written independently of the oracle)."""
    o64, e64 = np.asarray(o, np.float64), np.asarray(e, np.float64)
    d = e64 - o64
    r = math.sqrt(float(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]))
    u = d / r
    b0 = o64 + max(r - tau, 0.0) * u
    b1 = o64 + (r + tau) * u
    scale = 2.0 ** mp.fixed_bits / mp.voxel_size
    q0 = [int(np.rint((b0[a] - mp.map_origin[a]) * scale)) for a in range(3)]
    q1 = [int(np.rint((b1[a] - mp.map_origin[a]) * scale)) for a in range(3)]
    return q0, q1, r, u


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_band_voxels_and_distances_brute_force(seed):
    """Single rays in general position: the updated voxels are exactly the
    voxels an exact-rational search finds on the quantised band (half-open
    boxes), and each holds clamp(r - (c - o).u) computed here."""
    rng = np.random.default_rng(seed)
    mp = MP.replace(voxel_size=0.1)
    for _ in range(25):
        o = rng.uniform(-0.5, 0.5, 3).astype(np.float32)
        dirv = rng.normal(size=3)
        e = (o + dirv / np.linalg.norm(dirv) * rng.uniform(0.1, 2.0)).astype(np.float32)
        d, w, _ = oracle.tsdf_integrate(mp, one_ray(o, e))
        q0, q1, r, u = _band_ends_fp64(o, e, TAU, mp)
        want = segment_voxels(q0, q1, mp.fixed_bits, "halfopen")
        got = {(int(x), int(y), int(z)) for z, y, x in zip(*np.nonzero(w))}
        assert got == want
        for kx, ky, kz in got:
            c = np.array(mp.map_origin) + (np.array([kx, ky, kz]) + 0.5) * mp.voxel_size
            sd = min(max(r - float(np.dot(c - o.astype(np.float64), u)), -TAU), TAU)
            assert abs(d[kz, ky, kx] - sd) <= 2e-7 and w[kz, ky, kx] == 1.0


def test_running_mean_and_weight_cap():
    """One voxel observed by several scans: D is the mean of the clamped
    distances while W is below the cap; beyond it, D is the weighted mean
    with the capped weight: W=2 cap, three observations d1, d2, d3 give
    D = ((d1 + d2) / 2 * 2 + d3) / 3, W = 2 (rational arithmetic)."""
    mp = MP.replace(tsdf_max_weight=2.0)
    samples = [(1.23, 0.05, 0.05), (1.26, 0.05, 0.05), (1.31, 0.05, 0.05)]
    origin = (0.0, 0.05, 0.05)
    batch = RayBatch(np.tile(np.asarray(origin, np.float32), (3, 1)), np.asarray(samples, np.float32),
                     np.array([0, 1, 2, 3], np.uint32))
    d, w, _ = oracle.tsdf_integrate(mp, batch)
    k = 43  # centre x = 1.15: inside every band
    c = Fraction(-32, 10) + Fraction(2 * k + 1, 20)
    ds = [min(max(Fraction(float(np.float32(s[0]))) - c, Fraction(-3, 10)), Fraction(3, 10)) for s in samples]
    D1 = ds[0]
    D2 = (D1 * 1 + ds[1]) / 2
    D3 = (D2 * 2 + ds[2]) / 3
    assert abs(d[32, 32, k] - float(D3)) <= 1e-7 and w[32, 32, k] == 2.0
    # the same three rays in one scan: one application of the sum, W capped after
    one = RayBatch(np.asarray(origin, np.float32).reshape(1, 3), np.asarray(samples, np.float32),
                   np.array([0, 3], np.uint32))
    d1, w1, _ = oracle.tsdf_integrate(mp, one)
    assert abs(d1[32, 32, k] - float(sum(ds) / 3)) <= 1e-7 and w1[32, 32, k] == 2.0


def test_count_and_per_update_agree_without_cap():
    """With the cap out of reach, the running mean does not depend on how the
    updates are grouped: count mode and per-update mode agree to rounding."""
    rng = np.random.default_rng(7)
    o = np.zeros((2, 3), np.float32)
    dirs = rng.normal(size=(4000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    s = (dirs * rng.uniform(0.5, 2.5, (4000, 1))).astype(np.float32)
    batch = RayBatch(o, s, np.array([0, 2000, 4000], np.uint32))
    d1, w1, st1 = oracle.tsdf_integrate(MP, batch, mode=1)
    d0, w0, st0 = oracle.tsdf_integrate(MP, batch, mode=0)
    assert st1 == st0 and st1["updates"] > 10000
    np.testing.assert_array_equal(w1, w0)
    assert np.max(np.abs(d1 - d0)) <= 1e-6
    assert w1.max() > 3
