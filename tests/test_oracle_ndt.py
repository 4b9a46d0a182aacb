"""Pins for the oracle's NDT-OM path (paper Sec. II-D, III-C): closed forms of
the NDT-weighted miss, the quadratic form against numpy.linalg.solve, the
sample statistics against numpy.mean / numpy.cov(bias=True), and reduction to
the plain occupancy oracle when no voxel holds samples yet."""
import math

import numpy as np
import pytest

import oracle
from bruteforce import sequential_clamp
from workloads import scenes
from workloads.scenes import RayBatch


def f32(v):
    return float(np.float32(v))


def logit(p):
    return math.log(p / (1.0 - p))


def sig(x):
    return 1.0 / (1.0 + math.exp(-x))


MP = scenes.grid_map((-1.6, -1.6, -1.6), (1.6, 1.6, 1.6), 0.1, sensor_noise=0.05, adaptation_rate=1.0,
                     ndt_min_samples=4)


def test_miss_through_mean_is_plain_miss():
    d = oracle.ndt_miss_delta(MP, [0, 0, 0], [1.0, 0.2, -0.1], [0.5, 0.1, -0.05],
                              [0.002, 0.0003, 0.0, 0.001, 0.0001, 0.003], 9)
    assert abs(d - f32(-0.405)) < 1e-12


def test_zero_adaptation_gives_zero_miss():
    mp = MP.replace(adaptation_rate=0.0)
    d = oracle.ndt_miss_delta(mp, [0, 0, 0], [1, 0, 0], [0.3, 0.02, 0.0], [0.001, 0, 0, 0.001, 0, 0.001], 9)
    assert abs(d) < 1e-12


def test_too_few_samples_gives_plain_miss():
    d = oracle.ndt_miss_delta(MP, [0, 0, 0], [1, 0, 0], [0.3, 0.5, 0.0], [0.001, 0, 0, 0.001, 0, 0.001], 3)
    assert d == f32(-0.405)


@pytest.mark.parametrize("c,off", [(0.001, 0.03), (0.0004, 0.08), (0.01, 0.2)])
def test_isotropic_closed_form(c, off):
    """Sigma = c I and a perpendicular offset: D^T S^-1 D = off^2 / (c + s^2)."""
    g = math.exp(-0.5 * off * off / (c + 0.05 ** 2))
    exp = logit(0.5 - 1.0 * g * (0.5 - sig(f32(-0.405))))
    d = oracle.ndt_miss_delta(MP, [0, 0, 0], [1, 0, 0], [0.4, off, 0.0], [c, 0, 0, c, 0, c], 12)
    assert abs(d - exp) < 1e-12


@pytest.mark.parametrize("t_case", ["before", "inside", "after"])
def test_closest_point_and_anisotropic_form(t_case):
    """Anisotropic covariance against numpy.linalg.solve, with the closest
    point clamped to the segment ends."""
    rng = np.random.default_rng(4)
    A = rng.normal(size=(3, 3)) * 0.03
    cov = A @ A.T + np.eye(3) * 1e-4
    cov6 = [cov[0, 0], cov[0, 1], cov[0, 2], cov[1, 1], cov[1, 2], cov[2, 2]]
    o = np.array([0.1, -0.2, 0.05])
    e = np.array([0.9, 0.4, -0.3])
    mu = {"before": o - 0.2 * (e - o) + np.array([0.0, 0.01, 0.02]),
          "inside": o + 0.6 * (e - o) + np.array([0.01, -0.02, 0.01]),
          "after": e + 0.3 * (e - o) + np.array([0.02, 0.0, -0.01])}[t_case]
    t = np.clip(np.dot(mu - o, e - o) / np.dot(e - o, e - o), 0.0, 1.0)
    assert (t == 0.0) == (t_case == "before") and (t == 1.0) == (t_case == "after")
    D = o + t * (e - o) - mu
    S = cov + np.eye(3) * 0.05 ** 2
    q = float(D @ np.linalg.solve(S, D))
    exp = logit(0.5 - math.exp(-0.5 * q) * (0.5 - sig(f32(-0.405))))
    d = oracle.ndt_miss_delta(MP, o, e, mu, cov6, 20)
    assert abs(d - exp) < 1e-10


def _cluster_rays(rng, n, target, spread, origin=(0.0, 0.0, 0.0)):
    pts = (np.asarray(target) + rng.normal(scale=spread, size=(n, 3))).astype(np.float32)
    return pts


def test_welford_matches_numpy_across_scans():
    rng = np.random.default_rng(8)
    # all samples inside voxel (21, 19, 17) of MP: centre (0.55, 0.35, 0.15)
    s1 = _cluster_rays(rng, 40, (0.55, 0.35, 0.15), 0.012)
    s2 = _cluster_rays(rng, 25, (0.55, 0.35, 0.15), 0.012)
    allp = np.concatenate([s1, s2])
    key = np.floor((allp.astype(np.float64) + 1.6) / 0.1).astype(int)
    keep1 = np.all(key[:40] == (21, 19, 17), axis=1)
    keep2 = np.all(key[40:] == (21, 19, 17), axis=1)
    s1, s2 = s1[keep1], s2[keep2]
    o = np.array([[0.02, 0.03, 0.01], [0.05, -0.02, 0.0]], np.float32)
    batch = RayBatch(o, np.concatenate([s1, s2]), np.array([0, len(s1), len(s1) + len(s2)], np.uint32))
    occ, st, _, _ = oracle.ndt_integrate(MP, batch)
    n = st.n[17, 19, 21]
    assert n == len(s1) + len(s2)
    x = np.concatenate([s1, s2]).astype(np.float64) - np.array([0.55, 0.35, 0.15])
    np.testing.assert_allclose(st.mu[17, 19, 21], x.mean(axis=0), atol=1e-12)
    C = np.cov(x.T, bias=True)
    cov6 = st.cov[17, 19, 21]
    full = np.array([[cov6[0], cov6[1], cov6[2]], [cov6[1], cov6[3], cov6[4]], [cov6[2], cov6[4], cov6[5]]])
    np.testing.assert_allclose(full, C, atol=1e-12)
    assert np.linalg.eigvalsh(full).min() >= -1e-15


def test_first_scan_equals_plain_oracle():
    """With no samples in any voxel every NDT miss is a plain miss, so the
    first scan's occupancy equals the plain count-then-clamp oracle."""
    mp = scenes.grid_map((-3.2, -3.2, -3.2), (3.2, 3.2, 3.2), 0.1, max_range=2.5)
    batch = scenes.random_rays(3000, 12, None, None, (0.01, 0.02, -0.03), 0.3, 3.5)
    occ_n, st, _, stn = oracle.ndt_integrate(mp, batch)
    occ_p, hits, _, stp = oracle.integrate_count(mp, batch)
    np.testing.assert_allclose(occ_n, occ_p, atol=1e-6, rtol=0)
    assert stn == stp
    # every hit left one sample
    assert int(st.n.sum()) == int(hits.sum()) == stp["hits"]


def test_per_update_mode_is_misses_then_hits():
    """Two-phase per-update semantics: a voxel's misses land first, then its
    hits, each clamped; compare with the sequential brute force."""
    mp = scenes.grid_map((-1.6, -1.6, -1.6), (1.6, 1.6, 1.6), 0.1, l_min=-0.9, l_max=1.2)
    o = np.array([[0.05, 0.05, 0.05]], np.float32)
    hit = np.array([[0.55, 0.05, 0.05]], np.float32)        # ends in voxel (21, 16, 16)
    through = np.array([[0.95, 0.05, 0.05]], np.float32)    # passes through it
    samples = np.concatenate([np.repeat(hit, 2, 0), np.repeat(through, 4, 0)])
    batch = RayBatch(o, samples, np.array([0, 6], np.uint32))
    occ, _, _, _ = oracle.ndt_integrate(mp, batch, mode=0)
    exp = sequential_clamp(0.0, [f32(-0.405)] * 4 + [f32(0.847)] * 2, f32(-0.9), f32(1.2))
    assert abs(occ[16, 16, 21] - exp) < 1e-6
    occ_c, _, _, _ = oracle.ndt_integrate(mp, batch, mode=1)
    assert abs(occ_c[16, 16, 21] - min(max(2 * f32(0.847) + 4 * f32(-0.405), f32(-0.9)), f32(1.2))) < 1e-6


def test_clearing_threshold_drops_statistics():
    mp = MP.replace(ndt_clear_below=-0.5)
    rng = np.random.default_rng(3)
    s1 = _cluster_rays(rng, 6, (0.55, 0.05, 0.05), 0.005)
    o = np.array([[0.05, 0.05, 0.05]], np.float32)
    through = np.array([[0.95, 0.05, 0.05]], np.float32)
    # scan 1: samples land (l saturates at 3.5); scan 2: 16 rays pass
    # through the samples' mean (plain misses) -> l = max(3.5 - 16 * 0.405, -2) < -0.5
    batch = RayBatch(np.concatenate([o, o]), np.concatenate([s1, np.repeat(through, 16, 0)]),
                     np.array([0, 6, 22], np.uint32))
    _, st, _, _ = oracle.ndt_integrate(mp, batch.scans(0, 1))
    assert st.n[16, 16, 21] == 6
    occ, st2, _, _ = oracle.ndt_integrate(mp, batch)
    assert occ[16, 16, 21] < -0.5 and st2.n[16, 16, 21] == 0
