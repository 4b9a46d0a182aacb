"""Closed-form pins of two NDT-OM readings (paper Sec. II-D, III-C), through
the oracle's integrators rather than its single-voxel helper:

* the sample threshold: a voxel with exactly ``ndt_min_samples`` samples
  weights a miss by its Gaussian, one with a sample fewer takes a plain miss;
* the closest point of a truncated ray is taken on the truncated segment
  (its end at max range), not on the segment to the raw sample.

Scan 1 lays four samples at the vertices of a regular tetrahedron around a
point mu, so their population covariance is exactly a^2 I (the vertices and
mu are float32-exact dyadic values); scan 2 sends one ray past mu.  With an
isotropic covariance the quadratic form is |D|^2 / (a^2 + sigma_n^2), so the
second scan's occupancy is l1 + delta with delta written out from that
closed form.  Both the NDT integrator and the adjoint's fp64 forward are
checked, since each evaluates the miss on its own.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import scenes
from workloads.scenes import RayBatch

A = 1.0 / 64.0                        # tetrahedron half-edge: covariance a^2 I
MU = np.array([71.0, 7.0, 7.0]) / 128  # 0.5546875, 0.0546875, 0.0546875: inside voxel (21, 16, 16)
KEY = (21, 16, 16)
OFF = 3.0 / 128                        # perpendicular offset of the scan-2 ray from mu
SIGMA_N = 0.05
L_HIT, L_MISS = np.float32(0.847), np.float32(-0.405)

MP = scenes.grid_map((-1.6, -1.6, -1.6), (1.6, 1.6, 1.6), 0.1, sensor_noise=SIGMA_N, adaptation_rate=1.0,
                     ndt_min_samples=4)


def tetra(n):
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], np.float64)[:n]
    pts = MU[None, :] + A * v
    assert np.array_equal(pts.astype(np.float32).astype(np.float64), pts)
    return pts.astype(np.float32)


def logit(p):
    return math.log(p / (1.0 - p))


def delta_isotropic(d2):
    """NDT miss for an isotropic covariance a^2 I at squared distance d2."""
    g = math.exp(-0.5 * d2 / (A * A + SIGMA_N * SIGMA_N))
    s = 1.0 / (1.0 + math.exp(-float(L_MISS)))
    return logit(0.5 - 1.0 * g * (0.5 - s))


def two_scans(n_samples, scan2_sample, max_range=0.0):
    """Scan 1: n_samples tetrahedron vertices from an origin beside the voxel;
    scan 2: one ray from (-0.45, mu_y + OFF, mu_z) to scan2_sample."""
    o1 = np.array([0.05, -0.35, 0.45], np.float32)
    o2 = np.array([-0.453125, MU[1] + OFF, MU[2]], np.float32)
    s = np.concatenate([tetra(n_samples), np.asarray(scan2_sample, np.float32).reshape(1, 3)])
    batch = RayBatch(np.stack([o1, o2]), s, np.array([0, n_samples, n_samples + 1], np.uint32))
    return MP.replace(max_range=max_range), batch, o2


def ndt_occ(mp, batch):
    box_min, box_dim = KEY, (1, 1, 1)
    occ, st, _, _ = oracle.ndt_integrate(mp, batch, box_min, box_dim)
    return float(occ[0, 0, 0]), int(st.n[0, 0, 0])


def adjoint_occ(mp, batch):
    r = oracle.adjoint(mp, batch, KEY, (1, 1, 1), np.zeros(1), ndt=True, grads=False)
    return float(r["occ"][0, 0, 0])


def test_tetrahedron_has_isotropic_covariance():
    mp, batch, _ = two_scans(4, (1.05, MU[1] + OFF, MU[2]))
    _, st, _, _ = oracle.ndt_integrate(mp, batch.scans(0, 1), KEY, (1, 1, 1))
    assert st.n[0, 0, 0] == 4
    centre = np.array([-1.6 + 21.5 * 0.1, -1.6 + 16.5 * 0.1, -1.6 + 16.5 * 0.1])
    np.testing.assert_allclose(st.mu[0, 0, 0], MU - centre, atol=1e-15)
    np.testing.assert_allclose(st.cov[0, 0, 0], [A * A, 0, 0, A * A, 0, A * A], atol=1e-18)


@pytest.mark.parametrize("occ_of", [ndt_occ, adjoint_occ], ids=["ndt_integrate", "adjoint_forward"])
@pytest.mark.parametrize("n_samples", [3, 4])
def test_sample_threshold_boundary(occ_of, n_samples):
    """N_min = 4 samples: the Gaussian weights the miss; 3: a plain miss."""
    mp, batch, _ = two_scans(n_samples, (1.05, MU[1] + OFF, MU[2]))
    l1 = n_samples * float(L_HIT)              # scan 1: hits only (below l_max)
    got = occ_of(mp, batch)
    got = got[0] if isinstance(got, tuple) else got
    d = delta_isotropic(OFF * OFF) if n_samples >= 4 else float(L_MISS)
    assert abs(got - (l1 + d)) < 1e-6
    # the two cases differ by far more than the tolerance
    assert abs(delta_isotropic(OFF * OFF) - float(L_MISS)) > 0.03


@pytest.mark.parametrize("occ_of", [ndt_occ, adjoint_occ], ids=["ndt_integrate", "adjoint_forward"])
def test_truncated_ray_uses_segment_end(occ_of):
    """Scan 2's raw sample lies 1.5 m beyond mu, but max range cuts the ray at
    x = -0.453125 + 0.97 = 0.516875, inside the sample voxel and before mu:
    the closest point is that end, D = (0.516875 - mu_x, OFF, 0)."""
    mp, batch, o2 = two_scans(4, (2.05, MU[1] + OFF, MU[2]), max_range=0.97)
    end_x = float(o2[0]) + 0.97
    assert 0.5 <= end_x < MU[0]
    l1 = 4 * float(L_HIT)
    got = occ_of(mp, batch)
    got = got[0] if isinstance(got, tuple) else got
    d_trunc = delta_isotropic((end_x - MU[0]) ** 2 + OFF * OFF)
    d_raw = delta_isotropic(OFF * OFF)
    assert abs(got - (l1 + d_trunc)) < 1e-6
    assert abs(d_trunc - d_raw) > 1e-3


def test_cross_scan_occupancy_is_float_of_clamped_sum():
    """The NDT integrator stores occupancy as float32 after every scan: scan 2
    gives float32(clamp(float32(l1) + delta)) exactly (count mode)."""
    mp, batch, _ = two_scans(4, (1.05, MU[1] + OFF, MU[2]))
    got, n = ndt_occ(mp, batch)
    l1 = float(np.float32(4 * float(L_HIT)))
    exp = float(np.float32(min(max(l1 + delta_isotropic(OFF * OFF), -2.0), 3.5)))
    assert n == 4 and got == exp
