"""Pins of the oracle's NDT-TM (paper Sec. II-D, III-C): the checked miss
count M behind a voxel's permeability H / (H + M), and the 1D Gaussian of
sample intensity.

Readings pinned here: a miss counts toward M only where the voxel holds at
least ``ndt_min_samples`` samples (so the check has a Gaussian to test the
ray against) and the ray's closest point lies within the squared
Mahalanobis distance ``ndt_tm_gate`` of it, measured on the (truncated) ray
segment with the statistics from before the scan; H is the voxel's sample
count; the intensity mean and variance are the population statistics of the
samples' intensities.

The closed forms use the regular-tetrahedron voxel of the NDT-OM pins
(covariance a^2 I), where q = |D|^2 / (a^2 + sigma_n^2).
"""
import numpy as np
import pytest

import oracle
from workloads import scenes
from workloads.scenes import RayBatch

A = 1.0 / 64.0
MU = np.array([71.0, 7.0, 7.0]) / 128  # inside voxel (21, 16, 16) of the 3.2 m map below
KEY = (21, 16, 16)
SIGMA_N = 0.05
VAR = A * A + SIGMA_N * SIGMA_N  # isotropic S

MP = scenes.grid_map((-1.6, -1.6, -1.6), (1.6, 1.6, 1.6), 0.1, sensor_noise=SIGMA_N, adaptation_rate=1.0,
                     ndt_min_samples=4)


def tetra(n):
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], np.float64)[:n]
    return (MU[None, :] + A * v).astype(np.float32)


def scans(n_samples, offsets, end_x=1.05):
    """Scan 1 lays n_samples tetrahedron vertices; then one single-ray scan
    per (dy, dz) offset, each ray parallel to x from x = -0.453125 past mu at
    that offset (every scan has one origin, so parallel rays take a scan
    each)."""
    o1 = np.array([0.05, -0.35, 0.45], np.float32)
    origins = [o1]
    samples = [tetra(n_samples)]
    offs = [0, n_samples]
    for dy, dz in offsets:
        o = np.array([-0.453125, MU[1] + dy, MU[2] + dz], np.float32)
        origins.append(o)
        samples.append(np.array([[end_x, MU[1] + dy, MU[2] + dz]], np.float32))
        offs.append(offs[-1] + 1)
    return RayBatch(np.stack(origins), np.concatenate(samples), np.array(offs, np.uint32))


def run(mp, batch, intens=None, box_min=KEY, box_dim=(1, 1, 1)):
    inten = np.zeros(batch.n_rays, np.float32) if intens is None else intens
    return oracle.ndt_tm_integrate(mp, batch, inten, box_min, box_dim)


# offsets (dy, dz) in metres from mu; all stay inside the voxel's y/z extent
OFFSETS = [(0.0, 0.0), (0.01, 0.0), (0.03, 0.03), (-0.03, 0.02), (0.04, 0.04), (-0.045, -0.045), (0.0, -0.05)]


@pytest.mark.parametrize("gate", [0.25, 1.0, 1.3, 9.0])
def test_checked_miss_count_isotropic_closed_form(gate):
    mp = MP.replace(ndt_tm_gate=gate)
    batch = scans(4, OFFSETS)
    _, st, _ = run(mp, batch)
    # scan 1 has no earlier samples: none of its misses counts; each later
    # ray passes the voxel once, at perpendicular distance r from mu
    expect = sum(1 for dy, dz in OFFSETS if (dy * dy + dz * dz) / VAR <= gate)
    assert 0 < expect < len(OFFSETS) or gate >= 9.0
    assert int(st.miss[0, 0, 0]) == expect
    assert int(st.near[0, 0, 0]) == 0
    assert int(st.n[0, 0, 0]) == 4


def test_no_count_below_sample_threshold():
    """Three samples: no Gaussian, so no ray is checked and none counts,
    even one straight through mu."""
    mp = MP.replace(ndt_tm_gate=9.0)
    _, st, _ = run(mp, scans(3, OFFSETS[:3]))
    assert int(st.miss[0, 0, 0]) == 0 and int(st.n[0, 0, 0]) == 3


def test_check_uses_truncated_segment_end():
    """A ray cut by max range ends before mu (x = 0.516875 < mu_x): its closest
    point is the truncated end.  With gate 0.5 the raw segment would count
    (q = OFF^2 / var = 0.20) but the truncated one does not (q = 0.72)."""
    off = 3.0 / 128
    mp = MP.replace(ndt_tm_gate=0.5, max_range=0.97)
    batch = scans(4, [(off, 0.0)], end_x=2.05)
    end_x = -0.453125 + 0.97
    q_trunc = ((end_x - MU[0]) ** 2 + off * off) / VAR
    q_raw = off * off / VAR
    assert q_raw < 0.5 < q_trunc
    _, st, _ = run(mp, batch)
    assert int(st.miss[0, 0, 0]) == 0
    _, st, _ = run(mp.replace(ndt_tm_gate=q_trunc * 1.001), batch)
    assert int(st.miss[0, 0, 0]) == 1


def test_closest_q_matches_linear_solve():
    """The check's q against numpy's solve of S y = D for anisotropic
    covariances (a textbook routine in place of the oracle's Cholesky)."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        B = rng.normal(size=(3, 3)) * 0.05
        cov = B @ B.T
        cov6 = np.array([cov[0, 0], cov[0, 1], cov[0, 2], cov[1, 1], cov[1, 2], cov[2, 2]])
        o, e, mu = rng.normal(size=3), rng.normal(size=3), rng.normal(size=3) * 0.3
        d = e - o
        t = np.clip(np.dot(mu - o, d) / np.dot(d, d), 0.0, 1.0)
        D = o + t * d - mu
        S = cov + SIGMA_N ** 2 * np.eye(3)
        q = float(D @ np.linalg.solve(S, D))
        got = oracle.ndt_closest_q(MP, o, e, mu, cov6)
        assert abs(got - q) <= 1e-9 * max(1.0, q)


def _random_case(seed, n_scans=3, n_rays=400):
    mp = scenes.grid_map((-0.8, -0.8, -0.8), (0.8, 0.8, 0.8), 0.2, sensor_noise=0.05, adaptation_rate=1.0,
                         ndt_min_samples=4, ndt_tm_gate=4.0)
    rng = np.random.default_rng(seed)
    origins, samples = [], []
    for k in range(n_scans):
        o = rng.uniform(-0.1, 0.1, 3).astype(np.float32)
        # samples clustered around a few points so voxels collect >= 4 samples
        centres = rng.uniform(-0.6, 0.6, (6, 3))
        pts = centres[rng.integers(0, 6, n_rays)] + rng.normal(scale=0.04, size=(n_rays, 3))
        origins.append(o)
        samples.append(pts.astype(np.float32))
    batch = RayBatch(np.stack(origins), np.concatenate(samples), np.arange(0, n_rays * (n_scans + 1), n_rays,
                                                                             dtype=np.uint32))
    inten = rng.uniform(0.0, 255.0, batch.n_rays).astype(np.float32)
    return mp, batch, inten


@pytest.mark.parametrize("seed", [1, 2])
def test_checked_misses_brute_force(seed):
    """M over every voxel of a random three-scan case, recounted from the
    per-ray walk lists with q from a linear solve against the statistics of
    the scans before (taken from the NDT-OM integrator, pinned elsewhere)."""
    mp, batch, inten = _random_case(seed)
    box_min, box_dim = mp.key_min, tuple(b - a for a, b in zip(mp.key_min, mp.key_max))
    _, st, _ = run(mp, batch, inten, box_min, box_dim)
    expect = np.zeros_like(st.miss)
    cov_s = mp.sensor_noise ** 2 * np.eye(3)
    for k in range(batch.n_scans):
        prev = batch.scans(0, k)
        _, pst, _, _ = oracle.ndt_integrate(mp, prev, box_min, box_dim) if k else (None, None, None, None)
        scan = batch.scans(k, 1)
        counts, flags, offs, upd = oracle.trace(mp, scan)
        o = scan.origins[0].astype(np.float64)
        for r in range(scan.n_rays):
            rows = upd[offs[r]:offs[r + 1]]
            if k == 0:
                continue
            e = scan.samples[r].astype(np.float64)
            if flags[r] & oracle.F_TRUNCATED:
                d = e - o
                e = o + d * (mp.max_range / np.linalg.norm(d))
            for kx, ky, kz, kind in rows:
                if kind != 0:
                    continue
                iz, iy, ix = kz - box_min[2], ky - box_min[1], kx - box_min[0]
                if pst.n[iz, iy, ix] < mp.ndt_min_samples:
                    continue
                c = np.array(mp.map_origin) + (np.array([kx, ky, kz]) + 0.5) * mp.voxel_size
                mu = c + pst.mu[iz, iy, ix]
                cv = pst.cov[iz, iy, ix]
                S = np.array([[cv[0], cv[1], cv[2]], [cv[1], cv[3], cv[4]], [cv[2], cv[4], cv[5]]]) + cov_s
                d = e - o
                t = np.clip(np.dot(mu - o, d) / np.dot(d, d), 0.0, 1.0)
                D = o + t * d - mu
                if D @ np.linalg.solve(S, D) <= mp.ndt_tm_gate:
                    expect[iz, iy, ix] += 1
    assert int(expect.sum()) > 20
    assert int(st.near.sum()) == 0
    np.testing.assert_array_equal(st.miss, expect)


@pytest.mark.parametrize("seed", [1, 2])
def test_intensity_gaussian_and_shared_state(seed):
    """Intensity mean and variance equal numpy's mean and var(ddof=0) of the
    intensities of each voxel's samples; occupancy and the position
    statistics equal the NDT-OM integrator's bit for bit; permeability is
    n / (n + M)."""
    mp, batch, inten = _random_case(seed)
    box_min, box_dim = mp.key_min, tuple(b - a for a, b in zip(mp.key_min, mp.key_max))
    occ, st, _ = run(mp, batch, inten, box_min, box_dim)
    occ2, st2, _, _ = oracle.ndt_integrate(mp, batch, box_min, box_dim)
    np.testing.assert_array_equal(occ, occ2)
    np.testing.assert_array_equal(st.n, st2.n)
    np.testing.assert_array_equal(st.mu, st2.mu)
    np.testing.assert_array_equal(st.cov, st2.cov)
    counts, flags, offs, upd = oracle.trace(mp, batch)
    per_voxel = {}
    for r in range(batch.n_rays):
        if not flags[r] & oracle.F_HAS_HIT:
            continue
        kx, ky, kz, kind = upd[offs[r + 1] - 1]
        assert kind == 1
        per_voxel.setdefault((kz - box_min[2], ky - box_min[1], kx - box_min[0]), []).append(inten[r])
    assert len(per_voxel) > 5
    for idx, vals in per_voxel.items():
        v = np.asarray(vals, np.float64)
        assert st.n[idx] == len(v)
        assert abs(st.in_mean[idx] - v.mean()) <= 1e-9 * max(1.0, abs(v.mean()))
        assert abs(st.in_var[idx] - v.var()) <= 1e-9 * max(1.0, v.var())
    perm = st.permeability()
    tot = st.n.astype(np.float64) + st.miss
    nz = tot > 0
    np.testing.assert_allclose(perm[nz], st.n[nz] / tot[nz], rtol=0, atol=0)
    assert np.all(perm[~nz] == 0.0)


def test_clearing_resets_tm_state():
    """A voxel whose occupancy falls below ndt_clear_below loses M and its
    intensity Gaussian with its position statistics."""
    mp = MP.replace(ndt_tm_gate=9.0, ndt_clear_below=-0.6)
    # scan 1: 4 samples (l = 4 * 0.847); scans 2..k: rays through mu lower it
    # by |l_miss| each (ray through mu: delta = l_miss); clearing engages once
    # l < -0.6, i.e. after 10 misses (3.388 - 10 * 0.405 = -0.662)
    batch = scans(4, [(0.0, 0.0)] * 10)
    inten = np.full(batch.n_rays, 100.0, np.float32)
    _, st, _ = run(mp, batch, inten)
    assert int(st.n[0, 0, 0]) == 0 and int(st.miss[0, 0, 0]) == 0
    assert st.in_mean[0, 0, 0] == 0.0 and st.in_var[0, 0, 0] == 0.0
    _, st9, _ = run(mp, scans(4, [(0.0, 0.0)] * 9), inten[:13])
    assert int(st9.n[0, 0, 0]) == 4 and int(st9.miss[0, 0, 0]) == 9 and st9.in_mean[0, 0, 0] == 100.0
