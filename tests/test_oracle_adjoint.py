"""Pins for the oracle's adjoint (gradients of a BCE loss on final log-odds with
respect to l_hit, l_miss, sensor noise and per-ray weights): every analytic
gradient is checked against fp64 central finite differences of the oracle's
own forward, away from clamp switches; plus exact closed forms."""
import numpy as np
import pytest

import oracle
from workloads import scenes
from workloads.scenes import RayBatch


def wall_scene(n_scans=3, n_rays=1500, seed=0):
    """Rays from a sensor moving along x towards a 1.2 m x 1.2 m wall patch at
    x = 2 m with 5 cm range noise, so wall voxels collect samples and later
    rays pass through them."""
    rng = np.random.default_rng(seed)
    origins, chunks, offs = [], [], [0]
    for k in range(n_scans):
        o = np.array([0.1 * k - 0.05, 0.02, -0.03])
        tgt = np.stack([np.full(n_rays, 2.0), rng.uniform(-0.6, 0.6, n_rays), rng.uniform(-0.6, 0.6, n_rays)], 1)
        d = tgt - o
        rng_len = np.linalg.norm(d, axis=1)
        d /= rng_len[:, None]
        r = rng_len + rng.normal(0, 0.05, n_rays)
        chunks.append((o + d * r[:, None]).astype(np.float32))
        origins.append(o.astype(np.float32))
        offs.append(offs[-1] + n_rays)
    batch = RayBatch(np.asarray(origins), np.concatenate(chunks), np.asarray(offs, np.uint32))
    batch.weights = rng.uniform(0.5, 1.0, batch.n_rays).astype(np.float32)
    return batch


MP = scenes.grid_map((-1.6, -1.6, -1.6), (3.2, 1.6, 1.6), 0.1, l_min=-2.0, l_max=3.5,
                     sensor_noise=0.05, adaptation_rate=1.0, ndt_min_samples=4)
BOX_MIN, BOX_DIM = (0, 0, 0), MP.dims


def labels_for(mp):
    # occupied beyond x = 1.95 m, free before
    x = mp.map_origin[0] + (np.arange(BOX_DIM[0]) + 0.5) * mp.voxel_size
    y = np.zeros((BOX_DIM[2], BOX_DIM[1], BOX_DIM[0]))
    y[:, :, x > 1.95] = 1.0
    return y


def loss_at(mp, batch, labels, mask, ndt=True):
    return oracle.adjoint(mp, batch, BOX_MIN, BOX_DIM, labels, mask, ndt=ndt, grads=False)


def central_fd(f, theta, h):
    return (f(theta + h) - f(theta - h)) / (2 * h)


def rel_ok(g, g_fd, scale):
    return abs(g - g_fd) <= 1e-4 * max(abs(g_fd), 1e-8 * scale) + 1e-9


@pytest.fixture(scope="module")
def setup():
    batch = wall_scene()
    labels = labels_for(MP)
    first = oracle.adjoint(MP, batch, BOX_MIN, BOX_DIM, labels, None, ndt=True, grads=False)
    mask = (first["near"] == 0).astype(np.float64)
    ref = oracle.adjoint(MP, batch, BOX_MIN, BOX_DIM, labels, mask, ndt=True, grads=True)
    return batch, labels, mask, ref


def test_ndt_weighting_is_exercised(setup):
    batch, labels, mask, ref = setup
    assert abs(ref["grad_scalars"][2]) > 0.0       # d/d sensor_noise needs NDT-weighted misses
    assert (ref["clamp_last"] > 0).sum() > 10       # some clamps engaged
    assert mask.mean() > 0.5


@pytest.mark.parametrize("idx,name", [(0, "l_hit"), (1, "l_miss"), (2, "sensor_noise")])
def test_scalar_gradients_match_fd(setup, idx, name):
    batch, labels, mask, ref = setup
    theta = getattr(MP, name)
    h = 1e-5 * max(1.0, abs(theta))
    # l_hit / l_miss are float32 parameters: step between representable values
    tp, tm = (float(np.float32(theta + h)), float(np.float32(theta - h))) if idx < 2 else (theta + h, theta - h)

    def f(t):
        return loss_at(MP.replace(**{name: t}), batch, labels, mask)

    lo, hi = f(tm), f(tp)
    assert np.array_equal(lo["clamp_last"], hi["clamp_last"])
    g_fd = (hi["loss"] - lo["loss"]) / (tp - tm)
    g = ref["grad_scalars"][idx]
    assert rel_ok(g, g_fd, abs(g_fd)), (g, g_fd)


def test_weight_gradients_match_fd(setup):
    batch, labels, mask, ref = setup
    rng = np.random.default_rng(11)
    gw = ref["grad_w"]
    scale = np.abs(gw).max()
    checked = 0
    for i in rng.choice(batch.n_rays, 40, replace=False):
        w0 = float(batch.weights[i])
        h = 1e-4  # one weight moves the loss by ~1e-8 h^-1: keep roundoff small

        def f(wv):
            b = RayBatch(batch.origins, batch.samples, batch.offsets, batch.weights.copy())
            b.weights[i] = np.float32(wv)
            return loss_at(MP, b, labels, mask)

        # perturb in the weight's float32 representation: use the exact
        # difference of the stored values
        wp, wm = np.float32(w0 + h), np.float32(w0 - h)
        fp, fm = f(float(wp)), f(float(wm))
        if not np.array_equal(fp["clamp_last"], fm["clamp_last"]):
            continue
        g_fd = (fp["loss"] - fm["loss"]) / (float(wp) - float(wm))
        assert rel_ok(gw[i], g_fd, scale) or abs(gw[i] - g_fd) < 1e-6 * scale, (i, gw[i], g_fd)
        checked += 1
    assert checked >= 30


def test_plain_model_closed_forms():
    """Without NDT: d/d sensor_noise = 0 exactly, and with no clamp engaged
    d/d l_hit = sum_r w_r G_hit(r) -- the loss is linear in l_hit per voxel."""
    batch = wall_scene(n_scans=2, n_rays=400, seed=3)
    mp = MP.replace(l_min=-1e6, l_max=1e6)
    labels = labels_for(mp)
    ref = oracle.adjoint(mp, batch, BOX_MIN, BOX_DIM, labels, None, ndt=False, grads=True)
    assert ref["grad_scalars"][2] == 0.0
    assert (ref["clamp_last"] == 0).all()
    # G per voxel from the final occupancy, then sum over hits
    G = 1.0 / (1.0 + np.exp(-ref["occ"])) - labels
    counts, flags, offs, keys = oracle.trace(mp, batch)
    exp = 0.0
    for i in range(batch.n_rays):
        if flags[i] & oracle.F_HAS_HIT:
            k = keys[offs[i + 1] - 1]
            exp += float(batch.weights[i]) * G[k[2], k[1], k[0]]
    assert abs(ref["grad_scalars"][0] - exp) <= 1e-9 * max(1.0, abs(exp))
    # and each ray's weight gradient is sum over its walk of G * delta
    i = int(np.nonzero(flags & oracle.F_HAS_HIT)[0][5])
    ks = keys[offs[i]:offs[i + 1]]
    exp_w = sum(G[k[2], k[1], k[0]] * (np.float32(0.847) if k[3] else np.float32(-0.405)) for k in ks)
    assert abs(ref["grad_w"][i] - exp_w) <= 1e-9 * max(1.0, abs(exp_w))


def test_forward_matches_ndt_oracle():
    """The differentiable forward is the same model as the NDT oracle (which
    stores float occupancy per scan): equal within float rounding."""
    batch = wall_scene(n_scans=3, n_rays=800, seed=5)
    labels = labels_for(MP)
    ref = oracle.adjoint(MP, batch, BOX_MIN, BOX_DIM, labels, None, ndt=True, grads=False)
    occ, _, _, _ = oracle.ndt_integrate(MP, batch, BOX_MIN, BOX_DIM, mode=1)
    np.testing.assert_allclose(ref["occ"], occ, atol=1e-5, rtol=0)
