"""Pins for the oracle's batch update (paper Sec. II-B, Eq. (2)-(3) and the
clamping paragraph; per-update CAS semantics of Sec. III-B).

Counts are rebuilt from the exact-rational brute-force voxel sets (not from
the oracle's walk); the per-update bracket is checked against enumerating
every interleaving of the updates.
"""
import numpy as np
import pytest

import oracle
from bruteforce import all_orders_range, segment_voxels
from workloads import scenes
from workloads.scenes import MapParams, RayBatch

F = 16
ONE = 1 << F


def unit_map(n, **kw):
    return MapParams(voxel_size=1.0, map_origin=(0.0, 0.0, 0.0), key_min=(0, 0, 0),
                     key_max=(n, n, n), fixed_bits=F, **kw)


def general_position_rays(rng, n, origin_q, lo, hi):
    """Rays from one origin whose closed-box and owned voxel sets coincide
    (no edge or corner passes), so the walk's voxel set is fixed by geometry
    alone."""
    out = []
    while len(out) < n:
        q1 = tuple(int(v) for v in rng.integers(lo, hi, size=3))
        closed = segment_voxels(origin_q, q1, F, "closed")
        owned = segment_voxels(origin_q, q1, F, "halfopen")
        if closed == owned:
            out.append((q1, owned))
    return out


def test_counts_and_values_match_bruteforce():
    rng = np.random.default_rng(7)
    n = 10
    mp = unit_map(n)
    oq = (5 * ONE + 1234, 4 * ONE + 777, 5 * ONE + 4321)
    rays = general_position_rays(rng, 120, oq, 0, n * ONE)
    H = np.zeros((n, n, n), np.int64)
    M = np.zeros((n, n, n), np.int64)
    for q1, vox in rays:
        k1 = tuple(q >> F for q in q1)
        for k in vox:
            if k == k1:
                H[k[2], k[1], k[0]] += 1
            else:
                M[k[2], k[1], k[0]] += 1
    batch = RayBatch(np.array([[v / ONE for v in oq]], np.float32),
                     np.array([[v / ONE for v in q1] for q1, _ in rays], np.float32),
                     np.array([0, len(rays)], np.uint32))
    occ, lh, lm, st = oracle.integrate_count(mp, batch)
    assert (lh == H).all() and (lm == M).all()
    assert st["updates"] == int(H.sum() + M.sum())
    assert st["hits"] == len(rays)
    # fp32 count-then-clamp from zero
    exp = np.clip(np.float32(0) + H.astype(np.float32) * np.float32(mp.l_hit) + M.astype(np.float32) * np.float32(mp.l_miss),
                  np.float32(mp.l_min), np.float32(mp.l_max))
    assert np.array_equal(occ, exp)
    # the sensor voxel takes one miss per ray
    ko = tuple(q >> F for q in oq)
    assert M[ko[2], ko[1], ko[0]] == len(rays)


def test_count_mode_single_voxel_closed_forms():
    """Many rays ending in one voxel: l = min(H*l_hit, l_max); a voxel crossed
    by many rays: l = max(M*l_miss, l_min)."""
    mp = unit_map(8)
    o = np.array([[0.5, 0.5, 0.5]], np.float32)
    for nh, exp in [(1, 0.847), (3, np.float32(3) * np.float32(0.847)), (5, 3.5)]:
        s = np.tile(np.array([[6.5, 0.5, 0.5]], np.float32), (nh, 1))
        occ, lh, lm, _ = oracle.integrate_count(mp, RayBatch(o, s, np.array([0, nh], np.uint32)))
        assert occ[0, 0, 6] == np.float32(exp)
        assert lm[0, 0, 3] == nh
        exp_m = max(np.float32(nh) * np.float32(-0.405), np.float32(-2.0))
        assert occ[0, 0, 3] == np.float32(exp_m)


def test_multi_scan_is_sequential_per_scan_clamp():
    """Two scans integrate as scan 1 then scan 2, each clamped once."""
    mp = unit_map(12, l_min=-1.0, l_max=1.5)
    rng = np.random.default_rng(2)
    o1, o2 = np.array([5.5, 5.5, 5.5]), np.array([6.25, 5.75, 5.125])
    s1 = (o1 + rng.uniform(-5, 5, size=(300, 3))).astype(np.float32)
    s2 = (o2 + rng.uniform(-5, 5, size=(300, 3))).astype(np.float32)
    both = RayBatch(np.stack([o1, o2]).astype(np.float32), np.concatenate([s1, s2]),
                    np.array([0, 300, 600], np.uint32))
    occ2, _, _, _ = oracle.integrate_count(mp, both)
    a, lh1, lm1, _ = oracle.integrate_count(mp, both.scans(0, 1))
    b, lh2, lm2, _ = oracle.integrate_count(mp, both.scans(1, 1), occ=a)
    assert np.array_equal(occ2, b)
    # and scan 2 alone from scan 1's state is the closed form on its counts
    exp = np.clip((a + lh2 * np.float32(mp.l_hit)) + lm2 * np.float32(mp.l_miss),
                  np.float32(mp.l_min), np.float32(mp.l_max)).astype(np.float32)
    touched = (lh2 + lm2) > 0
    assert np.array_equal(b[touched], exp[touched])
    assert np.array_equal(b[~touched], a[~touched])


def test_config0_invariants_small():
    """Config-0 style batch on a 64^3 map: update totals, hits, the sensor
    voxel's exact miss count, clamp bounds."""
    mp = scenes.grid_map((-3.2, -3.2, -3.2), (3.2, 3.2, 3.2), 0.1)
    batch = scenes.random_rays(3000, 9, None, None, (0.0, 0.0, 0.0), 1.0, 4.0)
    counts, flags, offs, keys = oracle.trace(mp, batch)
    occ, lh, lm, st = oracle.integrate_count(mp, batch)
    assert st["updates"] == int(counts.sum()) == int(lh.sum() + lm.sum())
    assert st["hits"] == int(((flags & oracle.F_HAS_HIT) > 0).sum()) == int(lh.sum())
    assert st["clipped"] == int(((flags & oracle.F_CLIPPED) > 0).sum()) > 0
    assert lm[32, 32, 32] == 3000 and lh[32, 32, 32] == 0
    assert occ.min() >= np.float32(mp.l_min) and occ.max() <= np.float32(mp.l_max)


def test_weighted_count_mode_unit_weights_equal_unweighted():
    mp = unit_map(10)
    batch = scenes.random_rays(400, 4, None, None, (5.1, 4.9, 5.3), 0.0, 6.0)
    occ_a, _, _, _ = oracle.integrate_count(mp, batch)
    batch.weights = np.ones(batch.n_rays, np.float32)
    occ_b, _, _, _ = oracle.integrate_count(mp, batch)
    np.testing.assert_allclose(occ_a, occ_b, atol=1e-6, rtol=0)
    batch.weights = np.full(batch.n_rays, 0.5, np.float32)
    occ_c, lh, lm, _ = oracle.integrate_count(mp, batch)
    exp = np.clip(lh.astype(np.float64) * np.float32(0.847) + lm.astype(np.float64) * np.float32(-0.405), -2.0, 3.5)
    np.testing.assert_allclose(occ_c, exp, atol=1e-6, rtol=0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_per_update_bracket_equals_all_orders(seed):
    """For one scan, [lo, hi] equals min/max over every interleaving of the
    voxel's hit and miss updates, each applied as l <- clamp(l + delta)."""
    n = 6
    mp = unit_map(n, l_min=-0.9, l_max=1.2, l_init=0.25)
    rng = np.random.default_rng(100 + seed)
    oq = (3 * ONE + 2000, 2 * ONE + 5000, 3 * ONE + 100)
    rays = general_position_rays(rng, 20, oq, 0, n * ONE)
    batch = RayBatch(np.array([[v / ONE for v in oq]], np.float32),
                     np.array([[v / ONE for v in q1] for q1, _ in rays], np.float32),
                     np.array([0, len(rays)], np.uint32))
    lo, hi, nupd, _ = oracle.integrate_envelope(mp, batch)
    H = {}
    M = {}
    for q1, vox in rays:
        k1 = tuple(q >> F for q in q1)
        for k in vox:
            d = H if k == k1 else M
            d[k] = d.get(k, 0) + 1
    checked = 0
    for k in set(H) | set(M):
        h, m = H.get(k, 0), M.get(k, 0)
        if h + m > 8 or h == 0 or m == 0:
            continue
        f = lambda v: float(np.float32(v))
        blo, bhi = all_orders_range(f(0.25), [f(0.847)] * h, [f(-0.405)] * m, f(-0.9), f(1.2))
        z, y, x = k[2], k[1], k[0]
        assert abs(lo[z, y, x] - blo) < 1e-12 and abs(hi[z, y, x] - bhi) < 1e-12
        assert nupd[z, y, x] == h + m
        checked += 1
    assert checked >= 2


def test_per_update_bracket_two_scans_all_orders():
    """Across two scans the bracket propagates through the monotone maps:
    it equals min/max over all interleavings in both scans."""
    mp = unit_map(4, l_min=-0.9, l_max=1.2, l_init=0.0)
    # voxel (1,1,1): scan 1 = 2 hits + 3 misses, scan 2 = 1 hit + 3 misses
    o = np.array([[0.5, 1.5, 1.5]], np.float32)
    hit1 = np.array([[1.5, 1.5, 1.5]], np.float32)
    through = np.array([[2.5, 1.5, 1.5]], np.float32)
    s1 = np.concatenate([np.repeat(hit1, 2, 0), np.repeat(through, 3, 0)])
    s2 = np.concatenate([np.repeat(hit1, 1, 0), np.repeat(through, 3, 0)])
    batch = RayBatch(np.concatenate([o, o]), np.concatenate([s1, s2]), np.array([0, 5, 9], np.uint32))
    lo, hi, nupd, _ = oracle.integrate_envelope(mp, batch)
    import itertools
    f = lambda v: float(np.float32(v))
    seq1 = [f(0.847)] * 2 + [f(-0.405)] * 3
    seq2 = [f(0.847)] * 1 + [f(-0.405)] * 3
    lmin, lmax = f(-0.9), f(1.2)
    vals = set()
    for p1 in set(itertools.permutations(seq1)):
        l1 = 0.0
        for d in p1:
            l1 = min(max(l1 + d, lmin), lmax)
        for p2 in set(itertools.permutations(seq2)):
            l2 = l1
            for d in p2:
                l2 = min(max(l2 + d, lmin), lmax)
            vals.add(l2)
    assert abs(lo[1, 1, 1] - min(vals)) < 1e-12 and abs(hi[1, 1, 1] - max(vals)) < 1e-12
    assert nupd[1, 1, 1] == 9
