"""Pins for the oracle's voxel walk (paper Sec. III-B, Amanatides & Woo line
walk, one voxel per step) against exact-rational brute force and closed forms.

Unit frame for most tests: voxel size 1, map origin 0, F = 16, so a point
p = q / 2^16 is exactly representable in fp32 and quantises to q.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from bruteforce import segment_voxels
from workloads.scenes import MapParams, RayBatch

F = 16
ONE = 1 << F


def unit_map(n=16, **kw):
    return MapParams(voxel_size=1.0, map_origin=(0.0, 0.0, 0.0), key_min=(0, 0, 0),
                     key_max=(n, n, n), fixed_bits=F, **kw)


def rays_from_q(pairs):
    """RayBatch with one scan per ray so every ray has its own origin."""
    origins = np.array([[v / ONE for v in q0] for q0, _ in pairs], np.float32)
    samples = np.array([[v / ONE for v in q1] for _, q1 in pairs], np.float32)
    for (q0, q1), o, s in zip(pairs, origins, samples):
        assert all(int(x * ONE) == v for x, v in zip(o, q0))
        assert all(int(x * ONE) == v for x, v in zip(s, q1))
    offsets = np.arange(len(pairs) + 1, dtype=np.uint32)
    return RayBatch(origins, samples, offsets)


def walks(mp, batch):
    counts, flags, offs, keys = oracle.trace(mp, batch)
    return [(keys[offs[i]:offs[i + 1]], int(flags[i])) for i in range(len(counts))]


def check_walk_against_bruteforce(q0, q1, walk):
    keys = [tuple(int(v) for v in k[:3]) for k in walk]
    k0 = tuple(q >> F for q in q0)
    k1 = tuple(q >> F for q in q1)
    L1 = sum(abs(a - b) for a, b in zip(k0, k1))
    # length, endpoints, face-connected monotone steps
    assert len(keys) == 1 + L1
    assert keys[0] == k0 and keys[-1] == k1
    sg = [(b > a) - (b < a) for a, b in zip(q0, q1)]
    for u, v in zip(keys, keys[1:]):
        diff = [b - a for a, b in zip(u, v)]
        assert sum(abs(d) for d in diff) == 1
        ax = next(i for i in range(3) if diff[i] != 0)
        assert diff[ax] == sg[ax]
    assert len(set(keys)) == len(keys)
    # set bounds from exact geometry
    closed = segment_voxels(q0, q1, F, "closed")
    opened = segment_voxels(q0, q1, F, "open")
    owned = segment_voxels(q0, q1, F, "halfopen")
    ks = set(keys)
    assert owned <= ks, f"walk misses owned voxels {owned - ks}"
    assert (opened | {k0, k1}) <= ks
    assert ks <= closed, f"walk leaves the closed-box set {ks - closed}"
    # order: first contact parameter never decreases along the walk
    D = [b - a for a, b in zip(q0, q1)]

    def entry_t(k):
        lo = Fraction(0)
        for a in range(3):
            if D[a] == 0:
                continue
            t_lo = Fraction(k[a] * ONE - q0[a], D[a])
            t_hi = Fraction((k[a] + 1) * ONE - q0[a], D[a])
            lo = max(lo, min(t_lo, t_hi))
        return lo

    ts = [entry_t(k) for k in keys]
    assert all(a <= b for a, b in zip(ts, ts[1:]))


def test_random_general_rays_match_bruteforce():
    rng = np.random.default_rng(11)
    pairs = []
    for _ in range(60):
        q0 = tuple(int(v) for v in rng.integers(0, 12 * ONE, size=3))
        q1 = tuple(int(v) for v in rng.integers(0, 12 * ONE, size=3))
        pairs.append((q0, q1))
    mp = unit_map(16)
    for (q0, q1), (walk, flags) in zip(pairs, walks(mp, rays_from_q(pairs))):
        assert flags & oracle.F_HAS_HIT
        check_walk_against_bruteforce(q0, q1, walk)


@pytest.mark.parametrize("q0,q1", [
    # axis aligned, positive and negative
    ((ONE // 2, ONE // 2, ONE // 2), (ONE // 2 + 5 * ONE, ONE // 2, ONE // 2)),
    ((5 * ONE + 7, 3 * ONE + 1, 2 * ONE + 9), (5 * ONE + 7, 3 * ONE + 1, 9 * ONE + 2)),
    ((9 * ONE + 3, 2 * ONE, 4 * ONE), (1 * ONE + 5, 2 * ONE, 4 * ONE)),
    # exact diagonals through voxel corners and edges
    ((0, 0, 0), (4 * ONE, 4 * ONE, 4 * ONE)),
    ((4 * ONE, 4 * ONE, 4 * ONE), (ONE // 2, ONE // 2, ONE // 2)),
    ((ONE // 2, 0, ONE // 2), (ONE // 2 + 3 * ONE, 3 * ONE, ONE // 2)),
    ((2 * ONE, 2 * ONE, 3 * ONE + 5), (5 * ONE, 8 * ONE, 3 * ONE + 5)),
    # origin on a face moving negative (zero-length first visit)
    ((3 * ONE, ONE // 2, ONE // 2), (ONE + ONE // 2, ONE // 2, ONE // 2)),
    ((3 * ONE, 3 * ONE, 3 * ONE), (2 * ONE + 1, ONE + 7, 5 * ONE + 3)),
    # zero length, same voxel, endpoint exactly on a boundary
    ((5 * ONE + 3, 5 * ONE + 3, 5 * ONE + 3), (5 * ONE + 3, 5 * ONE + 3, 5 * ONE + 3)),
    ((5 * ONE + 3, 5 * ONE + 3, 5 * ONE + 3), (5 * ONE + 900, 5 * ONE + 77, 5 * ONE + 5)),
    ((ONE + 11, ONE + 13, ONE + 17), (6 * ONE, 4 * ONE, 2 * ONE)),
])
def test_special_rays_match_bruteforce(q0, q1):
    mp = unit_map(16)
    (walk, flags), = walks(mp, rays_from_q([(q0, q1)]))
    assert flags & oracle.F_HAS_HIT
    check_walk_against_bruteforce(q0, q1, walk)


def test_corner_diagonal_tie_order_closed_form():
    """A ray through voxel corners steps x, then y, then z at each corner
    (ties to the lower axis); reversed direction does the same from the far
    corner."""
    mp = unit_map(16)
    pairs = [((0, 0, 0), (4 * ONE, 4 * ONE, 4 * ONE)),
             ((4 * ONE, 4 * ONE, 4 * ONE), (ONE // 2, ONE // 2, ONE // 2))]
    (w_fwd, _), (w_rev, _) = walks(mp, rays_from_q(pairs))
    exp = [(0, 0, 0)]
    for i in range(4):
        exp += [(i + 1, i, i), (i + 1, i + 1, i), (i + 1, i + 1, i + 1)]
    assert [tuple(k[:3]) for k in w_fwd] == exp
    exp_r = [(4, 4, 4)]
    for i in range(4, 0, -1):
        exp_r += [(i - 1, i, i), (i - 1, i - 1, i), (i - 1, i - 1, i - 1)]
    assert [tuple(k[:3]) for k in w_rev] == exp_r


def test_axis_aligned_consecutive_keys_and_kinds():
    mp = unit_map(16)
    (walk, flags), = walks(mp, rays_from_q([((ONE // 2, 2 * ONE + 5, 3 * ONE + 5),
                                              (7 * ONE + 3, 2 * ONE + 5, 3 * ONE + 5))]))
    assert [tuple(k) for k in walk] == [(x, 2, 3, 1 if x == 7 else 0) for x in range(8)]
    assert flags == oracle.F_HAS_HIT


def test_zero_length_ray_is_single_hit():
    mp = unit_map(16)
    q = (5 * ONE + 1, 6 * ONE + 2, 7 * ONE + 3)
    (walk, flags), = walks(mp, rays_from_q([(q, q)]))
    assert [tuple(k) for k in walk] == [(5, 6, 7, 1)]


def test_clipping_stops_at_first_outside_key():
    small = unit_map(8)
    big = unit_map(64)
    rng = np.random.default_rng(5)
    pairs = []
    for _ in range(40):
        q0 = tuple(int(v) for v in rng.integers(0, 8 * ONE, size=3))
        q1 = tuple(int(v) for v in rng.integers(-4 * ONE, 20 * ONE, size=3))
        pairs.append((q0, q1))
    batch = rays_from_q([(q0, tuple(max(v, 0) for v in q1)) for q0, q1 in pairs])
    for (ws, fs), (wb, fb) in zip(walks(small, batch), walks(big, batch)):
        full = [tuple(k[:3]) for k in wb]
        inside = []
        for k in full:
            if all(0 <= v < 8 for v in k):
                inside.append(k)
            else:
                break
        assert [tuple(k[:3]) for k in ws] == inside
        clipped = len(inside) < len(full)
        assert bool(fs & oracle.F_CLIPPED) == clipped
        assert bool(fs & oracle.F_HAS_HIT) == (not clipped)
        assert all(k[3] == 0 for k in ws[:-1])
        if ws.shape[0]:
            assert ws[-1][3] == (0 if clipped else 1)


def test_truncation_moves_endpoint_and_drops_hit():
    mp = unit_map(16, max_range=2.5)
    q0 = (ONE // 2, ONE // 2 + 3, ONE // 2 + 9)
    q1 = (ONE // 2 + 5 * ONE, ONE // 2 + 3, ONE // 2 + 9)
    (walk, flags), = walks(mp, rays_from_q([(q0, q1)]))
    # 0.5 + 2.5 = 3.0 exactly on the boundary of voxel 3
    assert [tuple(k) for k in walk] == [(x, 0, 0, 0) for x in range(4)]
    assert flags & oracle.F_TRUNCATED and not flags & oracle.F_HAS_HIT
    # a ray shorter than max range keeps its hit
    (walk2, flags2), = walks(mp, rays_from_q([(q0, (q0[0] + 2 * ONE, q0[1], q0[2]))]))
    assert flags2 == oracle.F_HAS_HIT and walk2[-1][3] == 1


def test_invalid_and_origin_outside_rays_are_rejected():
    mp = unit_map(8)
    batch = RayBatch(np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5], [9.0, 0.5, 0.5], [-0.25, 1, 1]], np.float32),
                     np.array([[np.nan, 1, 1], [1, np.inf, 1], [1, 1, 1], [1, 1, 1]], np.float32),
                     np.arange(5, dtype=np.uint32))
    counts, flags, _, _ = oracle.trace(mp, batch)
    assert counts.tolist() == [0, 0, 0, 0]
    assert flags.tolist() == [oracle.F_INVALID, oracle.F_INVALID, oracle.F_ORIGIN_OOB, oracle.F_ORIGIN_OOB]


def test_keys_equal_exact_floor_away_from_boundaries():
    """With a decimal voxel size the fixed-point key equals the exact-real
    floor((p - m) / s) whenever p is farther than 2^-15 voxel from a face."""
    mp = MapParams(voxel_size=0.1, map_origin=(-10.0, -10.0, -10.0), key_min=(0, 0, 0),
                   key_max=(200, 200, 200))
    rng = np.random.default_rng(3)
    pts = rng.uniform(-9.99, 9.99, size=(400, 3)).astype(np.float32)
    batch = RayBatch(pts, pts.copy(), np.arange(401, dtype=np.uint32))
    counts, flags, offs, keys = oracle.trace(mp, batch)
    assert (counts == 1).all()
    s = Fraction(0.1)
    checked = 0
    for p, k in zip(pts, keys):
        for a in range(3):
            u = (Fraction(float(p[a])) - Fraction(-10.0)) / s
            if abs(u - round(u)) < Fraction(1, 1 << 15):
                continue
            assert k[a] == math.floor(u)
            checked += 1
    assert checked > 1000


def test_sensor_at_voxel_corner_config0():
    """Config 0's sensor at (0,0,0) sits on the corner of voxel (100,100,100):
    every ray starts there (rays moving negative visit it with zero length)."""
    from workloads import scenes
    mp, batch = scenes.config0(n_rays=512)
    counts, flags, offs, keys = oracle.trace(mp, batch)
    assert (keys[offs[:-1]][:, :3] == 100).all()
