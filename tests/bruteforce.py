"""Independent brute-force checks used to pin the oracle (test helper).

Everything here works on exact rationals (``fractions.Fraction``) and shares
nothing with the oracle: for a segment p(t) = q0 + t (q1 - q0), t in [0, 1],
given in fixed-point units where one voxel spans ``2**F``, it finds the
voxels whose box the segment meets, under three box conventions:

* ``closed``    -- [k 2^F, (k+1) 2^F] on every axis,
* ``open``      -- (k 2^F, (k+1) 2^F),
* ``halfopen``  -- [k 2^F, (k+1) 2^F), i.e. the voxel that owns each point
  under floor semantics.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from typing import Iterable, List, Set, Tuple


def _axis_interval(q0: int, d: int, lo: int, hi: int, lo_closed: bool, hi_closed: bool):
    """Interval of t in R where lo <(=) q0 + t d <(=) hi; None if empty, 'all'
    if every t qualifies (d == 0 and q0 inside)."""
    if d == 0:
        ok_lo = q0 >= lo if lo_closed else q0 > lo
        ok_hi = q0 <= hi if hi_closed else q0 < hi
        return "all" if (ok_lo and ok_hi) else None
    a = Fraction(lo - q0, d)
    b = Fraction(hi - q0, d)
    if d > 0:
        return (a, lo_closed, b, hi_closed)
    return (b, hi_closed, a, lo_closed)


def _intersect(ivs) -> bool:
    """Is the intersection of [0, 1] with every interval non-empty?"""
    lo, lo_c, hi, hi_c = Fraction(0), True, Fraction(1), True
    for iv in ivs:
        if iv is None:
            return False
        if iv == "all":
            continue
        a, ac, b, bc = iv
        if a > lo:
            lo, lo_c = a, ac
        elif a == lo:
            lo_c = lo_c and ac
        if b < hi:
            hi, hi_c = b, bc
        elif b == hi:
            hi_c = hi_c and bc
    return lo < hi or (lo == hi and lo_c and hi_c)


def segment_voxels(q0, q1, F: int, kind: str) -> Set[Tuple[int, int, int]]:
    one = 1 << F
    k0 = [q >> F for q in q0]
    k1 = [q >> F for q in q1]
    ranges = [range(min(a, b) - 1, max(a, b) + 2) for a, b in zip(k0, k1)]
    out = set()
    for k in itertools.product(*ranges):
        ivs = []
        for a in range(3):
            lo, hi = k[a] * one, (k[a] + 1) * one
            d = q1[a] - q0[a]
            if kind == "closed":
                ivs.append(_axis_interval(q0[a], d, lo, hi, True, True))
            elif kind == "open":
                ivs.append(_axis_interval(q0[a], d, lo, hi, False, False))
            else:
                ivs.append(_axis_interval(q0[a], d, lo, hi, True, False))
        if _intersect(ivs):
            out.add(tuple(k))
    return out


def sequential_clamp(l: float, deltas: Iterable[float], lo: float, hi: float) -> float:
    for d in deltas:
        l = min(max(l + d, lo), hi)
    return l


def all_orders_range(l: float, hits: List[float], misses: List[float], lo: float, hi: float):
    """Min and max of the sequential clamp over every distinct interleaving
    of the given hit and miss deltas (brute force)."""
    seq = [("h", v) for v in hits] + [("m", v) for v in misses]
    best_lo, best_hi = None, None
    for perm in set(itertools.permutations(range(len(seq)))):
        v = sequential_clamp(l, (seq[i][1] for i in perm), lo, hi)
        best_lo = v if best_lo is None else min(best_lo, v)
        best_hi = v if best_hi is None else max(best_hi, v)
    return best_lo, best_hi


def segment_box_interval(q0, q1, k, F: int):
    """Exact parameter interval [t_lo, t_hi] (Fractions, clipped to [0, 1])
    of the segment inside the closed box of voxel k, or None."""
    one = 1 << F
    lo_t, hi_t = Fraction(0), Fraction(1)
    for a in range(3):
        lo, hi = k[a] * one, (k[a] + 1) * one
        d = q1[a] - q0[a]
        if d == 0:
            if not (lo <= q0[a] <= hi):
                return None
            continue
        t0, t1 = Fraction(lo - q0[a], d), Fraction(hi - q0[a], d)
        if t0 > t1:
            t0, t1 = t1, t0
        lo_t, hi_t = max(lo_t, t0), min(hi_t, t1)
    return (lo_t, hi_t) if lo_t <= hi_t else None
