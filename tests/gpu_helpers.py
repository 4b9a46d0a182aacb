"""Shared helpers for the GPU parity tests: run a workload through the HIP
C-ABI and through the oracle on the same seeded inputs."""
import numpy as np
import torch

import paper_2206_06079_amd as ohm


def device():
    return torch.device("cuda", 0)


def to_dev(batch):
    d = device()
    o = torch.from_numpy(np.ascontiguousarray(batch.origins)).to(d)
    s = torch.from_numpy(np.ascontiguousarray(batch.samples)).to(d)
    w = None if batch.weights is None else torch.from_numpy(np.ascontiguousarray(batch.weights)).to(d)
    return o, s, np.asarray(batch.offsets, np.uint32), w


def full_box(mp):
    return tuple(mp.key_min), tuple(b - a for a, b in zip(mp.key_min, mp.key_max))


def gpu_integrate(mp, batch, capacity, box_min, box_dim, scans_per_call=None, layers=ohm.LAYER_OCC, column_rays=0):
    """Integrate through ohm_integrate_rays; returns (occ, hits, misses, stats)
    over the box (hits/misses are the last scan's weights).  column_rays: the
    scans' column layout declared to the map (0: none)."""
    m = ohm.OhmMap(mp, capacity, layers=layers, device=device())
    if column_rays:
        m.set_scan_layout(column_rays)
    o, s, off, w = to_dev(batch)
    if scans_per_call is None:
        m.integrate(o, s, off, w)
    else:
        for first in range(0, batch.n_scans, scans_per_call):
            cnt = min(scans_per_call, batch.n_scans - first)
            sub = batch.scans(first, cnt)
            so, ss, soff, sw = to_dev(sub)
            m.integrate(so, ss, soff, sw)
    occ = m.read_dense(ohm.READ_OCC, box_min, box_dim).cpu().numpy()
    hits = m.read_dense(ohm.READ_HITS, box_min, box_dim).cpu().numpy()
    miss = m.read_dense(ohm.READ_MISSES, box_min, box_dim).cpu().numpy()
    st = m.stats()
    m.close()
    return occ, hits, miss, st


def gpu_trace(mp, batch, capacity=8):
    m = ohm.OhmMap(mp, capacity, device=device())
    o, s, off, _ = to_dev(batch)
    counts, flags, offs, upd = m.trace(o, s, off)
    torch.cuda.synchronize()
    out = counts.cpu().numpy(), flags.cpu().numpy(), offs.cpu().numpy(), upd.cpu().numpy()
    m.close()
    return out


def per_update_tolerance(nupd):
    """fp32 rounding bound for a voxel that took k updates applied one by one
    (|l| <= 4, each add rounds by at most half an ulp of 4): k * 2^-22 + 1e-6."""
    return nupd.astype(np.float64) * 2.0 ** -22 + 1e-6
