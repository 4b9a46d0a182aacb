#!/usr/bin/env python3
"""Throughput benchmark of lidar ray integration on one MI355X.

Headline workload (one "step"): the 100-scan spinning-lidar sequence -- 64 beams x
2048 columns = 131,072 rays per scan, sensor moving 0.1 m per scan along a
4 x 3 m box tunnel with 200 random boxes, 30 m max range -- integrated scan by
scan into a 0.1 m occupancy map of 32^3-voxel regions over 200 x 200 x 40 m.
Inputs are generated once (seeded) and stay resident in HBM; a step is one
ohm_integrate_rays call over all 100 scans on a map with scan groups of G
(default 50) accumulator slots (the voxel walk with its atomic updates over G
scans per launch, then the in-order per-scan clamp of the group); the same
call on a map that launches once per scan is timed beside it.

Reported alongside: the per-update (CAS) mode, NDT-OM integration of the
same scans, the adjoint on the 20-scan 0.2 m workload, and the batched
multi-sensor plan against per-scan launches.  Prints one JSON line on
stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def walk_bytes(rays, updates, scans=1.0):
    """Algorithmic bytes of the walk kernel: each ray reads its 12-byte sample
    (plus each scan's 12-byte origin), and each voxel update is one 4-byte
    read-modify-write at the coherence point (4 B read + 4 B written)."""
    return 12.0 * rays + 12.0 * scans + 8.0 * updates


def kernel_source_digest():
    """sha256 over the library's kernel sources (names and contents)."""
    import hashlib

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2206_06079_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".h", ".hip")):
            h.update(f.encode())
            h.update(b"\0")
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from its committed byte-counter
    summary, or None once the kernel sources differ from those the counters
    were taken on."""
    import re

    path = os.path.join(ROOT, "profiles", f"{kernel}_config1_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    tb = re.search(r"^traffic_bytes_per_launch:\s*(\d+)", text, re.M)
    sha = re.search(r"^kernel_source_sha256:\s*([0-9a-f]{64})", text, re.M)
    if not tb or not sha or sha.group(1) != kernel_source_digest():
        return None
    return int(tb.group(1))


def run_gpu(args, params, batch, mode, layers=1):
    import torch

    import paper_2206_06079_amd as ohm

    dev = torch.device("cuda", 0)
    o = torch.from_numpy(batch.origins).to(dev)
    s = torch.from_numpy(batch.samples).to(dev)
    off = batch.offsets
    m = ohm.OhmMap(params.replace(mode=mode), args.capacity, layers=layers, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        m.integrate(o, s, off)
    torch.cuda.synchronize()
    st0 = m.stats()
    steps = args.steps if mode == ohm.MODE_COUNT_CLAMP else max(2, args.steps // 2)
    m.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(steps):
        m.integrate(o, s, off)
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = m.kernel_times()
    m.set_profiling(False)
    st1 = m.stats()
    m.close()
    ms_total = e0.elapsed_time(e1)
    upd = (st1["voxel_updates"] - st0["voxel_updates"]) / steps
    rays = (st1["rays_in"] - st0["rays_in"]) / steps
    return {
        "steps": steps,
        "ms_per_step": ms_total / steps,
        "wall_ms_per_step": (t1 - t0) * 1e3 / steps,
        "rays_per_step": rays,
        "updates_per_step": upd,
        "kernels": kt,
        "stats": st1,
    }


def generate_batched(args):
    """The multi-sensor workload's inputs, generated before anything touches
    the GPU (the generator's worker processes must not start from a process
    that holds GPU state)."""
    from workloads import scenes

    jobs = max(1, min(16, os.cpu_count() or 1))
    log(f"generating the batched workload ({args.batched_scans} scans, {jobs} processes)")
    t0 = time.perf_counter()
    params, batches = scenes.config3(n_scans=args.batched_scans, jobs=jobs)
    log(f"generated {sum(b.n_rays for b in batches)} rays in {time.perf_counter() - t0:.1f} s")
    return params, batches


def run_batched(args, generated):
    """The multi-sensor workload: 16 streams, scans of log-uniform size in
    [8192, 262144] rays with unordered directions, half into a 0.1 m map and
    half into a 0.05 m map.  Times one graph launch of the batched plan
    (schedule from the autotuner) against per-scan launches of the plain
    path over the same maps (walking each scan in direction order, and in
    its given order), all with inputs resident in HBM."""
    import numpy as np
    import torch

    import paper_2206_06079_amd as ohm

    params, batches = generated
    n_rays = sum(b.n_rays for b in batches)
    dev = torch.device("cuda", 0)
    caps = (512, 1536)
    inputs = [(torch.from_numpy(b.origins).to(dev), torch.from_numpy(b.samples).to(dev), b.offsets)
              for b in batches]

    def fresh_sets():
        maps = [ohm.OhmMap(p.replace(mode=ohm.MODE_COUNT_CLAMP), c, device=dev) for p, c in zip(params, caps)]
        return maps, [ohm.ScanSetArgs(m, o, s, off) for m, (o, s, off) in zip(maps, inputs)]

    maps, sets = fresh_sets()
    choice = ohm.autotune(sets, groups=args.batched_groups, tiles=args.batched_tiles, orders=(0, 1), reps=1, log=log)
    plan = ohm.OhmBatch(sets, **choice)
    stream = torch.cuda.current_stream()
    plan.run(stream)
    torch.cuda.synchronize()
    st0 = [m.stats() for m in maps]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = args.batched_reps
    e0.record(stream)
    for _ in range(reps):
        plan.run(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_batched = e0.elapsed_time(e1) / reps
    st1 = [m.stats() for m in maps]
    upd = sum(b["voxel_updates"] - a["voxel_updates"] for a, b in zip(st0, st1)) / reps
    plan.close()
    for m in maps:
        m.close()
    # per-scan plain launches over the same scans, in the same per-map order,
    # with the scans walked in direction order and in their given order
    max_scan = max(int(np.diff(b.offsets.astype(np.int64)).max()) for b in batches)
    ms_plain = {}
    for label, order in (("direction_order", max_scan), ("given_order", 0)):
        maps, _ = fresh_sets()
        for m, (o, s, off) in zip(maps, inputs):
            m.set_ray_order(order)
            m.integrate(o, s, off)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            for m, (o, s, off) in zip(maps, inputs):
                m.integrate(o, s, off)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_plain[label] = e0.elapsed_time(e1) / reps
        for m in maps:
            m.close()
    log(f"batched {choice}: {ms_batched:.2f} ms per pass; per-scan launches: {ms_plain}")
    return {
        "workload": f"16 sensor streams, {args.batched_scans} scans of log-uniform size in [8192, 262144] rays "
                    f"({n_rays} rays), tunnel scene, maps at 0.1 m and 0.05 m",
        "rays_per_s": round(n_rays / (ms_batched * 1e-3), 1),
        "voxel_updates_per_s": round(upd / (ms_batched * 1e-3), 1),
        "ms_per_pass": round(ms_batched, 3),
        "schedule": choice,
        "per_scan_plain_rays_per_s": round(n_rays / (ms_plain["direction_order"] * 1e-3), 1),
        "per_scan_plain_ms_per_pass": round(ms_plain["direction_order"], 3),
        "speedup_vs_per_scan": round(ms_plain["direction_order"] / ms_batched, 3),
        "per_scan_plain_given_order_rays_per_s": round(n_rays / (ms_plain["given_order"] * 1e-3), 1),
    }


def run_batched_headline(args, params, batch):
    """The headline scans through the batched plan: groups of G scans per
    launch (G, tile and ray order from the autotuner), timed per graph
    replay -- the same 100 scans, so the figure compares directly with
    `value`."""
    import torch

    import paper_2206_06079_amd as ohm

    dev = torch.device("cuda", 0)
    o = torch.from_numpy(batch.origins).to(dev)
    s = torch.from_numpy(batch.samples).to(dev)
    p = params.replace(mode=ohm.MODE_COUNT_CLAMP)
    m = ohm.OhmMap(p, args.capacity, device=dev)
    sets = [ohm.ScanSetArgs(m, o, s, batch.offsets)]
    choice = ohm.autotune(sets, groups=(4, 16, 50), tiles=((32, 512),), orders=(0, 1), reps=1)
    plan = ohm.OhmBatch(sets, **choice)
    stream = torch.cuda.current_stream()
    plan.run(stream)
    torch.cuda.synchronize()
    st0 = m.stats()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, args.steps // 2)
    e0.record(stream)
    for _ in range(reps):
        plan.run(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    st1 = m.stats()
    plan.close()
    m.close()
    rays = (st1["rays_in"] - st0["rays_in"]) / reps
    upd = (st1["voxel_updates"] - st0["voxel_updates"]) / reps
    log(f"headline scans through the batched plan {choice}: {ms:.3f} ms per pass")
    return {
        "workload": f"the same {batch.n_scans} scans through the batched plan (one map)",
        "rays_per_s": round(rays / (ms * 1e-3), 1),
        "voxel_updates_per_s": round(upd / (ms * 1e-3), 1),
        "ms_per_pass": round(ms, 3),
        "schedule": choice,
    }


def run_ndt(args, params, batch):
    """NDT-OM integration of the same 100 scans (sensor noise 0.05 m,
    adaptation rate 1, 4 samples before a voxel weights its misses), count
    mode, timed like the plain path."""
    import torch

    import paper_2206_06079_amd as ohm

    p = params.replace(sensor_noise=0.05, adaptation_rate=1.0, ndt_min_samples=4, mode=ohm.MODE_COUNT_CLAMP)
    dev = torch.device("cuda", 0)
    o = torch.from_numpy(batch.origins).to(dev)
    s = torch.from_numpy(batch.samples).to(dev)
    m = ohm.OhmMap(p, args.capacity, layers=ohm.LAYER_NDT, device=dev)
    stream = torch.cuda.current_stream()
    m.ndt_integrate(o, s, batch.offsets)
    torch.cuda.synchronize()
    st0 = m.stats()
    steps = max(1, args.steps // 3)
    m.set_profiling(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        m.ndt_integrate(o, s, batch.offsets)
    e1.record(stream)
    torch.cuda.synchronize()
    kt = m.kernel_times()
    st1 = m.stats()
    m.close()
    ms = e0.elapsed_time(e1) / steps
    rays = (st1["rays_in"] - st0["rays_in"]) / steps
    upd = (st1["voxel_updates"] - st0["voxel_updates"]) / steps
    log(f"ndt: {ms:.3f} ms per {batch.n_scans}-scan pass")
    return {
        "workload": f"the same {batch.n_scans} scans into an NDT-OM map (count mode)",
        "rays_per_s": round(rays / (ms * 1e-3), 1),
        "voxel_updates_per_s": round(upd / (ms * 1e-3), 1),
        "ms_per_pass": round(ms, 3),
        "kernel_us_per_scan": {k: round(v[1] / v[0] * 1e3, 1) for k, v in kt.items()},
    }


def run_adjoint(args):
    """The differentiable workload: 20 scans at 0.2 m with per-ray weights
    into an NDT map, then the adjoint for an upstream gradient on a 64^3
    box (traversals recomputed, statistics replayed)."""
    import torch

    import paper_2206_06079_amd as ohm
    from workloads import scenes

    params, batch, box_min, box_dim, _ = scenes.config4(n_scans=20)
    dev = torch.device("cuda", 0)
    o = torch.from_numpy(batch.origins).to(dev)
    s = torch.from_numpy(batch.samples).to(dev)
    w = torch.from_numpy(batch.weights).to(dev)
    g = torch.full((box_dim[2], box_dim[1], box_dim[0]), 1e-3, dtype=torch.float32, device=dev)
    gw = torch.zeros_like(w)
    stream = torch.cuda.current_stream()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd, bwd = [], []
    for _ in range(2):  # the first pass warms up
        m = ohm.OhmMap(params, 256, layers=ohm.LAYER_NDT | ohm.LAYER_ADJOINT, device=dev)
        e[0].record(stream)
        m.ndt_integrate(o, s, batch.offsets, w)
        e[1].record(stream)
        m.backward(g, box_min, box_dim, o, s, batch.offsets, w, ndt=True, grad_weights=gw)
        e[2].record(stream)
        torch.cuda.synchronize()
        m.close()
        fwd.append(e[0].elapsed_time(e[1]))
        bwd.append(e[1].elapsed_time(e[2]))
    log(f"adjoint: forward {fwd[-1]:.2f} ms, backward {bwd[-1]:.2f} ms")
    return {
        "workload": f"{batch.n_scans} scans x {batch.n_rays // batch.n_scans} weighted rays at 0.2 m, NDT, "
                    "64^3 loss box",
        "forward_ms": round(fwd[-1], 3),
        "backward_ms": round(bwd[-1], 3),
        "backward_rays_per_s": round(batch.n_rays / (bwd[-1] * 1e-3), 1),
    }


def cpu_baseline(params, batch, n_scans):
    import oracle

    box_min, box_dim = (690, 978, 183), (720, 44, 34)
    sub = batch.scans(0, n_scans)
    t0 = time.perf_counter()
    _, _, _, st = oracle.integrate_count(params, sub, box_min, box_dim)
    dt = time.perf_counter() - t0
    return {
        "value": st["rays"] / dt,
        "unit": "rays/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {n_scans} of the 100 scans ({st['rays']} rays, {st['updates']} voxel updates), "
                  f"single-threaded C oracle, count-then-clamp, {dt:.1f} s",
        "voxel_updates_per_s": st["updates"] / dt,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scans", type=int, default=100)
    ap.add_argument("--capacity", type=int, default=512)
    ap.add_argument("--scan-group-slots", type=int, default=50,
                    help="accumulator slots of the headline map (scans walked per launch)")
    ap.add_argument("--cpu-scans", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-update", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-ndt", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--batched-scans", type=int, default=1000)
    ap.add_argument("--batched-reps", type=int, default=3)
    ap.add_argument("--batched-groups", type=lambda v: tuple(int(x) for x in v.split(",")), default=(16, 64))
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this size (reference for HBM byte counters)")
    ap.add_argument("--batched-tiles", type=lambda v: tuple(tuple(int(y) for y in x.split("/")) for x in v.split(",")),
                    default=((32, 512),), help="walk tiles K/T,K/T,...")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(how it would shard is described in the design notes)", file=sys.stderr)
        return 2

    from workloads import scenes

    batched_inputs = None if args.no_batched else generate_batched(args)

    import torch

    import paper_2206_06079_amd as ohm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    ohm._lib.load()  # fails loudly when the HIP library is missing
    log(f"generating {args.scans} scans")
    t0 = time.perf_counter()
    params, batch = scenes.config1(n_scans=args.scans)
    log(f"generated {batch.n_rays} rays in {time.perf_counter() - t0:.1f} s")

    single = run_gpu(args, params, batch, ohm.MODE_COUNT_CLAMP)
    log(f"count mode, one launch per scan: {single['ms_per_step']:.3f} ms/step, kernels {single['kernels']}")
    res = run_gpu(args, params, batch, ohm.MODE_COUNT_CLAMP,
                  ohm.LAYER_OCC | ohm.LAYER_SCAN_GROUPS | ohm.scan_group_slots(args.scan_group_slots))
    log(f"count mode, {args.scan_group_slots}-scan groups: {res['ms_per_step']:.3f} ms/step, kernels {res['kernels']}")
    per_update = None
    if not args.no_per_update:
        pu = run_gpu(args, params, batch, ohm.MODE_PER_UPDATE)
        log(f"per-update mode: {pu['ms_per_step']:.3f} ms/step, kernels {pu['kernels']}")
        per_update = {
            "rays_per_s": pu["rays_per_step"] / (pu["ms_per_step"] * 1e-3),
            "voxel_updates_per_s": pu["updates_per_step"] / (pu["ms_per_step"] * 1e-3),
            "ms_per_step": pu["ms_per_step"],
            "walk_kernel_ms": pu["kernels"].get("walk", (0, 0.0))[1] / max(1, pu["kernels"].get("walk", (1, 0))[0]),
        }

    sec = res["ms_per_step"] * 1e-3
    rays_per_s = res["rays_per_step"] / sec
    upd_per_s = res["updates_per_step"] / sec
    scans = args.scans
    rays_per_scan = res["rays_per_step"] / scans
    upd_per_scan = res["updates_per_step"] / scans
    # dominant kernel: the group walk (scans that took the single-scan walk
    # instead, if any, are not its work)
    n_walk, ms_walk = res["kernels"].get("walk_group", (0, 0.0))
    walk_avg_ms = ms_walk / max(1, n_walk)
    single_scans = res["kernels"].get("walk", (0, 0.0))[0] / res["steps"]
    scans_per_launch = (scans - single_scans) * res["steps"] / max(1, n_walk)
    launch_bytes = walk_bytes(rays_per_scan * scans_per_launch, upd_per_scan * scans_per_launch, scans_per_launch)
    achieved = launch_bytes / (walk_avg_ms * 1e-3) / 1e9
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic("walk_group_kernel"),
        "kernel": f"walk_group_kernel (count mode, up to {args.scan_group_slots} scans per launch)",
        "kernel_avg_ms": round(walk_avg_ms, 5),
        "scans_per_launch": round(scans_per_launch, 3),
        "bytes_per_launch": launch_bytes,
    }
    s_walk_n, s_walk_ms = single["kernels"].get("walk", (0, 0.0))
    s_walk_avg = s_walk_ms / max(1, s_walk_n)
    s_sec = single["ms_per_step"] * 1e-3
    one_launch_per_scan = {
        "rays_per_s": round(single["rays_per_step"] / s_sec, 1),
        "voxel_updates_per_s": round(single["updates_per_step"] / s_sec, 1),
        "ms_per_step": round(single["ms_per_step"], 4),
        "kernel": "walk_seg_kernel",
        "kernel_avg_ms": round(s_walk_avg, 5),
        "hbm_frac": round(walk_bytes(rays_per_scan, upd_per_scan) / (s_walk_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic("walk_seg_kernel"),
        "kernel_ms_per_step": {k: round(v[1] / single["steps"], 4) for k, v in single["kernels"].items()},
    }
    # the atomic roofline: one f32 atomic add per voxel update (before lane
    # merging) against the device's measured rate of independent f32 atomic
    # adds at the footprint of the touched regions' accumulator layer
    footprint = max(1, res["stats"]["regions_used"]) * 32768 * 8 * int(round(scans_per_launch))
    ceiling = ohm.probe_atomic_rate(footprint)
    ceiling_seq = ohm.probe_atomic_rate(footprint, sequential=True)
    upd_rate = upd_per_scan * scans_per_launch / (walk_avg_ms * 1e-3)
    roofline["atomic"] = {
        "unit": "voxel updates/s",
        "achieved": round(upd_rate, 1),
        "ceiling_random_f32_atomics_per_s": round(ceiling, 1),
        "ceiling_consecutive_f32_atomics_per_s": round(ceiling_seq, 1),
        "footprint_bytes": footprint,
        # against the best case of the memory-side atomic units (each wave's
        # adds on consecutive words); the random-address rate is the floor
        # an unmerged walk would see
        "frac": round(upd_rate / ceiling_seq, 4),
        "frac_vs_random": round(upd_rate / ceiling, 4),
    }
    log(f"atomic roofline: {upd_rate / 1e9:.2f} G updates/s vs {ceiling_seq / 1e9:.2f} G consecutive "
        f"and {ceiling / 1e9:.2f} G random f32 atomics/s")
    if args.calibrate_copy_mb:
        n = args.calibrate_copy_mb << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.calibrate_copy_mb} MiB three times (byte-counter reference)")
        del src, dst
    headline_batched = None if args.no_batched else run_batched_headline(args, params, batch)
    ndt = None if args.no_ndt else run_ndt(args, params, batch)
    adjoint = None if args.no_adjoint else run_adjoint(args)
    batched = None if args.no_batched else run_batched(args, batched_inputs)
    cpu = None
    if not args.no_cpu_baseline:
        log(f"timing the oracle on {args.cpu_scans} scans")
        cpu = cpu_baseline(params, batch, min(args.cpu_scans, scans))
        log(f"oracle: {cpu['value']:.0f} rays/s")
    out = {
        "metric": "rays/s (voxel-updates/s alongside), plain occupancy through ohm_integrate_rays, "
                  "config-1 spinning-lidar scans",
        "value": round(rays_per_s, 1),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": res["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{scans} spinning-lidar scans x {int(rays_per_scan)} rays (64x2048), tunnel scene, "
                        "0.1 m voxels, 32^3 regions over 200x200x40 m, 30 m max range",
            "mode": "count_clamp",
            "scan_groups": args.scan_group_slots,
            "n_scans": scans,
            "rays_per_scan": int(rays_per_scan),
        },
        "voxel_updates_per_s": round(upd_per_s, 1),
        "voxel_updates_per_step": int(res["updates_per_step"]),
        "kernel_ms_per_step": {k: round(v[1] / res["steps"], 4) for k, v in res["kernels"].items()},
        "one_launch_per_scan": one_launch_per_scan,
        "per_update_mode": per_update,
        "batched_same_scans": headline_batched,
        "batched": batched,
        "ndt": ndt,
        "adjoint": adjoint,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
