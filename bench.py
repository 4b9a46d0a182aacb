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

Reported alongside, each with its roofline: the 32,768-ray single-batch
workload, the per-update (CAS) mode, the occupancy map with the voxel-mean
layer (what the paper's occupancy timings include) and with the decay-rate
layer, NDT-OM, NDT-TM and TSDF integration of the same scans, the adjoint on
the 20-scan 0.2 m workload, and the batched multi-sensor plan against
per-scan launches.  Prints one JSON line on stdout; progress goes to stderr.
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

# Algorithmic bytes per unit of work (the figures the roofline fractions use).
RAY_BYTES = 12.0          # one sample (3 x f32)
SCAN_BYTES = 12.0         # one sensor origin per scan
COUNT_UPDATE_BYTES = 16.0 # count mode: one 8-byte counter read-modify-write at the coherence point
CAS_UPDATE_BYTES = 8.0    # per-update mode: one 4-byte f32 read-modify-write
NDT_MISS_EXTRA = 40.0     # NDT: the voxel's statistics (n, mean, covariance) read by a miss
NDT_SAMPLE_BYTES = 12.0 + 10 * 16.0  # NDT: the sample plus ten 8-byte moment read-modify-writes
ADJ_VISIT_BYTES = 8.0     # adjoint: the voxel's upstream gradient and clamp record per visit


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def walk_bytes(rays, updates, scans=1.0, per_update=COUNT_UPDATE_BYTES):
    """Algorithmic bytes of an occupancy walk: each ray reads its 12-byte
    sample, each scan its 12-byte origin, and each voxel update is one
    counter read-modify-write at the coherence point (16 B in count mode,
    8 B for the per-update mode's f32 compare-and-swap)."""
    return RAY_BYTES * rays + SCAN_BYTES * scans + per_update * updates


def percentiles(ms):
    import numpy as np

    a = np.asarray(ms, np.float64)
    return {"median": round(float(np.median(a)), 5), "p10": round(float(np.percentile(a, 10)), 5),
            "p90": round(float(np.percentile(a, 90)), 5)}


def hbm(bytes_, ms):
    """GB/s and fraction of the published HBM peak for `bytes_` moved in `ms`."""
    gbs = bytes_ / (ms * 1e-3) / 1e9
    return {"achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes": int(bytes_)}


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


def measured_counters(name):
    """Per-launch counter figures of a kernel from its committed summary
    (profiles/<name>_pmc.md), or {} once the kernel sources differ from
    those the counters were taken on."""
    import re

    path = os.path.join(ROOT, "profiles", f"{name}_pmc.md")
    if not os.path.exists(path):
        return {}
    text = open(path).read()
    sha = re.search(r"^kernel_source_sha256:\s*([0-9a-f]{64})", text, re.M)
    if not sha or sha.group(1) != kernel_source_digest():
        return {}
    out = {}
    for key in ("traffic_bytes_per_launch", "atomic_requests_per_launch"):
        m = re.search(rf"^{key}:\s*(\d+)", text, re.M)
        if m:
            out[key] = int(m.group(1))
    return out


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def timed(fn, steps, stream):
    """Run fn() `steps` times with a pair of HIP events around each run on
    `stream`; returns the per-run milliseconds."""
    import torch

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def run_map(args, params, batch, mode, layers=1, call="integrate", steps=None, capacity=None, extra=None,
            column_rays=0):
    """Time `steps` calls of OhmMap.<call> over the whole batch on one map
    (after the warm-up calls); returns per-step times, kernel times and the
    per-step rays and updates.  column_rays: the scans' column layout
    declared to the map (OhmMap.set_scan_layout), 0 for none."""
    import torch

    import paper_2206_06079_amd as ohm

    dev = torch.device("cuda", 0)
    o = torch.from_numpy(batch.origins).to(dev)
    s = torch.from_numpy(batch.samples).to(dev)
    off = batch.offsets
    m = ohm.OhmMap(params.replace(mode=mode), capacity or args.capacity, layers=layers, device=dev)
    if column_rays:
        m.set_scan_layout(column_rays)
    fn_call = getattr(m, call)
    x = extra or ()
    if call == "ndt_tm_integrate":
        fn = lambda: fn_call(o, s, *x, off)  # noqa: E731
    else:
        fn = lambda: fn_call(o, s, off)  # noqa: E731
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    st0 = m.stats()
    steps = steps or args.steps
    # the timed steps run as a caller runs them; per-kernel times come from
    # further steps with the map's event profiling on (its events sit
    # between the launches and would stretch the timed steps)
    ms = timed(fn, steps, stream)
    st1 = m.stats()
    m.set_profiling(True)
    for _ in range(max(1, min(steps, 3))):
        fn()
    torch.cuda.synchronize()
    kt = m.kernel_times()
    kt_steps = max(1, min(steps, 3))
    m.set_profiling(False)
    m.close()
    return {
        "steps": steps,
        "ms": ms,
        "ms_per_step": sum(ms) / steps,
        "rays_per_step": (st1["rays_in"] - st0["rays_in"]) / steps,
        "updates_per_step": (st1["voxel_updates"] - st0["voxel_updates"]) / steps,
        "hits_per_step": (st1["rays_hit"] - st0["rays_hit"]) / steps,
        "kernels": kt,
        "kernel_steps": kt_steps,
        "stats": st1,
    }


def leg_summary(r, workload):
    sec = r["ms_per_step"] * 1e-3
    return {
        "workload": workload,
        "rays_per_s": round(r["rays_per_step"] / sec, 1),
        "voxel_updates_per_s": round(r["updates_per_step"] / sec, 1),
        "ms_per_step": round(r["ms_per_step"], 4),
        "ms_per_step_pct": percentiles(r["ms"]),
        "kernel_ms_per_step": {k: round(v[1] / r["kernel_steps"], 4) for k, v in r["kernels"].items()},
    }


def kernel_avg_ms(r, kind):
    n, ms = r["kernels"].get(kind, (0, 0.0))
    return ms / max(1, n), n


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
    half into a 0.05 m map.  Times graph launches of the batched plan
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
    reps = args.batched_reps
    ms = timed(lambda: plan.run(stream), reps, stream)
    ms_batched = sum(ms) / reps
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

        def one_pass():
            for m, (o, s, off) in zip(maps, inputs):
                m.integrate(o, s, off)

        ms_plain[label] = sum(timed(one_pass, reps, stream)) / reps
        for m in maps:
            m.close()
    log(f"batched {choice}: {ms_batched:.2f} ms per pass; per-scan launches: {ms_plain}")
    pass_bytes = walk_bytes(n_rays, upd, sum(b.n_scans for b in batches))
    return {
        "workload": f"16 sensor streams, {args.batched_scans} scans of log-uniform size in [8192, 262144] rays "
                    f"({n_rays} rays), tunnel scene, maps at 0.1 m and 0.05 m",
        "rays_per_s": round(n_rays / (ms_batched * 1e-3), 1),
        "voxel_updates_per_s": round(upd / (ms_batched * 1e-3), 1),
        "ms_per_pass": round(ms_batched, 3),
        "ms_per_pass_pct": percentiles(ms),
        "schedule": choice,
        "roofline_hbm": hbm(pass_bytes, ms_batched),
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
    reps = max(1, args.steps // 2)
    ms = timed(lambda: plan.run(stream), reps, stream)
    ms_avg = sum(ms) / reps
    st1 = m.stats()
    plan.close()
    m.close()
    rays = (st1["rays_in"] - st0["rays_in"]) / reps
    upd = (st1["voxel_updates"] - st0["voxel_updates"]) / reps
    log(f"headline scans through the batched plan {choice}: {ms_avg:.3f} ms per pass")
    return {
        "workload": f"the same {batch.n_scans} scans through the batched plan (one map)",
        "rays_per_s": round(rays / (ms_avg * 1e-3), 1),
        "voxel_updates_per_s": round(upd / (ms_avg * 1e-3), 1),
        "ms_per_pass": round(ms_avg, 3),
        "ms_per_pass_pct": percentiles(ms),
        "schedule": choice,
        "roofline_hbm": hbm(walk_bytes(rays, upd, batch.n_scans), ms_avg),
    }


def run_config0(args):
    """The single-batch workload: 32,768 rays from the centre of a 20 m cube
    of 0.1 m voxels (every ray starts in the same voxel), count mode, one
    integrate call per step."""
    from workloads import scenes

    import paper_2206_06079_amd as ohm

    mp, batch = scenes.config0()
    r = run_map(args, mp, batch, ohm.MODE_COUNT_CLAMP, steps=max(5, args.steps * 2), capacity=343)
    out = leg_summary(r, "32,768 rays from a voxel corner at the centre of a 20 m cube, 0.1 m voxels, "
                         "ranges U[1, 15] m, one batch per step")
    walk_ms, _ = kernel_avg_ms(r, "walk")
    out["walk_kernel_ms"] = round(walk_ms, 5)
    out["roofline_hbm"] = hbm(walk_bytes(r["rays_per_step"], r["updates_per_step"]), walk_ms)
    log(f"config 0: {r['ms_per_step']:.4f} ms per batch, walk {walk_ms * 1e3:.1f} us")
    return out


def run_layers(args, params, batch):
    """Occupancy with the voxel-mean layer (the paper's occupancy timings
    maintain the mean too) and with the decay-rate layer, scan-grouped like
    the headline."""
    import paper_2206_06079_amd as ohm

    out = {}
    groups = ohm.LAYER_SCAN_GROUPS | ohm.scan_group_slots(args.scan_group_slots)
    for name, layer in (("occupancy_with_mean", ohm.LAYER_MEAN), ("occupancy_with_decay_rate", ohm.LAYER_DECAY)):
        r = run_map(args, params, batch, ohm.MODE_COUNT_CLAMP, ohm.LAYER_OCC | groups | layer,
                    steps=max(2, args.steps // 2), column_rays=args.scan_layout)
        out[name] = leg_summary(r, f"the {batch.n_scans} headline scans, count mode, "
                                   f"{args.scan_group_slots}-scan groups, with the layer")
        log(f"{name}: {r['ms_per_step']:.3f} ms per step")
    return out


def run_ndt(args, params, batch, tm=False):
    """NDT-OM (or NDT-TM) integration of the same 100 scans (sensor noise
    0.05 m, adaptation rate 1, 4 samples before a voxel weights its misses),
    count mode, timed like the plain path."""
    import torch

    import paper_2206_06079_amd as ohm
    from workloads import scenes

    p = params.replace(sensor_noise=0.05, adaptation_rate=1.0, ndt_min_samples=4)
    layers = ohm.LAYER_NDT | (ohm.LAYER_NDT_TM if tm else 0)
    extra = None
    if tm:
        extra = (torch.from_numpy(scenes.lidar_intensities(batch)).to("cuda"),)
    r = run_map(args, p, batch, ohm.MODE_COUNT_CLAMP, layers, call="ndt_tm_integrate" if tm else "ndt_integrate",
                steps=max(2, args.steps // 3), extra=extra)
    name = "NDT-TM" if tm else "NDT-OM"
    out = leg_summary(r, f"the same {batch.n_scans} scans into an {name} map (count mode)")
    walk_ms, n_walk = kernel_avg_ms(r, "walk")
    scans = batch.n_scans
    rays, upd, hits = r["rays_per_step"] / scans, r["updates_per_step"] / scans, r["hits_per_step"] / scans
    walk_b = (RAY_BYTES * rays + SCAN_BYTES + (COUNT_UPDATE_BYTES + NDT_MISS_EXTRA) * (upd - hits)
              + (COUNT_UPDATE_BYTES + NDT_SAMPLE_BYTES) * hits)
    out["kernel_us_per_scan"] = {k: round(v[1] / v[0] * 1e3, 1) for k, v in r["kernels"].items()}
    out["roofline_hbm"] = dict(hbm(walk_b, walk_ms), kernel="ndt_seg_kernel", unit="per scan")
    if not tm:
        counters = measured_counters("ndt_seg_kernel_config2")
        out["roofline_hbm"]["traffic"] = counters.get("traffic_bytes_per_launch")
        out["roofline_hbm"]["atomic_requests"] = counters.get("atomic_requests_per_launch")
    log(f"{name}: {r['ms_per_step']:.3f} ms per {scans}-scan pass")
    return out


def run_tsdf(args, params, batch):
    """TSDF integration of the same 100 scans (band of 0.3 m on each side of
    the sample), count mode."""
    import paper_2206_06079_amd as ohm

    r = run_map(args, params, batch, ohm.MODE_COUNT_CLAMP, ohm.LAYER_TSDF, call="tsdf_integrate",
                steps=max(2, args.steps // 2))
    out = leg_summary(r, f"the same {batch.n_scans} scans into a TSDF layer (count mode, tau = "
                         f"{params.tsdf_truncation} m)")
    walk_ms, _ = kernel_avg_ms(r, "walk")
    scans = batch.n_scans
    out["roofline_hbm"] = dict(hbm(walk_bytes(r["rays_per_step"] / scans, r["updates_per_step"] / scans), walk_ms),
                               kernel="tsdf_kernel", unit="per scan")
    log(f"TSDF: {r['ms_per_step']:.3f} ms per {scans}-scan pass")
    return out


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
    st = None
    for _ in range(4):  # the first pass warms up
        m = ohm.OhmMap(params, 256, layers=ohm.LAYER_NDT | ohm.LAYER_ADJOINT, device=dev)
        e[0].record(stream)
        m.ndt_integrate(o, s, batch.offsets, w)
        e[1].record(stream)
        m.backward(g, box_min, box_dim, o, s, batch.offsets, w, ndt=True, grad_weights=gw)
        e[2].record(stream)
        torch.cuda.synchronize()
        st = m.stats()
        m.close()
        fwd.append(e[0].elapsed_time(e[1]))
        bwd.append(e[1].elapsed_time(e[2]))
    fwd, bwd = fwd[1:], bwd[1:]
    f_ms, b_ms = sum(fwd) / len(fwd), sum(bwd) / len(bwd)
    visits = st["voxel_updates"]
    # the backward re-walks every ray: per visit the gradient and clamp
    # record, plus each voxel's statistics (NDT), and the ray's sample
    bwd_bytes = RAY_BYTES * batch.n_rays + (ADJ_VISIT_BYTES + NDT_MISS_EXTRA) * visits
    log(f"adjoint: forward {f_ms:.2f} ms, backward {b_ms:.2f} ms")
    return {
        "workload": f"{batch.n_scans} scans x {batch.n_rays // batch.n_scans} weighted rays at 0.2 m, NDT, "
                    "64^3 loss box",
        "forward_ms": round(f_ms, 3),
        "backward_ms": round(b_ms, 3),
        "backward_ms_pct": percentiles(bwd),
        "backward_rays_per_s": round(batch.n_rays / (b_ms * 1e-3), 1),
        "voxel_visits": int(visits),
        "roofline_hbm_backward": hbm(bwd_bytes, b_ms),
        # HBM bytes of the backward walk per launch (one scan), from the
        # committed counters, times the scans of a pass
        "traffic_backward_walk": (traffic * batch.n_scans if (traffic := measured_counters(
            "backward_seg_kernel_config4").get("traffic_bytes_per_launch")) else None),
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
        "host": host_cpu(),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scans", type=int, default=100)
    ap.add_argument("--capacity", type=int, default=512)
    ap.add_argument("--scan-layout", type=int, default=64,
                    help="rays per column declared for the grouped legs (the scans are column-major "
                         "64-beam range images; 0: walk them in the given order)")
    ap.add_argument("--scan-group-slots", type=int, default=50,
                    help="accumulator slots of the headline map (scans walked per launch)")
    ap.add_argument("--cpu-scans", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-update", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-ndt", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-layers", action="store_true", help="skip the mean, decay-rate, NDT-TM and TSDF legs")
    ap.add_argument("--no-config0", action="store_true")
    ap.add_argument("--only-headline", action="store_true", help="the headline legs only (profiling runs)")
    ap.add_argument("--only", default="",
                    help="comma list of legs to run besides the headline (profiling runs): per_update, config0, "
                         "batched, layers, ndt, adjoint, cpu")
    ap.add_argument("--batched-scans", type=int, default=1000)
    ap.add_argument("--batched-reps", type=int, default=3)
    ap.add_argument("--batched-groups", type=lambda v: tuple(int(x) for x in v.split(",")), default=(16, 64))
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this size (reference for HBM byte counters)")
    ap.add_argument("--batched-tiles", type=lambda v: tuple(tuple(int(y) for y in x.split("/")) for x in v.split(",")),
                    default=((16, 512), (32, 512)), help="walk tiles K/T,K/T,...")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(how it would shard is described in the design notes)", file=sys.stderr)
        return 2
    if args.only_headline or args.only:
        keep = set(x for x in args.only.split(",") if x)
        unknown = keep - {"per_update", "config0", "batched", "layers", "ndt", "adjoint", "cpu"}
        if unknown:
            ap.error(f"unknown legs {sorted(unknown)}")
        args.no_batched = "batched" not in keep
        args.no_ndt = "ndt" not in keep
        args.no_adjoint = "adjoint" not in keep
        args.no_layers = "layers" not in keep
        args.no_config0 = "config0" not in keep
        args.no_cpu_baseline = "cpu" not in keep
        args.no_per_update = "per_update" not in keep

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

    single = run_map(args, params, batch, ohm.MODE_COUNT_CLAMP)
    log(f"count mode, one launch per scan: {single['ms_per_step']:.3f} ms/step, kernels {single['kernels']}")
    res = run_map(args, params, batch, ohm.MODE_COUNT_CLAMP,
                  ohm.LAYER_OCC | ohm.LAYER_SCAN_GROUPS | ohm.scan_group_slots(args.scan_group_slots),
                  column_rays=args.scan_layout)
    log(f"count mode, {args.scan_group_slots}-scan groups: {res['ms_per_step']:.3f} ms/step, kernels {res['kernels']}")
    scans = args.scans
    rays_per_scan = res["rays_per_step"] / scans
    upd_per_scan = res["updates_per_step"] / scans

    per_update = None
    if not args.no_per_update:
        pu = run_map(args, params, batch, ohm.MODE_PER_UPDATE, steps=max(2, args.steps // 2))
        log(f"per-update mode: {pu['ms_per_step']:.3f} ms/step, kernels {pu['kernels']}")
        per_update = leg_summary(pu, f"the {scans} headline scans, per-update (compare-and-swap) mode, one launch "
                                     "per scan")
        pu_walk, _ = kernel_avg_ms(pu, "walk")
        per_update["walk_kernel_ms"] = round(pu_walk, 5)
        per_update["roofline_hbm"] = dict(hbm(walk_bytes(rays_per_scan, upd_per_scan, per_update=CAS_UPDATE_BYTES),
                                              pu_walk), kernel="walk_seg_kernel<per-update>", unit="per scan")
        # the atomic ceiling of the mode: independent f32 clamp-adds by
        # compare-and-swap at the occupancy layer's footprint
        occ_bytes = max(1, pu["stats"]["regions_used"]) * 32768 * 4
        cas_rand = ohm.probe_atomic_rate(occ_bytes, op="f32_cas")
        cas_seq = ohm.probe_atomic_rate(occ_bytes, sequential=True, op="f32_cas")
        rate = upd_per_scan / (pu_walk * 1e-3)
        per_update["roofline_atomic"] = {
            "unit": "voxel updates/s", "achieved": round(rate, 1),
            "ceiling_random_f32_cas_per_s": round(cas_rand, 1),
            "ceiling_consecutive_f32_cas_per_s": round(cas_seq, 1),
            "frac_vs_random": round(rate / cas_rand, 4), "frac_vs_consecutive": round(rate / cas_seq, 4),
            "footprint_bytes": occ_bytes,
        }
        counters = measured_counters("walk_seg_kernel_per_update_config1")
        per_update["traffic"] = counters.get("traffic_bytes_per_launch")

    # dominant kernel: the group walk
    walk_avg_ms, n_walk = kernel_avg_ms(res, "walk_group")
    single_scans = res["kernels"].get("walk", (0, 0.0))[0] / res["kernel_steps"]
    scans_per_launch = (scans - single_scans) * res["kernel_steps"] / max(1, n_walk)
    launch_rays = rays_per_scan * scans_per_launch
    launch_upd = upd_per_scan * scans_per_launch
    launch_bytes = walk_bytes(launch_rays, launch_upd, scans_per_launch)
    launch_bytes_f32 = walk_bytes(launch_rays, launch_upd, scans_per_launch, per_update=8.0)
    achieved = launch_bytes / (walk_avg_ms * 1e-3) / 1e9
    counters = measured_counters("walk_group_kernel_config1")
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": counters.get("traffic_bytes_per_launch"),
        "kernel": f"walk_group_kernel (count mode, up to {args.scan_group_slots} scans per launch)",
        "kernel_avg_ms": round(walk_avg_ms, 5),
        "scans_per_launch": round(scans_per_launch, 3),
        "bytes_per_launch": launch_bytes,
        "bytes_per_unit": {"ray": RAY_BYTES, "scan": SCAN_BYTES, "voxel_update": COUNT_UPDATE_BYTES},
        # the same launch priced at what its counters are (one 4-byte f32
        # read-modify-write per update, hit and miss counted separately)
        "at_8B_per_update": {"achieved": round(launch_bytes_f32 / (walk_avg_ms * 1e-3) / 1e9, 1),
                             "frac": round(launch_bytes_f32 / (walk_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }
    # the device's measured streaming bandwidth (1 GiB copy and read, well
    # beyond the last-level cache) beside the published peak
    stream_copy = ohm.probe_stream_rate(1 << 30) / 1e9
    stream_read = ohm.probe_stream_rate(1 << 30, read_only=True) / 1e9
    roofline["measured_stream"] = {"copy_gbs": round(stream_copy, 1), "read_gbs": round(stream_read, 1),
                                   "frac_vs_copy": round(achieved / stream_copy, 4)}
    log(f"stream: copy {stream_copy:.0f} GB/s, read {stream_read:.0f} GB/s")
    s_walk_avg, _ = kernel_avg_ms(single, "walk")
    one_launch_per_scan = leg_summary(single, f"the {scans} headline scans, one walk launch per scan")
    one_launch_per_scan.update({
        "kernel": "walk_seg_kernel",
        "kernel_avg_ms": round(s_walk_avg, 5),
        "roofline_hbm": hbm(walk_bytes(rays_per_scan, upd_per_scan), s_walk_avg),
        "traffic": measured_counters("walk_seg_kernel_config1").get("traffic_bytes_per_launch"),
    })
    # the atomic roofline: one counter update per voxel update (before lane
    # merging) against the device's measured rate of independent f32 atomic
    # adds at the footprint of the group's accumulator slots
    footprint = max(1, res["stats"]["regions_used"]) * 32768 * 8 * int(round(scans_per_launch))
    ceiling = ohm.probe_atomic_rate(footprint)
    ceiling_seq = ohm.probe_atomic_rate(footprint, sequential=True)
    ceiling_u64 = ohm.probe_atomic_rate(footprint, op="u64_add")
    upd_rate = launch_upd / (walk_avg_ms * 1e-3)
    requests = counters.get("atomic_requests_per_launch")
    roofline["atomic"] = {
        "unit": "voxel updates/s",
        "achieved": round(upd_rate, 1),
        "ceiling_random_f32_atomics_per_s": round(ceiling, 1),
        "ceiling_consecutive_f32_atomics_per_s": round(ceiling_seq, 1),
        "ceiling_random_u64_atomics_per_s": round(ceiling_u64, 1),
        "footprint_bytes": footprint,
        # updates per second against the distinct-address rate: above 1 only
        # because lane merging and the tile tables combine updates first
        "frac_vs_random": round(upd_rate / ceiling, 4),
        "frac_vs_consecutive": round(upd_rate / ceiling_seq, 4),
        # what reaches memory: the L2 atomic requests per launch (counter
        # TCC_ATOMIC), their share of the updates and their rate
        "atomic_requests_per_launch": requests,
        "merge_factor": round(launch_upd / requests, 2) if requests else None,  # updates per atomic request
        "request_rate_per_s": round(requests / (walk_avg_ms * 1e-3), 1) if requests else None,
        "request_frac_vs_random": round(requests / (walk_avg_ms * 1e-3) / ceiling, 4) if requests else None,
    }
    log(f"roofline: {achieved:.0f} GB/s at 16 B per update ({achieved / HBM_PEAK_GBS:.3f} of peak); "
        f"{upd_rate / 1e9:.2f} G updates/s vs {ceiling / 1e9:.2f} G random f32 atomics/s")
    if args.calibrate_copy_mb:
        n = args.calibrate_copy_mb << 18  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.calibrate_copy_mb} MiB three times (byte-counter reference)")
        del src, dst
    config0 = None if args.no_config0 else run_config0(args)
    headline_batched = None if args.no_batched else run_batched_headline(args, params, batch)
    layers = None if args.no_layers else run_layers(args, params, batch)
    ndt = None if args.no_ndt else run_ndt(args, params, batch)
    ndt_tm = None if (args.no_ndt or args.no_layers) else run_ndt(args, params, batch, tm=True)
    tsdf = None if args.no_layers else run_tsdf(args, params, batch)
    adjoint = None if args.no_adjoint else run_adjoint(args)
    batched = None if args.no_batched else run_batched(args, batched_inputs)
    cpu = None
    if not args.no_cpu_baseline:
        log(f"timing the oracle on {args.cpu_scans} scans")
        cpu = cpu_baseline(params, batch, min(args.cpu_scans, scans))
        log(f"oracle: {cpu['value']:.0f} rays/s")
    sec = res["ms_per_step"] * 1e-3
    out = {
        "metric": "rays/s (voxel-updates/s alongside), scan-grouped occupancy integration through "
                  "ohm_integrate_rays (50 scans per walk launch), config-1 spinning-lidar scans",
        "value": round(res["rays_per_step"] / sec, 1),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": res["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "ms_per_step_pct": percentiles(res["ms"]),
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
            "scan_layout_column_rays": args.scan_layout,
            "n_scans": scans,
            "rays_per_scan": int(rays_per_scan),
        },
        "voxel_updates_per_s": round(res["updates_per_step"] / sec, 1),
        "voxel_updates_per_step": int(res["updates_per_step"]),
        "kernel_ms_per_step": {k: round(v[1] / res["kernel_steps"], 4) for k, v in res["kernels"].items()},
        "one_launch_per_scan": one_launch_per_scan,
        "config0": config0,
        "per_update_mode": per_update,
        "batched_same_scans": headline_batched,
        "batched": batched,
        "layers": layers,
        "ndt": ndt,
        "ndt_tm": ndt_tm,
        "tsdf": tsdf,
        "adjoint": adjoint,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
