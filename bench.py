"""Throughput of the event-manifold reconstruction on one MI355X.

Workload: 240x180 sensor, rotating + translating Gaussian-blob texture at
~1e6 signal events/s plus 1 % uniform noise events, a 2 s stream cut into
blocks of 1000 events; every step pushes one block (events already resident
in device memory) and solves it with 50 primal-dual iterations (lambda 90,
contrast threshold 0.2).  Prints one JSON line.

  value        PD iter*Mpix/s = steps * 50 * 240*180 / timed seconds / 1e6
  events_per_s events consumed per timed second
  roofline     the primal-dual kernel: algorithmic bytes (44 B per pixel-
               iteration: read u, p, f, tx, ty; write u, p) per second of
               kernel time, against 8 TB/s HBM
  cpu_baseline the FP64 C oracle, single thread, on the first blocks of the
               same stream (about 10 s of CPU work)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PD iter*Mpix/s and events/s at 50 it/batch; fwd+bwd vs plain; %HBM BW"
HBM_PEAK_GBS = 8000.0
BYTES_PER_PX_ITER = 44  # u 4 + p 12 + f 4 + tx/ty 8 read, u 4 + p 12 written
BYTES_PER_PX_ITER_16 = 28  # same with p and tx/ty stored in 16 bits
# HBM traffic of the fused kernel from rocprofv3 --pmc runs (FETCH_SIZE and
# WRITE_SIZE in separate runs, KiB per dispatch averaged over the kernel's
# dispatches), scaled by the same counters' reading for a 256 MiB device
# copy: FETCH_SIZE read 131084 KiB and WRITE_SIZE 262144 KiB for 262144 KiB
# moved each way, so fetched bytes = 2 x 1024 x FETCH_SIZE and written bytes
# = 1024 x WRITE_SIZE.  Each entry holds for the kernel sources it was taken
# with (hash of kernels.hip, pd_math.h, kernels.h, tile.h, and shape.h,
# which picks the default tile); after a change the bench reports traffic
# null until the counters are taken again.
TRAFFIC_SOURCES = ("kernels.hip", "pd_math.h", "kernels.h", "tile.h", "shape.h")
MEASURED_TRAFFIC = {
    # (workload, storage): (source hash, fetched bytes, written bytes) per launch
    ("davis240", "f32"): ("cdb8079d22c58ad3", 2 * 1024 * 1071.9, 1024 * 820.7),
    ("probe", "f32"): ("cdb8079d22c58ad3", 2 * 1024 * 553205.9, 1024 * 545699.2),
    # the probe with one iteration per launch on 2 x 8 x 64 tiles
    ("probe_k1", "f32"): ("cdb8079d22c58ad3", 2 * 1024 * 409075.7, 1024 * 477091.9),
    # the batched solve of all 64 cameras: bytes of one whole solve (every
    # launch of every class chain), for the class geometries below
    ("streams64", "f32"): ("cdb8079d22c58ad3", 2 * 1024 * 814279.2, 1024 * 1070089.7),
}
# class geometries the 64-camera counters were taken with: (width, height of
# the class's first camera, rows, waves, columns, iterations per launch)
STREAMS64_MEASURED_SHAPE = [(640, 480, 8, 8, 64, 6), (240, 180, 8, 8, 64, 8),
                            (346, 260, 8, 8, 64, 9), (128, 128, 8, 8, 64, 10)]
STREAMS64_PINNED = "640x480:8x8x64:6,240x180:8x8x64:8,346x260:8x8x64:9,128x128:8x8x64:10"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1607_06283_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


W_, H_ = 240, 180
EVENTS_PER_BATCH = 1000
ITERS = 50

# Other shapes for kernel measurements (same JSON line format; the default
# workload above is the one the headline figure is quoted on):
#   hd720  1280x720 sensor, ~2e7 events/s, blocks of 20000 events, 100 iterations
#   probe  5120x5760 frame (29.5 Mpx, ~1.8 GB of state: beyond the 256 MB
#          Infinity Cache), uniform random events, blocks of 20000, 50 iterations
WORKLOADS = {
    "davis240": (240, 180, 1000, 50),
    "hd720": (1280, 720, 20000, 100),
    "probe": (5120, 5760, 20000, 50),
    "streams64": (0, 0, 0, 50),
    "diff16": (346, 260, 2000, 100),
    "frame": (0, 0, 1000, 50),  # size from --frame
}
#   streams64  64 independent cameras: 16 each of 128x128, 240x180, 346x260 and
#          640x480 (7.3 Mpx, ~440 MB of state: beyond the Infinity Cache);
#          per camera an event rate log-uniform in [1e5, 5e6] /s and a block
#          size log-uniform in [200, 5000] events (seeded); uniform random
#          pixels and polarities, exponential inter-event times at that rate;
#          50 iterations per block; all cameras solved by one batched launch
#          sequence (autotuned tiles), compared with per-camera solves.


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def load_stream(n_batches: int):
    """The calibrated 240x180 stream, long enough for n_batches blocks (cached in /tmp)."""
    import evgen

    duration = max(2_000_000, int(math.ceil(n_batches * EVENTS_PER_BATCH / 1e6 * 1e6 * 1.02)))
    key = hashlib.sha1(f"davis240-seed2-{duration}".encode()).hexdigest()[:12]
    path = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"evrec_stream_{key}.npz")
    if os.path.exists(path):
        z = np.load(path)
        return evgen.Events(z["t"], z["x"], z["y"], z["p"], z["n"])
    s, _, _, _ = evgen.davis240(seed=2, duration_us=duration)
    ev = s.events
    try:
        np.savez(path, t=ev.t, x=ev.x, y=ev.y, p=ev.p, n=ev.is_noise)
    except OSError:
        pass
    return ev


def random_stream(W, H, n, seed=7):
    """Uniform random events (pixel, polarity), timestamps 1 us apart."""
    import evgen

    rng = np.random.default_rng(seed)
    t = evgen.T0_US + np.arange(n, dtype=np.int64)
    x = rng.integers(0, W, n).astype(np.uint16)
    y = rng.integers(0, H, n).astype(np.uint16)
    p = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    return evgen.Events(t, x, y, p, np.zeros(n, np.uint8))


def hd720_stream(n_batches):
    import evgen

    key = f"hd720-seed3-{n_batches}"
    path = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"evrec_stream_{key}.npz")
    if os.path.exists(path):
        z = np.load(path)
        return evgen.Events(z["t"], z["x"], z["y"], z["p"], z["n"])
    dur = max(500_000, int(n_batches * 20000 / 2e7 * 1e6 * 1.05))
    s, _, _, _ = evgen.hd720(seed=3, duration_us=dur)
    ev = s.events
    try:
        np.savez(path, t=ev.t, x=ev.x, y=ev.y, p=ev.p, n=ev.is_noise)
    except OSError:
        pass
    return ev


def run_gpu(ev, steps, warmup, fuse, profile, shape=(W_, H_), batch=EVENTS_PER_BATCH,
            iters=ITERS, rows=0, waves=0, storage=0, tvl1=0, cols=0, host_events=False):
    """Push + solve `steps` blocks after `warmup`.  The events are resident in
    device memory and pushed as device pointers, or with host_events pushed
    from host memory (the library stages them and copies them over PCIe)."""
    import torch
    from paper_1607_06283_amd import rec

    dev = torch.device("cuda", 0)
    if host_events:
        arrs = [np.ascontiguousarray(a) for a in (ev.t, ev.x, ev.y, ev.p)]
        base = [a.ctypes.data for a in arrs]
        on_dev = 0
    else:
        arrs = [torch.from_numpy(ev.t).to(dev), torch.from_numpy(ev.x.view(np.int16)).to(dev),
                torch.from_numpy(ev.y.view(np.int16)).to(dev), torch.from_numpy(ev.p).to(dev)]
        base = [a.data_ptr() for a in arrs]
        on_dev = 1
    r = rec.Reconstructor(shape[0], shape[1], fuse_iters=fuse, tile_rows=rows, tile_waves=waves,
                          tile_cols=cols, storage=storage, tvl1_iters=tvl1)
    B = batch

    def step(i):
        a = i * B
        rc = rec.rec_push_events(r.ctx, base[0] + 8 * a, base[1] + 2 * a, base[2] + 2 * a,
                                 base[3] + a, B, on_dev)
        if rc:
            raise rec.RecError(rc, "rec_push_events")
        rc, _ = rec.rec_solve(r.ctx, iters, False)
        if rc:
            raise rec.RecError(rc, "rec_solve")

    for i in range(warmup):
        step(i)
    r.sync()
    torch.cuda.synchronize()
    if profile:
        rec.rec_profile(r.ctx, True)
    t0 = time.perf_counter()
    for i in range(warmup, warmup + steps):
        step(i)
    torch.cuda.synchronize()
    r.sync()
    dt = time.perf_counter() - t0
    prof = rec.rec_profile_read(r.ctx) if profile else None
    u = r.image(rec.REC_U)
    r.close()
    return dt, prof, u


def streams64(steps, seed=400):
    """Per-camera (W, H, block size, events) for the 64-camera workload."""
    import evgen

    return evgen.streams64(steps, seed)


BATCH_MODES = {"serial": 0, "streams": 1, "graph": 2}


def run_streams64(steps, warmup, iters, tune=True, modes=("streams", "serial", "graph"),
                  geometry=None, per_camera=True, profile=True, host_events=False):
    """Time `steps` blocks of all 64 cameras: the batched solve in each of
    `modes` (each pass after 2 warm-up blocks of its own; the first listed
    is also profiled), then one solve per camera.  The events are resident
    in device memory and pushed as device pointers, or with host_events
    pushed from host memory.  Returns per-pass seconds, the profile of the
    first mode, the class configuration, the pixel count and the events per
    block."""
    import torch
    from paper_1607_06283_amd import rec

    passes = len(modes) + int(per_camera) + int(profile)
    cams = streams64(warmup + passes * (steps + 2))
    dev = torch.device("cuda", 0)
    recs, bufs = [], []
    for W, H, bs, ev in cams:
        recs.append(rec.Reconstructor(W, H))
        if host_events:
            arrs = [np.ascontiguousarray(a) for a in (ev.t, ev.x, ev.y, ev.p)]
            bufs.append((arrs, [a.ctypes.data for a in arrs], bs))
        else:
            arrs = [torch.from_numpy(ev.t).to(dev), torch.from_numpy(ev.x.view(np.int16)).to(dev),
                    torch.from_numpy(ev.y.view(np.int16)).to(dev), torch.from_numpy(ev.p).to(dev)]
            bufs.append((arrs, [a.data_ptr() for a in arrs], bs))
    on_dev = 0 if host_events else 1
    batch = rec.Batch(recs, tune_iters=iters if tune and not geometry else 0)
    for g in geometry or ():
        batch.set_geometry(*g)
    block = [0]

    def step(batched):
        i = block[0]
        block[0] += 1
        for r, (_, base, bs) in zip(recs, bufs):
            a = i * bs
            rc = rec.rec_push_events(r.ctx, base[0] + 8 * a, base[1] + 2 * a, base[2] + 2 * a,
                                     base[3] + a, bs, on_dev)
            if rc:
                raise rec.RecError(rc, "rec_push_events")
        if batched:
            batch.solve(iters)
        else:
            for r in recs:
                rc, _ = rec.rec_solve(r.ctx, iters, False)
                if rc:
                    raise rec.RecError(rc, "rec_solve")

    def timed_pass(batched, n_warm=2):
        for _ in range(n_warm):
            step(batched)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step(batched)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    for _ in range(warmup):
        step(True)
    out = {}
    for m in modes:
        batch.set_mode(BATCH_MODES[m])
        out[m] = timed_pass(True)
    batch.set_mode(BATCH_MODES[modes[0]])
    prof = None
    if profile:
        rec.rec_profile(recs[0].ctx, True)
        timed_pass(True)
        prof = rec.rec_profile_read(recs[0].ctx)
        rec.rec_profile(recs[0].ctx, False)
    if per_camera:
        out["per_camera"] = timed_pass(False)
    cfg = batch.config()
    px = sum(W * H for W, H, _, _ in cams)
    ev_per_step = sum(bs for _, _, bs, _ in cams)
    batch.close()
    for r in recs:
        r.close()
    return out, prof, cfg, px, ev_per_step


def streams64_result(steps, warmup, iters, tune=True, modes=("streams", "serial", "graph"),
                     geometry=None, per_camera=True, profile=True, host_events=False):
    """The 64-camera workload: the batched solve in its default mode (the
    first of the timed modes) with the other modes and one solve per camera
    beside it, the class geometries, and the roofline of the batched launch."""
    dts, prof, cfg, px, evs = run_streams64(steps, warmup, iters, tune=tune, modes=modes,
                                            geometry=geometry, per_camera=per_camera,
                                            profile=profile, host_events=host_events)
    dt = dts[modes[0]]
    rate = lambda d: round(steps * iters * px / d / 1e6, 2)
    res = {
        "value": rate(dt), "ms_per_step": round(dt / steps * 1e3, 4),
        "events_per_s": round(steps * evs / dt, 1),
        "modes": {m: {"PD iter*Mpix/s": rate(d), "ms_per_step": round(d / steps * 1e3, 4)}
                  for m, d in dts.items() if m != "per_camera"},
        "classes": [{k: (round(v, 1) if isinstance(v, float) else v) for k, v in c.items()}
                    for c in cfg],
    }
    if per_camera:
        res["per_camera_solves"] = {"PD iter*Mpix/s": rate(dts["per_camera"]),
                                    "ms_per_step": round(dts["per_camera"] / steps * 1e3, 4)}
        res["batched_speedup"] = round(dts["per_camera"] / dt, 3)
    if profile:
        res["roofline"] = batch_roofline(dt / steps, px * iters, cfg, prof)
    return res


def batch_roofline(step_s, px_iters, cfg, prof):
    """Roofline of the batched solve, whose class chains run concurrently:
    algorithmic bytes (44 per pixel-iteration) of one solve over the wall
    time of one solve; traffic = the counters' HBM bytes of one solve (all
    class launches) over the same time, when they were taken for these
    sources and class geometries.  The per-launch kernel times (events in
    the launch packets, overlapping across classes) are given beside it."""
    achieved = BYTES_PER_PX_ITER * px_iters / step_s / 1e9
    shapes = [(c["width"], c["height"], c["rows"], c["waves"], c["cols"], c["kiters"])
              for c in cfg]
    m = MEASURED_TRAFFIC.get(("streams64", "f32"))
    traffic = None
    if m and m[0] == kernel_source_hash() and shapes == STREAMS64_MEASURED_SHAPE:
        traffic = round((m[1] + m[2]) / step_s / 1e9, 1)
    solves = max(1.0, prof.pd_pixel_iters / px_iters)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_frac": None if traffic is None else round(traffic / HBM_PEAK_GBS, 4),
            "kernel": "k_pd_fused_batch, all class chains of one solve (wall time per solve)",
            "bytes_per_px_iter": BYTES_PER_PX_ITER,
            "algorithmic_bytes_per_solve": BYTES_PER_PX_ITER * px_iters,
            "kernel_us_sum_per_solve": round(prof.ms[2] * 1e3 / solves, 1),
            "launches_per_solve": round(prof.launches[2] / solves, 2)}


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads() -> int:
    """Threads the OpenMP oracle build runs with (OMP_NUM_THREADS, else all cores)."""
    try:
        return int(os.environ.get("OMP_NUM_THREADS", "")) or os.cpu_count() or 1
    except ValueError:
        return os.cpu_count() or 1


def _oracle_rate(ev, budget_s, W, H, batch, iters, threads):
    import oracle

    o = oracle.Oracle(oracle.Params(W, H), threads=threads)
    n = 0
    t0 = time.perf_counter()
    while True:
        b = ev.slice(n * batch, (n + 1) * batch)
        o.push_events(b)
        o.solve(iters)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or (n + 1) * batch > len(ev):
            break
    o.close()
    return n, el


def cpu_baseline(ev, budget_s=8.0, W=W_, H=H_, batch=EVENTS_PER_BATCH, iters=ITERS):
    """The FP64 C oracle on the first blocks of the same stream: its OpenMP
    build on all host cores (the reported value) and the single-threaded
    build beside it, each for about budget_s seconds."""
    cores = oracle_threads()
    n, el = _oracle_rate(ev, budget_s, W, H, batch, iters, threads=True)
    n1, el1 = _oracle_rate(ev, budget_s, W, H, batch, iters, threads=False)
    rate = n * iters * W * H / el / 1e6
    rate1 = n1 * iters * W * H / el1 / 1e6
    return {"value": round(rate, 3), "unit": "PD iter*Mpix/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} blocks of the same stream ({n * batch} events, "
                      f"{n * iters} iterations of {W}x{H}) in {el:.1f} s, FP64 C, OpenMP over "
                      f"pixels on {cores} threads",
            "events_per_s": round(n * batch / el, 1),
            "host_cpu": host_cpu_model(), "host_logical_cpus": os.cpu_count(),
            "single_thread": {"value": round(rate1, 3), "events_per_s": round(n1 * batch / el1, 1),
                              "sample": f"first {n1} blocks in {el1:.1f} s"}}


def oracle_c1_c3_c5():
    """The oracle (all host cores) on the 128x128 workload in full (20 blocks
    of 500 events, 50 iterations), on the first 10 blocks of the 1280x720
    workload (20000 events, 100 iterations each) and on the forward of the
    differentiation workload (16 x 346x260, 100 iterations from
    u0 = exp(L_gt(t0)))."""
    import evgen
    import oracle

    out = {}
    s, _, _, _ = evgen.hd720(seed=3, duration_us=11000)
    o = oracle.Oracle(oracle.Params(1280, 720), threads=True)
    blks = evgen.batches(s.events, 20000)[:10]
    t0 = time.perf_counter()
    for b in blks:
        o.push_events(b)
        o.solve(100)
    el = time.perf_counter() - t0
    o.close()
    out["hd720_first10"] = {"s": round(el, 3), "blocks": len(blks),
                            "PD iter*Mpix/s": round(len(blks) * 100 * 1280 * 720 / el / 1e6, 2),
                            "events_per_s": round(len(blks) * 20000 / el, 1)}
    s, bs, nb, iters = evgen.dvs128(seed=1, n_batches=20)
    o = oracle.Oracle(oracle.Params(128, 128), threads=True)
    t0 = time.perf_counter()
    for b in evgen.batches(s.events, bs)[:nb]:
        o.push_events(b)
        o.solve(iters)
    el = time.perf_counter() - t0
    o.close()
    out["dvs128_full"] = {"s": round(el, 3), "PD iter*Mpix/s": round(nb * iters * 128 * 128 / el / 1e6, 2),
                          "events_per_s": round(nb * bs / el, 1), "ms_per_image": round(el / nb * 1e3, 3)}
    blocks = evgen.diff_blocks(500, 16, 346, 260, 2000)
    t0 = time.perf_counter()
    for spec, blk, L0, _ in blocks:
        o = oracle.Oracle(oracle.Params(346, 260), u0=np.exp(L0).astype(np.float32).astype(np.float64),
                          threads=True)
        o.push_events(blk)
        o.solve(100)
        o.close()
    el = time.perf_counter() - t0
    out["diff16_forward"] = {"s": round(el, 3),
                             "PD iter*Mpix/s": round(16 * 100 * 346 * 260 / el / 1e6, 2)}
    return out


def copy_probe(mib=256, reps=5):
    """Plain copy of a known size: each launch reads and writes `mib` MiB, so
    the profiler's FETCH_SIZE / WRITE_SIZE per dispatch can be scaled to bytes."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                      "reps": reps, "GBps_read_plus_write": round(2 * n * 4 / dt / 1e9, 1)}),
          flush=True)


# Grids of the sync probe: the 240x180 workload's fused launch (234 tiles of
# 32x32 pixels, 1024 threads), and 512 workgroups of 512 threads, the most
# that are co-resident with the 64-camera batched launch's 8x8 tiles (two
# per compute unit), which a persistent form of that launch would run.
SYNC_PROBE_GRIDS = [(234, 1024), (512, 512)]


def sync_probe():
    import subprocess

    exe = os.path.join(ROOT, "paper_1607_06283_amd", "sync_probe")
    if not os.path.exists(exe):
        raise SystemExit(f"{exe} is missing: run paper_1607_06283_amd.build.build()")
    for nb, nt in SYNC_PROBE_GRIDS:
        log(f"bench: sync probe {nb} x {nt}")
        out = subprocess.run([exe, str(nb), str(nt)], capture_output=True, text=True, timeout=120)
        if out.returncode != 0:
            raise SystemExit(f"sync_probe failed ({out.returncode}): {out.stderr.strip()}")
        print(out.stdout.strip(), flush=True)


def main_streams64(args):
    steps = min(args.steps, 40)
    warmup = min(args.warmup, 5)
    IT = WORKLOADS["streams64"][3]
    log("bench: 64 cameras (batched in each mode, then one solve per camera)")
    geometry = parse_geometry(args.batch_geometry) if args.batch_geometry else None
    modes = tuple(args.batch_modes.split(","))
    r = streams64_result(steps, warmup, IT, tune=not args.no_tune, modes=modes, geometry=geometry,
                         per_camera=not args.no_per_camera, profile=not args.no_profile,
                         host_events=args.host_events)
    out = {
        "metric": METRIC, "value": r.pop("value"), "unit": "PD iter*Mpix/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": r.pop("ms_per_step"),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "storage": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["streams64"], "cameras": 64,
                   "iters_per_batch": IT, "autotuned": not (args.no_tune or geometry),
                   "mode": modes[0], "events_from": "host" if args.host_events else "device"},
    }
    out.update(r)
    print(json.dumps(out), flush=True)


# Algorithmic bytes per pixel-iteration of the differentiable solve's kernels
# (FP32 planes): forward primal (u, p, f, tx, ty, w read; u written) 36,
# forward dual (u twice, p, tx, ty read; p written) 40; reverse dual (u
# twice, p, tx, ty, q, ub read; q written) 56; reverse primal (u, p, f, tx,
# ty, w, q, uh, two sums read; ub, uh, two sums written) 72.
DIFF_FWD_B = 76
DIFF_REV_B = 128


def main_diff16(args):
    """16 x 346x260 blocks of 2000 events, 100 unrolled iterations, loss
    1/2 sum (log u_100 - L_gt(t_end))^2, checkpoints every 10: forward +
    backward against the library's batched forward solve of the same size."""
    import torch
    import evgen
    from paper_1607_06283_amd import rec

    K, CK, W, H, NB = 100, 10, 346, 260, 16
    steps = max(1, min(args.steps, 20))
    warmup = max(1, min(args.warmup, 3))
    log("bench: diff16 inputs")
    blocks = evgen.diff_blocks(500, NB, W, H, 2000)
    dev = torch.device("cuda", 0)
    npos, nneg, tx, ty = [], [], [], []
    recs = []
    for spec, blk, _, _ in blocks:
        r = rec.Reconstructor(W, H)
        r.push(blk.t, blk.x, blk.y, blk.p)
        npos.append(r.image(rec.REC_COUNT_POS))
        nneg.append(r.image(rec.REC_COUNT_NEG))
        r.solve(1)
        tx.append(r.image(rec.REC_TX))
        ty.append(r.image(rec.REC_TY))
        recs.append(r)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(np.stack(a))).to(dev)
    npos, nneg, tx, ty = T(npos), T(nneg), T(tx), T(ty)
    u0 = T([np.exp(b[2]).astype(np.float32) for b in blocks])
    L = T([b[3] for b in blocks])
    theta = torch.tensor([90.0, 0.2, 0.2], dtype=torch.float64, device=dev, requires_grad=True)
    w = torch.ones((NB, H, W), dtype=torch.float32, device=dev, requires_grad=True)
    out = {}

    def fwd_bwd():
        theta.grad = None
        w.grad = None
        u, _ = rec.unrolled(u0, npos, nneg, tx, ty, theta, K, w=w, ckpt_every=CK)
        loss = 0.5 * ((torch.log(u.double()) - L) ** 2).sum()
        loss.backward()
        out["loss"] = loss

    def fwd():
        with torch.no_grad():
            rec.unrolled(u0, npos, nneg, tx, ty, theta, K, w=w, ckpt_every=CK)

    def fwd_bwd_all_states():
        theta.grad = None
        w.grad = None
        u, _ = rec.unrolled(u0, npos, nneg, tx, ty, theta, K, w=w, ckpt_every=1)
        (0.5 * ((torch.log(u.double()) - L) ** 2).sum()).backward()

    batch = rec.Batch(recs, tune_iters=K)

    def plain():
        batch.solve(K)

    def timeit(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    log("bench: diff16 forward+backward")
    t_fb = timeit(fwd_bwd)
    t_f = timeit(fwd)
    t_all = timeit(fwd_bwd_all_states)
    log("bench: diff16 plain batched forward")
    t_p = timeit(plain)
    g_th = theta.grad.cpu().numpy()
    px = NB * W * H
    C = math.ceil(K / CK)
    bytes_fb = px * (K * DIFF_FWD_B + (K - C) * DIFF_FWD_B + K * DIFF_REV_B)
    achieved = bytes_fb / t_fb / 1e9
    res = {
        "metric": METRIC, "value": round(px * K / t_fb / 1e6, 2), "unit": "PD iter*Mpix/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(t_fb * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["diff16"], "images": NB, "width": W, "height": H,
                   "iters": K, "ckpt_every": CK},
        "fwd_bwd_ms": round(t_fb * 1e3, 3), "diff_fwd_ms": round(t_f * 1e3, 3),
        "plain_fwd_ms": round(t_p * 1e3, 3), "fwd_bwd_over_plain": round(t_fb / t_p, 2),
        "fwd_bwd_ms_every_state_kept": round(t_all * 1e3, 3),
        "loss": float(out["loss"].item()),
        "grad_theta": [float(v) for v in g_th],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "all kernels of forward + reverse sweep (wall clock)"},
    }
    batch.close()
    for r in recs:
        r.close()
    print(json.dumps(res), flush=True)


WORKLOAD_TEXT = {
    "diff16": "16 blocks of 2000 events from 346x260 streams (seeds 500-515), 100 unrolled FP32 "
              "primal-dual iterations from u0 = exp(L_gt(t0)), loss 1/2 sum (log u - L_gt)^2, "
              "gradients for lambda, Delta+, Delta- and per-pixel weights, checkpoints every 10",
    "streams64": "64 cameras (16 each of 128x128, 240x180, 346x260, 640x480), rates log-uniform "
                 "in [1e5, 5e6] events/s, blocks log-uniform in [200, 5000] events, uniform random "
                 "events, 50 FP32 primal-dual iterations per block, all cameras in one batched "
                 "launch sequence with autotuned tiles",
    "davis240": "240x180 sensor, rotating+translating texture, ~1e6 signal events/s + 1% noise, "
                "blocks of 1000 events, 50 FP32 primal-dual iterations per block, lambda 90, "
                "threshold 0.2",
    "hd720": "1280x720 sensor, rotating+translating texture, ~2e7 events/s, blocks of 20000 "
             "events, 100 FP32 primal-dual iterations per block, lambda 90, threshold 0.2",
    "probe": "5120x5760 frame (29.5 Mpx), uniform random events, blocks of 20000 events, 50 FP32 "
             "primal-dual iterations per block, lambda 90",
    "frame": "{w}x{h} frame, uniform random events, blocks of 1000 events, 50 FP32 primal-dual "
             "iterations per block, lambda 90",
}


def parse_frame(text):
    w, h = (int(v) for v in text.lower().split("x"))
    if not (1 <= w <= 65535 and 1 <= h <= 65535):
        raise SystemExit(f"--frame {text}: width and height in 1..65535")
    return w, h


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1980)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--fuse", type=int, default=-1,
                    help="iterations per fused launch (-1: chosen by the library, 0: unfused)")
    ap.add_argument("--rows", type=int, default=0, help="rows per lane of the fused tile (0: auto)")
    ap.add_argument("--waves", type=int, default=0, help="wavefronts per fused workgroup (0: auto)")
    ap.add_argument("--cols", type=int, default=0,
                    help="fused tile width, 64 or 32 (0: auto; needs --rows/--waves)")
    ap.add_argument("--workload", default="davis240", choices=sorted(WORKLOADS))
    ap.add_argument("--frame", default="640x480",
                    help="WxH of the 'frame' workload (uniform random events, 1000 per block)")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"],
                    help="storage of the dual field and time differences (arithmetic is FP32)")
    ap.add_argument("--tvl1", type=int, default=0,
                    help="TV-L1 timestamp-denoising iterations before each block's metric")
    ap.add_argument("--host-events", action="store_true",
                    help="push the events from host memory (PCIe-inclusive rate) instead of "
                         "from device memory")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel timing pass")
    ap.add_argument("--no-extras", action="store_true",
                    help="davis240: skip the 128x128, 64-camera and probe sections and the "
                         "oracle's 128x128 / differentiation-forward timings")
    ap.add_argument("--no-tune", action="store_true",
                    help="streams64: keep the default tile geometry instead of autotuning")
    ap.add_argument("--batch-geometry", default="",
                    help="streams64: fixed geometries instead of the autotuner, e.g. "
                         "640x480:8x8x64:6,240x180:8x8x64:8 (size:rows x waves x cols:K)")
    ap.add_argument("--batch-modes", default="streams,serial,graph",
                    help="streams64: launch modes to time, the first is the reported value")
    ap.add_argument("--no-per-camera", action="store_true",
                    help="streams64: skip the one-solve-per-camera comparison")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 256 MiB device-to-device copy (calibrates HBM byte counters)")
    ap.add_argument("--sync-probe", action="store_true",
                    help="only time the launch-to-launch and grid-barrier alternatives on the "
                         "240x180 fused launch's grid and on a co-resident grid at the 64-camera "
                         "scale (runs the sync_probe program built beside the library)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the reconstruction of one event stream runs on "
              "a single MI355X here (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe()
        return
    if args.sync_probe:
        return sync_probe()
    if args.workload == "diff16":
        if args.host_events:
            raise SystemExit("--host-events: the diff16 workload takes its events as device tensors")
        return main_diff16(args)
    if args.workload == "streams64":
        return main_streams64(args)
    need = args.warmup + args.steps
    W, H, B, IT = WORKLOADS[args.workload]
    if args.workload == "frame":
        W, H = parse_frame(args.frame)
    log(f"bench: generating {args.workload} stream for {need} blocks")
    if args.workload == "davis240":
        ev = load_stream(need)
    elif args.workload == "hd720":
        ev = hd720_stream(need)
    else:
        ev = random_stream(W, H, need * B)
    if len(ev) < need * B:
        raise SystemExit("stream too short")
    storage = {"f32": 0, "bf16": 1, "f16": 2}[args.storage]
    kw = dict(shape=(W, H), batch=B, iters=IT, rows=args.rows, waves=args.waves, storage=storage,
              tvl1=args.tvl1, cols=args.cols, host_events=args.host_events)
    log("bench: timed pass")
    dt, _, u = run_gpu(ev, args.steps, args.warmup, args.fuse, profile=False, **kw)
    px_iters = args.steps * IT * W * H
    value = px_iters / dt / 1e6
    ev_rate = args.steps * B / dt
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "PD iter*Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "storage": args.storage,
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload].format(w=W, h=H),
                   "width": W, "height": H, "events_per_batch": B,
                   "iters_per_batch": IT, "fuse_iters": args.fuse, "tvl1_iters": args.tvl1,
                   "tile_rows": args.rows, "tile_waves": args.waves, "tile_cols": args.cols,
                   "events_from": "host" if args.host_events else "device"},
        "events_per_s": round(ev_rate, 1),
        "realtime_factor": round(ev_rate / 1e6, 3),
    }
    if not args.no_profile:
        log("bench: per-kernel timing pass")
        _, prof, _ = run_gpu(ev, args.steps, args.warmup, args.fuse, profile=True, **kw)
        bpi = BYTES_PER_PX_ITER if storage == 0 else BYTES_PER_PX_ITER_16
        eligible = args.fuse == -1 and not args.rows and not args.tvl1 and not args.host_events
        out["roofline"] = roofline(prof, bpi, "k_pd_fused" if args.fuse else "k_primal+k_dual",
                                   (args.workload, args.storage) if eligible else None)
        out["kernel_ms"] = {"push": round(prof.ms[0], 3), "build": round(prof.ms[1], 3),
                            "pd": round(prof.ms[2], 3)}
    if args.workload == "davis240" and args.storage == "f32" and not (
            args.rows or args.tvl1 or args.fuse != -1 or args.no_extras):
        # the other configurations, each on its own clock, beside the headline
        log("bench: 128x128 blocks of 500 events (latency and throughput)")
        out["dvs128"] = bench_dvs128()
        log("bench: 64 cameras, batched")
        out["streams64"] = bench_streams64()
        log("bench: 5120x5760 probe")
        out["probe"] = bench_probe()
    # the oracle beside the GPU on the frames whose blocks it finishes in seconds
    if not args.no_cpu and args.workload in ("davis240", "hd720"):
        log("bench: oracle baseline (all host cores, then one thread)")
        out["cpu_baseline"] = cpu_baseline(ev, W=W, H=H, batch=B, iters=IT)
        if args.workload == "davis240" and not args.no_extras:
            out["cpu_baseline"].update(oracle_c1_c3_c5())
    print(json.dumps(out), flush=True)


def roofline(prof, bpi, kernel, traffic_key=None, shape_ok=True):
    """Roofline object of the primal-dual launches timed in `prof`:
    achieved = algorithmic bytes (bpi per pixel-iteration) / kernel time;
    traffic = the HBM bytes per launch measured by the counters for this
    workload and these sources (None when not measured or stale)."""
    pd_ms = prof.ms[2]
    launches = int(prof.launches[2])
    achieved = bpi * prof.pd_pixel_iters / (pd_ms * 1e-3) / 1e9
    avg_us = pd_ms / launches * 1e3
    traffic, tb = None, None
    m = MEASURED_TRAFFIC.get(traffic_key) if traffic_key else None
    if m and shape_ok and m[0] == kernel_source_hash():
        tb = m[1] + m[2]
        traffic = round(tb / (avg_us * 1e-6) / 1e9, 1)
    return {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "traffic_frac": None if traffic is None else round(traffic / HBM_PEAK_GBS, 4),
        "kernel": kernel, "avg_launch_us": round(avg_us, 3), "launches": launches,
        "bytes_per_px_iter": bpi,
        "algorithmic_bytes_per_launch": round(bpi * prof.pd_pixel_iters / launches),
        "hbm_bytes_per_launch": None if tb is None else round(tb),
    }


PAPER_REALTIME = ("1.7 ms per reconstructed 128x128 image from 500 events (about 580 images/s, "
                  "0.29 M events/s) on an NVIDIA Titan X with a 3.4 GHz CPU (Section 4.1)")


def bench_dvs128(n_blocks=200, warmup=20):
    """The paper's setting: 128x128 sensor, blocks of 500 events, 50
    iterations.  Throughput over n_blocks back-to-back blocks, and the
    latency of one image (push, solve, wait for it) averaged over blocks."""
    import torch
    import evgen
    from paper_1607_06283_amd import rec

    n_lat = 50
    s, bs, nb, iters = evgen.dvs128(seed=1, n_batches=n_blocks + warmup + n_lat)
    ev = s.events
    dev = torch.device("cuda", 0)
    t = torch.from_numpy(ev.t).to(dev)
    x = torch.from_numpy(ev.x.view(np.int16)).to(dev)
    y = torch.from_numpy(ev.y.view(np.int16)).to(dev)
    p = torch.from_numpy(ev.p).to(dev)
    r = rec.Reconstructor(128, 128)

    def step(i):
        a = i * bs
        rc = rec.rec_push_events(r.ctx, t.data_ptr() + 8 * a, x.data_ptr() + 2 * a,
                                 y.data_ptr() + 2 * a, p.data_ptr() + a, bs, 1)
        if rc:
            raise rec.RecError(rc, "rec_push_events")
        rc, _ = rec.rec_solve(r.ctx, iters, False)
        if rc:
            raise rec.RecError(rc, "rec_solve")

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warmup, warmup + n_blocks):
        step(i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat = []
    for i in range(warmup + n_blocks, warmup + n_blocks + n_lat):
        t1 = time.perf_counter()
        step(i)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
    r.sync()
    r.close()
    return {"workload": "128x128 sensor, texture translating at 200 px/s, blocks of 500 events, "
                        "50 FP32 iterations per block, device-resident events",
            "blocks": n_blocks, "PD iter*Mpix/s": round(n_blocks * iters * 128 * 128 / dt / 1e6, 2),
            "events_per_s": round(n_blocks * bs / dt, 1),
            "images_per_s": round(n_blocks / dt, 1),
            "ms_per_image_back_to_back": round(dt / n_blocks * 1e3, 4),
            "ms_per_image_latency": round(float(np.mean(lat)) * 1e3, 4),
            "paper_context": PAPER_REALTIME}


def parse_geometry(text):
    """'WxH:RxWVxC:K,...' -> [(W, H, rows, waves, cols, K), ...]"""
    out = []
    for item in text.split(","):
        size, shape, k = item.split(":")
        w, h = size.split("x")
        r, wv, c = shape.split("x")
        out.append((int(w), int(h), int(r), int(wv), int(c), int(k)))
    return out


def bench_streams64(steps=20, warmup=3):
    """64 cameras batched (autotuned), each launch mode, against one solve per
    camera; then the same cameras with the geometry the HBM counters were
    taken with, whose roofline carries the measured traffic."""
    IT = WORKLOADS["streams64"][3]
    r = streams64_result(steps, warmup, IT)
    r = {"workload": WORKLOAD_TEXT["streams64"], "steps": steps, "warmup": warmup,
         "PD iter*Mpix/s": r.pop("value"), **r}
    p = streams64_result(steps, warmup, IT, tune=False, modes=("streams",),
                         geometry=parse_geometry(STREAMS64_PINNED), per_camera=False)
    r["pinned_geometry"] = {"geometry": STREAMS64_PINNED, "PD iter*Mpix/s": p["value"],
                            "ms_per_step": p["ms_per_step"], "roofline": p["roofline"]}
    return r


# The HBM-bound form of the probe: one iteration per launch, so every
# pixel-iteration reads and writes the whole state (44 B) once; the tile that
# streams best in this form (2 rows x 8 wavefronts x 64 columns, a sweep of 11
# shapes in profiles/k_pd_fused_probe_hbm.md).
PROBE_K1_TILE = (2, 8, 64)


def bench_probe(steps=10, warmup=2):
    """5120x5760 frame, uniform random events, blocks of 20000, 50 iterations:
    a state beyond the Infinity Cache, so the fused loop streams from HBM.
    Also the one-iteration-per-launch form, whose algorithmic bytes are its
    HBM bytes."""
    W, H, B, IT = WORKLOADS["probe"]
    ev = random_stream(W, H, (steps + warmup) * B)
    kw = dict(shape=(W, H), batch=B, iters=IT)
    dt, _, _ = run_gpu(ev, steps, warmup, -1, profile=False, **kw)
    _, prof, _ = run_gpu(ev, steps, warmup, -1, profile=True, **kw)
    out = {"workload": WORKLOAD_TEXT["probe"], "steps": steps, "warmup": warmup,
           "PD iter*Mpix/s": round(steps * IT * W * H / dt / 1e6, 2),
           "ms_per_step": round(dt / steps * 1e3, 4),
           "roofline": roofline(prof, BYTES_PER_PX_ITER, "k_pd_fused", ("probe", "f32"))}
    r, w, c = PROBE_K1_TILE
    k1 = dict(kw, rows=r, waves=w, cols=c)
    s1, w1 = max(2, steps // 3), 1
    dt, _, _ = run_gpu(ev, s1, w1, 1, profile=False, **k1)
    _, prof, _ = run_gpu(ev, s1, w1, 1, profile=True, **k1)
    out["one_iteration_per_launch"] = {
        "tile": {"rows": r, "waves": w, "cols": c}, "steps": s1, "warmup": w1,
        "PD iter*Mpix/s": round(s1 * IT * W * H / dt / 1e6, 2),
        "ms_per_step": round(dt / s1 * 1e3, 4),
        "roofline": roofline(prof, BYTES_PER_PX_ITER, "k_pd_fused", ("probe_k1", "f32"))}
    return out


if __name__ == "__main__":
    main()
