"""Seeded synthetic event streams shaped like the paper's sensor workloads.

This package is the only code shared by the FP64 oracle side and the GPU side:
it produces plain arrays (int64 microsecond timestamps, uint16 x/y, int8
polarity) and ground-truth log-intensity frames, and contains none of the
reconstruction arithmetic.  The C core (``evgen.c``) is built with gcc into
``libevgen.so`` next to this file.

Event model (Section 3 of the paper): an event at pixel (x, y) with polarity
+1/-1 marks a rise/drop of the log intensity by one contrast threshold; the
paper's sensor is a 128x128 DVS with 1 us timestamps (Section 4), natural
scenes give about 5e5 events/s, and images are formed from blocks of 500
events (Section 4.1).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import List, NamedTuple, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "evgen.c")
_LIB_PATH = os.path.join(_HERE, "libevgen.so")

T0_US = 10 ** 10  # streams start ~2.8 h into the sensor clock (int64 us)


class _Params(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("n_blobs", ctypes.c_int32),
        ("sigma_lo", ctypes.c_double), ("sigma_hi", ctypes.c_double),
        ("threshold", ctypes.c_double),
        ("speed_px_s", ctypes.c_double), ("omega_rad_s", ctypes.c_double),
        ("t0_us", ctypes.c_int64), ("dt_us", ctypes.c_int64),
        ("duration_us", ctypes.c_int64),
        ("noise_frac", ctypes.c_double),
    ]


def build(force: bool = True) -> str:
    """Compile ``libevgen.so`` with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
            "-fno-fast-math", "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.evg_run.restype = ctypes.c_void_p
        lib.evg_run.argtypes = [ctypes.POINTER(_Params)]
        lib.evg_count.restype = ctypes.c_int64
        lib.evg_count.argtypes = [ctypes.c_void_p]
        lib.evg_noise_count.restype = ctypes.c_int64
        lib.evg_noise_count.argtypes = [ctypes.c_void_p]
        lib.evg_max_step_dl.restype = ctypes.c_double
        lib.evg_max_step_dl.argtypes = [ctypes.c_void_p]
        lib.evg_copy.restype = ctypes.c_int
        lib.evg_copy.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 5
        lib.evg_free.restype = None
        lib.evg_free.argtypes = [ctypes.c_void_p]
        lib.evg_frame.restype = ctypes.c_int
        lib.evg_frame.argtypes = [ctypes.POINTER(_Params), ctypes.c_int64, ctypes.c_void_p]
        lib.evg_ref0.restype = ctypes.c_int
        lib.evg_ref0.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclasses.dataclass(frozen=True)
class StreamSpec:
    """One synthetic stream.  Times are integer microseconds."""
    width: int
    height: int
    seed: int
    duration_us: int
    speed_px_s: float = 200.0
    omega_rad_s: float = 0.0
    threshold: float = 0.2
    noise_frac: float = 0.0
    dt_us: int = 0                  # 0: chosen so a sample step moves L by <= threshold/4
    n_blobs: int = 32
    sigma_lo: float = 0.03
    sigma_hi: float = 0.10
    t0_us: int = T0_US

    def _c(self, dt_us: Optional[int] = None, duration_us: Optional[int] = None) -> _Params:
        return _Params(
            self.width, self.height, self.seed & 0xFFFFFFFFFFFFFFFF, self.n_blobs,
            self.sigma_lo, self.sigma_hi, self.threshold, self.speed_px_s,
            self.omega_rad_s, self.t0_us,
            int(dt_us if dt_us is not None else self.dt_us),
            int(duration_us if duration_us is not None else self.duration_us),
            self.noise_frac)


class Events(NamedTuple):
    t: np.ndarray         # int64 us, non-decreasing
    x: np.ndarray         # uint16 column
    y: np.ndarray         # uint16 row
    p: np.ndarray         # int8 polarity, +1 / -1
    is_noise: np.ndarray  # uint8, 1 for injected noise events

    def __len__(self):
        return int(self.t.shape[0])

    def slice(self, a: int, b: int) -> "Events":
        return Events(self.t[a:b], self.x[a:b], self.y[a:b], self.p[a:b], self.is_noise[a:b])


class Stream(NamedTuple):
    spec: StreamSpec
    events: Events
    dt_us: int
    max_step_dl: float


def frame(spec: StreamSpec, t_rel_us: int) -> np.ndarray:
    """Ground-truth log-intensity frame L(., ., t) in [0, 1], shape (H, W), float64."""
    lib = _load()
    out = np.empty((spec.height, spec.width), dtype=np.float64)
    prm = spec._c(dt_us=1, duration_us=0)
    rc = lib.evg_frame(ctypes.byref(prm), int(t_rel_us), out.ctypes.data)
    if rc != 0:
        raise ValueError("evg_frame rejected the stream spec")
    return out


def ref0(spec: StreamSpec) -> np.ndarray:
    """Initial per-pixel reference log intensity R0, shape (H, W), float64.

    exp(R0) is the known initial image: integrating a noise-free stream's
    events onto it tracks the scene's log intensity to within one threshold.
    """
    lib = _load()
    out = np.empty((spec.height, spec.width), dtype=np.float64)
    prm = spec._c(dt_us=1, duration_us=0)
    if lib.evg_ref0(ctypes.byref(prm), out.ctypes.data) != 0:
        raise ValueError("evg_ref0 rejected the stream spec")
    return out


def auto_dt_us(spec: StreamSpec) -> int:
    """Sampling step so that one step changes L by at most about threshold/4.

    Uses the largest finite-difference slope of the t = 0 frame times the
    largest pixel speed (translation plus rotation at the frame corner), with
    a 0.8 safety factor.
    """
    f0 = frame(spec, 0)
    g = 0.0
    if spec.width > 1:
        g = max(g, float(np.abs(np.diff(f0, axis=1)).max()))
    if spec.height > 1:
        g = max(g, float(np.abs(np.diff(f0, axis=0)).max()))
    hd = 0.5 * math.hypot(spec.width, spec.height)
    vmax = abs(spec.speed_px_s) + abs(spec.omega_rad_s) * hd
    if g <= 0.0 or vmax <= 0.0:
        return 1000
    dt = 0.8 * (spec.threshold / 4.0) / (g * vmax) * 1e6
    return int(max(1, min(10000, math.floor(dt))))


def generate(spec: StreamSpec) -> Stream:
    """Run the generator; returns the time-sorted stream."""
    lib = _load()
    dt = spec.dt_us if spec.dt_us > 0 else auto_dt_us(spec)
    prm = spec._c(dt_us=dt)
    h = lib.evg_run(ctypes.byref(prm))
    if not h:
        raise ValueError("evg_run rejected the stream spec or ran out of memory")
    try:
        n = lib.evg_count(h)
        t = np.empty(n, np.int64)
        x = np.empty(n, np.uint16)
        y = np.empty(n, np.uint16)
        p = np.empty(n, np.int8)
        nz = np.empty(n, np.uint8)
        lib.evg_copy(h, spec.width, t.ctypes.data, x.ctypes.data, y.ctypes.data,
                     p.ctypes.data, nz.ctypes.data)
        mdl = lib.evg_max_step_dl(h)
    finally:
        lib.evg_free(h)
    return Stream(spec, Events(t, x, y, p, nz), dt, mdl)


def event_rate(spec: StreamSpec, pilot_us: int = 20000) -> float:
    """Signal events per second over a pilot window (noise excluded)."""
    s = generate(dataclasses.replace(spec, duration_us=pilot_us, noise_frac=0.0))
    return len(s.events) / (pilot_us * 1e-6)


def calibrate(spec: StreamSpec, target_rate: float, pilot_us: int = 20000) -> StreamSpec:
    """Scale translation speed and rotation rate together so that a pilot run
    of ``pilot_us`` hits ``target_rate`` signal events per second (the event
    rate is close to linear in the motion speed)."""
    spec = dataclasses.replace(spec, dt_us=0)
    r = event_rate(spec, pilot_us)
    for _ in range(3):
        if r <= 0:
            raise ValueError("pilot run produced no events")
        k = target_rate / r
        spec = dataclasses.replace(spec, speed_px_s=spec.speed_px_s * k,
                                   omega_rad_s=spec.omega_rad_s * k)
        r = event_rate(spec, pilot_us)
        if abs(r / target_rate - 1.0) < 0.05:
            break
    return spec


def batches(events: Events, size: int) -> List[Events]:
    """Cut a stream into consecutive blocks of ``size`` events (last may be short)."""
    n = len(events)
    return [events.slice(a, min(n, a + size)) for a in range(0, n, size)]


# ---------------------------------------------------------------------------
# Workloads shaped like the paper's sensor and the configurations measured
# here.  Each returns (spec, batch_size, n_batches, iterations).
# ---------------------------------------------------------------------------

def dvs128(seed: int = 1, n_batches: int = 20):
    """128x128 sensor (the paper's DVS128), texture translating at 200 px/s,
    blocks of 500 events (Section 4.1), 50 iterations, lambda 90."""
    need = 500 * n_batches
    dur = 20000
    while True:
        spec = StreamSpec(128, 128, seed, duration_us=dur, speed_px_s=200.0)
        s = generate(spec)
        if len(s.events) >= need:
            return s, 500, n_batches, 50
        dur *= 2


def davis240(seed: int = 2, duration_us: int = 2_000_000, rate: float = 1e6):
    """240x180 sensor, rotating and translating texture, ~1e6 events/s of
    signal plus 1 % uniform noise events, blocks of 1000 events, 50 iterations."""
    base = StreamSpec(240, 180, seed, duration_us=duration_us, speed_px_s=100.0,
                      omega_rad_s=100.0 / (0.5 * math.hypot(240, 180)), noise_frac=0.01)
    spec = calibrate(base, rate, pilot_us=duration_us)
    s = generate(dataclasses.replace(spec, duration_us=duration_us))
    return s, 1000, (len(s.events) + 999) // 1000, 50


def hd720(seed: int = 3, duration_us: int = 500_000, rate: float = 2e7):
    """1280x720 sensor at ~2e7 events/s, blocks of 20000 events, 100 iterations."""
    base = StreamSpec(1280, 720, seed, duration_us=duration_us, speed_px_s=100.0,
                      omega_rad_s=100.0 / (0.5 * math.hypot(1280, 720)))
    spec = calibrate(base, rate, pilot_us=20_000)
    s = generate(dataclasses.replace(spec, duration_us=duration_us))
    return s, 20000, (len(s.events) + 19999) // 20000, 100


def diff_inputs(seed: int, batch: int, height: int, width: int, levels=(0.25, 0.75),
                max_count: int = 3) -> dict:
    """Random inputs of the differentiable unrolled solve (no method
    arithmetic here): a smooth initial image u0 = exp(level), level in
    `levels` (inside (0, 1), so u0 is inside (1, e)), signed event counts up
    to max_count, a smooth time-surface slope field (tx, ty) with a little
    noise, and data weights w around 1.  Float planes are float32 so the GPU
    and the FP64 references see identical values.  Shapes [batch, H, W]."""
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    def smooth(lo, hi, waves=3):
        acc = np.zeros((batch, height, width))
        for b in range(batch):
            for _ in range(waves):
                kx, ky = rng.uniform(-0.35, 0.35, 2)
                ph = rng.uniform(0, 2 * np.pi)
                acc[b] += np.sin(kx * xx + ky * yy + ph)
        acc = (acc - acc.min()) / max(acc.max() - acc.min(), 1e-12)
        return lo + (hi - lo) * acc
    u0 = np.exp(smooth(*levels)).astype(np.float32)
    fired = rng.random((batch, height, width)) < 0.3
    npos = np.where(fired & (rng.random(fired.shape) < 0.5),
                    rng.integers(1, max_count + 1, fired.shape), 0)
    nneg = np.where(fired & (npos == 0), rng.integers(1, max_count + 1, fired.shape), 0)
    tx = (smooth(-1.5, 1.5) + 0.05 * rng.standard_normal(fired.shape)).astype(np.float32)
    ty = (smooth(-1.5, 1.5) + 0.05 * rng.standard_normal(fired.shape)).astype(np.float32)
    w = rng.uniform(0.5, 1.5, fired.shape).astype(np.float32)
    return {"u0": u0, "npos": npos.astype(np.int32), "nneg": nneg.astype(np.int32),
            "tx": tx, "ty": ty, "w": w}


def diff_blocks(seed0: int = 500, n: int = 16, width: int = 346, height: int = 260,
                events: int = 2000):
    """n independent 346x260 streams (seeds seed0 ...), the first `events`
    events of each: for a training batch of the differentiable solve.
    Returns a list of (spec, block, L_start, L_end): the ground-truth
    log-intensity frames at the stream start and at the block's last event."""
    out = []
    for i in range(n):
        dur = 20000
        while True:
            spec = StreamSpec(width, height, seed0 + i, duration_us=dur, speed_px_s=200.0)
            ev = generate(spec).events
            if len(ev) >= events:
                break
            dur *= 2
        blk = ev.slice(0, events)
        t_end = int(blk.t[-1]) - spec.t0_us
        out.append((spec, blk, frame(spec, 0), frame(spec, t_end)))
    return out


STREAMS64_SIZES = [(128, 128), (240, 180), (346, 260), (640, 480)]


def streams64(steps: int, seed: int = 400, sizes=None, per_size: int = 16):
    """Many independent cameras of uneven size and event rate: `per_size`
    cameras of each sensor size (default 16 each of 128x128, 240x180,
    346x260, 640x480), camera i seeded with seed + i.  Per camera an event
    rate log-uniform in [1e5, 5e6] /s and a block size log-uniform in
    [200, 5000] events; uniform random pixels and polarities, exponential
    inter-event times at that rate (floored to us), `steps` blocks.
    Returns a list of (W, H, block_size, Events)."""
    sizes = STREAMS64_SIZES if sizes is None else sizes
    cams = []
    for i in range(per_size * len(sizes)):
        rng = np.random.default_rng(seed + i)
        W, H = sizes[i // per_size]
        rate = float(np.exp(rng.uniform(np.log(1e5), np.log(5e6))))
        bs = int(round(np.exp(rng.uniform(np.log(200), np.log(5000)))))
        n = bs * steps
        dt = rng.exponential(1e6 / rate, n)
        t = T0_US + np.floor(np.cumsum(dt)).astype(np.int64)
        x = rng.integers(0, W, n).astype(np.uint16)
        y = rng.integers(0, H, n).astype(np.uint16)
        p = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
        cams.append((W, H, bs, Events(t, x, y, p, np.zeros(n, np.uint8))))
    return cams


def long_idle_blocks(width: int = 48, height: int = 32, seed: int = 11, n: int = 400):
    """Three blocks of uniform random events spanning 80 s: the whole frame
    fires in the first second, then only the left half at 75 s and the left
    third at 79 s, so pixels idle since the first second border pixels that
    fire 75 s later (time differences of ~75000 in milliseconds)."""
    rng = np.random.default_rng(seed)
    out = []
    for k, (t_lo, t_hi, x_hi) in enumerate([(0, 1_000_000, width),
                                            (75_000_000, 76_000_000, width // 2),
                                            (79_000_000, 80_000_000, width // 3)]):
        t = T0_US + t_lo + np.sort(rng.integers(0, t_hi - t_lo, n)).astype(np.int64)
        x = rng.integers(0, width if k == 0 else x_hi, n).astype(np.uint16)
        y = rng.integers(0, height, n).astype(np.uint16)
        p = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
        out.append(Events(t, x, y, p, np.zeros(n, np.uint8)))
    return out
