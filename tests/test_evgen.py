"""The seeded input generator: determinism, ordering, the sensor invariant and
the rate calibration."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import evgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "evgen_sha256.json")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def digest(ev) -> str:
    h = hashlib.sha256()
    for a in (ev.t, ev.x, ev.y, ev.p, ev.is_noise):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def small_spec(seed=11, noise=0.0):
    return evgen.StreamSpec(64, 48, seed, duration_us=30000, speed_px_s=300.0,
                            omega_rad_s=2.0, noise_frac=noise)


def test_deterministic_and_sorted():
    a = evgen.generate(small_spec(noise=0.02)).events
    b = evgen.generate(small_spec(noise=0.02)).events
    assert digest(a) == digest(b)
    assert len(a) > 1000
    assert (np.diff(a.t) >= 0).all()
    assert a.t[0] >= evgen.T0_US and a.t[-1] <= evgen.T0_US + 30000
    assert set(np.unique(a.p).tolist()) <= {-1, 1}
    assert a.x.max() < 64 and a.y.max() < 48
    c = evgen.generate(small_spec(seed=12)).events
    assert digest(a) != digest(c)


def test_thread_count_independent():
    code = ("import hashlib, numpy as np, evgen;"
            "e = evgen.generate(evgen.StreamSpec(64, 48, 11, duration_us=30000, speed_px_s=300.0,"
            " omega_rad_s=2.0, noise_frac=0.02)).events;"
            "h = hashlib.sha256();"
            "[h.update(np.ascontiguousarray(a).tobytes()) for a in (e.t, e.x, e.y, e.p, e.is_noise)];"
            "print(h.hexdigest())")
    outs = set()
    for n in ("1", "3", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=n, PYTHONPATH=ROOT)
        outs.add(subprocess.check_output([sys.executable, "-c", code], env=env, cwd=ROOT).strip())
    assert len(outs) == 1


def test_golden_digest():
    """SHA-256 of the 128x128 stream (seed 1) matches the committed fixture
    (written by tests/golden/make_evgen_golden.py)."""
    with open(GOLDEN) as fh:
        want = json.load(fh)
    s, _, _, _ = evgen.dvs128(seed=1, n_batches=20)
    assert digest(s.events) == want["dvs128_seed1"]


def test_reference_level_invariant():
    """Noise-free: |L - (R0 + Delta (n+ - n-))| < Delta at the end of the stream
    (events mark one-threshold changes of log intensity, Section 3)."""
    spec = small_spec()
    s = evgen.generate(spec)
    ev = s.events
    n = np.zeros((spec.height, spec.width))
    np.add.at(n, (ev.y.astype(int), ev.x.astype(int)), ev.p.astype(float))
    R = evgen.ref0(spec) + spec.threshold * n
    L = evgen.frame(spec, spec.duration_us)
    assert np.abs(L - R).max() < spec.threshold
    assert np.abs(evgen.frame(spec, 0) - evgen.ref0(spec)).max() < spec.threshold
    assert s.max_step_dl <= spec.threshold / 4 * 1.05


def test_noise_fraction():
    spec = small_spec(noise=0.05)
    s = evgen.generate(spec)
    frac = s.events.is_noise.mean()
    assert abs(frac - 0.05 / 1.05) < 0.002


def test_texture_range_and_static_scene():
    """Frames lie in [0, 1] (min-max normalised at t = 0); a static scene
    never changes, so it emits no events."""
    spec = evgen.StreamSpec(40, 30, 4, duration_us=50_000, speed_px_s=0.0)
    f0 = evgen.frame(spec, 0)
    assert f0.min() == 0.0 and 1.0 - 1e-12 <= f0.max() <= 1.0
    assert np.array_equal(evgen.frame(spec, 40_000), f0)
    assert len(evgen.generate(spec).events) == 0


@pytest.mark.slow
def test_rate_calibration():
    """Calibrated motion hits the requested event rate within +/-10 %."""
    base = evgen.StreamSpec(240, 180, 2, duration_us=200_000, speed_px_s=100.0,
                            omega_rad_s=0.6)
    spec = evgen.calibrate(base, 1e6, pilot_us=200_000)
    s = evgen.generate(spec)
    rate = len(s.events) / 0.2
    assert 0.9e6 <= rate <= 1.1e6
