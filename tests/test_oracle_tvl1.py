"""Pins of the oracle's timestamp denoising (Section 4: a few iterations of
TV-L1 on the timestamps before the manifold is built)."""
import math

import numpy as np
import pytest

import evgen
import oracle
from oracle import Oracle, Params

RNG = np.random.default_rng(1607)


def textbook_tvl1(f, iters, lam):
    """Chambolle-Pock 2011 for min TV(v) + lam |v - f|_1, written
    independently with numpy slicing: primal prox = soft shrinkage towards f,
    dual prox = projection onto the unit ball, steps 1/sqrt(8)."""
    s = 1.0 / math.sqrt(8.0)
    v = f.copy()
    qx = np.zeros_like(f)
    qy = np.zeros_like(f)
    for _ in range(iters):
        d = np.zeros_like(f)
        d[:, :-1] += qx[:, :-1]
        d[:, 1:] -= qx[:, :-1]
        d[:-1, :] += qy[:-1, :]
        d[1:, :] -= qy[:-1, :]
        w = v + s * d - f
        vn = f + np.sign(w) * np.maximum(np.abs(w) - s * lam, 0.0)
        vb = 2 * vn - v
        gx = np.zeros_like(f)
        gy = np.zeros_like(f)
        gx[:, :-1] = vb[:, 1:] - vb[:, :-1]
        gy[:-1, :] = vb[1:, :] - vb[:-1, :]
        a, b = qx + s * gx, qy + s * gy
        m = np.maximum(1.0, np.sqrt(a * a + b * b))
        qx, qy = a / m, b / m
        v = vn
    return v


def tv_l1_energy(v, f, lam):
    gx = np.zeros_like(v)
    gy = np.zeros_like(v)
    gx[:, :-1] = v[:, 1:] - v[:, :-1]
    gy[:-1, :] = v[1:, :] - v[:-1, :]
    return np.sqrt(gx ** 2 + gy ** 2).sum() + lam * np.abs(v - f).sum()


@pytest.mark.parametrize("lam", [0.3, 1.0, 5.0])
def test_matches_textbook(lam):
    f = RNG.normal(0, 20, (13, 17))
    assert np.allclose(oracle.tvl1(f, 40, lam), textbook_tvl1(f, 40, lam), rtol=0, atol=1e-10)


def test_constant_surface_is_fixed_point_and_shift_equivariant():
    f = np.full((9, 11), 37.5)
    assert np.array_equal(oracle.tvl1(f, 30, 1.0), f)
    g = RNG.normal(0, 5, (9, 11))
    a = oracle.tvl1(g, 25, 0.8)
    b = oracle.tvl1(g + 1000.0, 25, 0.8)
    assert np.allclose(b - 1000.0, a, atol=1e-9)


def test_isolated_spike_removed():
    """An isolated outlier (a noise event's timestamp) costs (2 + sqrt 2) h in
    the isotropic forward-difference TV and lambda h in the L1 term, so TV-L1
    removes it for lambda < 2 + sqrt 2 and keeps it above, whatever its
    height h."""
    f = np.full((15, 15), 10.0)
    f[7, 7] = 500.0
    v = oracle.tvl1(f, 3000, 1.0)
    assert np.abs(v - 10.0).max() < 1e-6
    v = oracle.tvl1(f, 3000, 2.0 + math.sqrt(2.0) + 0.2)
    assert abs(v[7, 7] - 500.0) < 1e-6


def test_large_lambda_keeps_data_and_energy_decreases():
    f = RNG.normal(0, 3, (10, 12))
    assert np.array_equal(oracle.tvl1(f, 20, 1e9), f)
    v = oracle.tvl1(f, 500, 0.7)
    assert tv_l1_energy(v, f, 0.7) < tv_l1_energy(f, f, 0.7)


def test_denoised_surface_drives_the_metric():
    """With denoising on, the time differences are the forward differences
    of the denoised surface; with it off they are the raw differences."""
    s, _, _, _ = evgen.dvs128(seed=1, n_batches=2)
    ev = s.events.slice(0, 1000)
    raw = Oracle(Params(128, 128))
    den = Oracle(Params(128, 128, tvl1_iters=5, tvl1_lambda=1.0))
    for o in (raw, den):
        o.push_events(ev)
        o.build()
    tau = raw.get(oracle.TAU)
    v = oracle.tvl1(tau, 5, 1.0)
    ex = np.zeros_like(v)
    ey = np.zeros_like(v)
    ex[:, :-1] = v[:, 1:] - v[:, :-1]
    ey[:-1, :] = v[1:, :] - v[:-1, :]
    assert np.array_equal(den.get(oracle.TX), ex) and np.array_equal(den.get(oracle.TY), ey)
    assert np.array_equal(den.get(oracle.TX32), ex.astype(np.float32))
    assert not np.array_equal(den.get(oracle.TX), raw.get(oracle.TX))
