"""Pins of the oracle's event-facing steps: scatter, data image, time surface,
push validation, and the gap along a real stream."""
import math

import numpy as np
import pytest

import evgen
import oracle
from oracle import Oracle, Params


@pytest.fixture(scope="module")
def c1():
    s, bs, nb, it = evgen.dvs128(seed=1, n_batches=6)
    return s


def test_scatter_brute_force(c1):
    """Every event adds one to its pixel's polarity count and raises its
    latest timestamp (Section 3: events carry pixel, polarity, timestamp)."""
    ev = c1.events.slice(0, 1500)
    o = Oracle(Params(128, 128))
    assert o.push_events(ev) == oracle.OK
    npos = np.zeros((128, 128), np.int32)
    nneg = np.zeros((128, 128), np.int32)
    last = {}
    for t, x, y, p in zip(ev.t.tolist(), ev.x.tolist(), ev.y.tolist(), ev.p.tolist()):
        if p > 0:
            npos[y, x] += 1
        else:
            nneg[y, x] += 1
        last[(y, x)] = max(last.get((y, x), t), t)
    assert np.array_equal(o.get(oracle.NPOS), npos)
    assert np.array_equal(o.get(oracle.NNEG), nneg)
    tl = o.get(oracle.TLAST)
    first = int(ev.t[0])
    for yy in range(128):
        for xx in range(128):
            assert tl[yy, xx] == last.get((yy, xx), first)
    assert o.t_ref == int(ev.t[-1])


def test_data_image_is_per_event_product(c1):
    """eqn. intensity_update applied event by event: f(x^n, y^n) is multiplied
    by c1 = exp(Delta+) for positive and c2 = exp(-Delta-) for negative events."""
    prm = Params(128, 128, delta_pos=0.23, delta_neg=0.17)
    rng = np.random.default_rng(5)
    u0 = np.exp(rng.uniform(0, 1, (128, 128)))
    o = Oracle(prm, u0=u0)
    ev = c1.events.slice(0, 2000)
    o.push_events(ev)
    o.build()
    f = u0.copy()
    c_pos, c_neg = math.exp(prm.delta_pos), math.exp(-prm.delta_neg)
    for x, y, p in zip(ev.x.tolist(), ev.y.tolist(), ev.p.tolist()):
        f[y, x] *= c_pos if p > 0 else c_neg
    assert np.allclose(o.get(oracle.F), f, rtol=1e-12, atol=0)


def test_perfect_integration_noise_free(c1):
    """Section 3: from a known u^0 and noise-free events, integration
    reconstructs the image up to the threshold quantisation."""
    spec = c1.spec
    u0 = np.exp(evgen.ref0(spec))
    o = Oracle(Params(128, 128), u0=u0)
    ev = c1.events
    o.push_events(ev)
    o.build()
    logf = np.log(o.get(oracle.F))
    n = np.zeros((128, 128))
    np.add.at(n, (ev.y.astype(int), ev.x.astype(int)), ev.p.astype(float))
    assert np.allclose(logf - np.log(u0), 0.2 * n, rtol=0, atol=1e-12)
    gt = evgen.frame(spec, spec.duration_us)
    assert np.abs(logf - gt).max() < 0.2


def test_time_surface_properties(c1):
    """t(x, y) = time since the last event (Section 3.1); differences of the
    surface are the forward differences of tau; T_s = 0 is the flat manifold."""
    ev = c1.events.slice(0, 3000)
    o = Oracle(Params(128, 128, time_unit_us=1000.0))
    o.push_events(ev)
    o.build()
    tau = o.get(oracle.TAU)
    assert tau.min() >= 0.0
    assert tau[int(ev.y[-1]), int(ev.x[-1])] == 0.0
    fired = np.zeros((128, 128), bool)
    fired[ev.y.astype(int), ev.x.astype(int)] = True
    assert np.allclose(tau[~fired], (int(ev.t[-1]) - int(ev.t[0])) / 1000.0)
    tx, ty = o.get(oracle.TX), o.get(oracle.TY)
    ex = np.zeros_like(tau)
    ey = np.zeros_like(tau)
    ex[:, :-1] = tau[:, 1:] - tau[:, :-1]
    ey[:-1, :] = tau[1:, :] - tau[:-1, :]
    assert np.allclose(tx, ex, rtol=1e-12, atol=1e-9)
    assert np.allclose(ty, ey, rtol=1e-12, atol=1e-9)
    # the FP32 side outputs are the FP64 values rounded once
    assert np.array_equal(o.get(oracle.TAU32), tau.astype(np.float32))
    assert np.array_equal(o.get(oracle.TX32), tx.astype(np.float32))
    flat = Oracle(Params(128, 128, time_unit_us=0.0))
    flat.push_events(ev)
    flat.build()
    assert not flat.get(oracle.TX).any() and not flat.get(oracle.TY).any()
    assert not flat.get(oracle.TAU).any()


def test_push_validation_all_or_nothing():
    """Polarity in {-1, 1}, coordinates inside Omega, timestamps monotone
    (Section 3); a rejected push leaves the state untouched."""
    o = Oracle(Params(8, 5))
    t = np.array([10, 11, 11, 15], np.int64)
    x = np.array([0, 7, 3, 2], np.uint16)
    y = np.array([0, 4, 1, 2], np.uint16)
    p = np.array([1, -1, 1, 1], np.int8)
    assert o.push(t, x, y, np.array([1, 0, 1, 1], np.int8)) == oracle.EINVAL
    assert o.push(t, np.array([0, 8, 3, 2], np.uint16), y, p) == oracle.ERANGE
    assert o.push(t, x, np.array([0, 4, 5, 2], np.uint16), p) == oracle.ERANGE
    assert o.push(np.array([10, 9, 11, 15], np.int64), x, y, p) == oracle.EORDER
    assert not o.get(oracle.NPOS).any() and not o.get(oracle.NNEG).any()
    assert o.push(t, x, y, p) == oracle.OK
    assert o.push(np.array([14], np.int64), x[:1], y[:1], p[:1]) == oracle.EORDER
    assert o.push(np.array([15], np.int64), x[:1], y[:1], p[:1]) == oracle.OK  # ties allowed
    assert o.get(oracle.NPOS).sum() == 4 and o.get(oracle.NNEG).sum() == 1


def test_empty_block_smooths_previous_image():
    """No events: f equals the previous image and the solve only regularises."""
    rng = np.random.default_rng(9)
    u0 = np.exp(rng.uniform(0, 1, (6, 9)))
    o = Oracle(Params(9, 6), u0=u0)
    o.solve(0)
    assert np.array_equal(o.get(oracle.F), u0)
    o.solve(25)
    assert np.allclose(o.get(oracle.F), u0)
    assert np.ptp(o.u) < np.ptp(u0)


def test_gap_nonnegative_and_decreasing_on_stream(c1):
    """Along the 128x128 stream (blocks of 500 events, 50 warm-started
    iterations, lambda 90), the primal-dual gap sampled every 10 iterations
    is non-negative and non-increasing within every block."""
    o = Oracle(Params(128, 128))
    for b in evgen.batches(c1.events, 500)[:6]:
        o.push_events(b)
        g, e = o.solve(50, gap_every=10)
        assert (g >= 0).all()
        assert (np.diff(g) <= 0).all(), g
        assert (e > 0).all()


def test_gap_goes_to_zero_on_stream_block(c1):
    """Long runs on one block drive the gap to zero and the energy to its
    minimum (the method converges; Section 3.2)."""
    o = Oracle(Params(128, 128))
    o.push_events(c1.events.slice(0, 500))
    g, e = o.solve(6000, gap_every=1000)
    assert (np.diff(g) < 0).all()
    assert g[-1] < 0.25 * g[0]
    assert g[-1] < 1e-6 * e[-1]
    assert (np.diff(e) <= 1e-9 * e[0]).all()


def test_threaded_oracle_build_gives_the_same_bits():
    """The OpenMP build of the oracle (the CPU baseline on all host cores)
    computes every pixel with the same operations and keeps the gap sum
    serial: u, p, f, the time differences and the gap history equal the
    single-threaded build's bit for bit."""
    s, bs, _, iters = evgen.dvs128(seed=1, n_batches=3)
    outs = []
    for threads in (False, True):
        o = oracle.Oracle(oracle.Params(128, 128), threads=threads)
        hist = []
        for b in evgen.batches(s.events, bs)[:3]:
            o.push_events(b)
            g, e = o.solve(iters, gap_every=10)
            hist.append((g, e))
        outs.append((o.u, o.p, o.get(oracle.F), o.get(oracle.TX), hist))
        o.close()
    for a, b in zip(outs[0][:4], outs[1][:4]):
        assert np.array_equal(a, b)
    for (g0, e0), (g1, e1) in zip(outs[0][4], outs[1][4]):
        assert np.array_equal(g0, g1) and np.array_equal(e0, e1)


def test_slope_cap_reading(c1):
    """The slope cap (the reading of 16-bit storage, which saturates at
    65504) clips the time differences and nothing else: with a cap above
    every difference the oracle gives the same bits as without one; on a
    stream whose differences exceed the cap, the capped differences are the
    plain ones clipped, the image stays finite, and it differs from the
    plain oracle's only where the problem changed."""
    blocks = evgen.batches(c1.events, 500)[:3]
    o, oc = Oracle(Params(128, 128)), Oracle(Params(128, 128, slope_cap=1e9))
    for b in blocks:
        for q in (o, oc):
            q.push_events(b)
            q.solve(20)
    assert np.array_equal(o.u, oc.u) and np.array_equal(o.p, oc.p)
    assert np.array_equal(o.get(oracle.TX), oc.get(oracle.TX))
    cap = 65504.0
    o, oc = Oracle(Params(48, 32)), Oracle(Params(48, 32, slope_cap=cap))
    for b in evgen.long_idle_blocks(48, 32):
        for q in (o, oc):
            q.push_events(b)
            q.solve(50)
        for plane in (oracle.TX, oracle.TY):
            plain = o.get(plane)
            assert np.array_equal(oc.get(plane), np.clip(plain, -cap, cap))
        assert np.isfinite(oc.u).all()
    assert np.abs(o.get(oracle.TX)).max() > 70000.0
    assert 0.0 < np.abs(o.u - oc.u).max() < 1e-2
    assert oracle.check_params(Params(8, 8, slope_cap=-1.0)) == oracle.EINVAL
