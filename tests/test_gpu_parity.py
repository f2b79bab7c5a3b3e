"""GPU parity: the HIP library through its C ABI against the FP64 oracle.

Bars: integer and timestamp work (scatter counts, latest timestamps) and the
FP32 time planes are bit-exact; the image u matches the oracle within
max-abs 1e-4 after every block of 50 iterations; the primal-dual gap within
1e-3 relative; the fused temporally-blocked loop is bit-identical to the
two-kernel loop.
"""
import math

import numpy as np
import pytest

import evgen
import oracle
from paper_1607_06283_amd import rec

pytestmark = pytest.mark.gpu

U_TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def c1():
    s, bs, nb, it = evgen.dvs128(seed=1, n_batches=20)
    return s


def oracle_params(prm: rec.rec_params) -> oracle.Params:
    return oracle.Params(prm.width, prm.height, lam=prm.lambda_, delta_pos=prm.delta_pos,
                         delta_neg=prm.delta_neg, u_min=prm.u_min, u_max=prm.u_max, tau=prm.tau,
                         sigma=prm.sigma, time_unit_us=prm.time_unit_us, u_init=prm.u_init,
                         tvl1_iters=prm.tvl1_iters, tvl1_lambda=prm.tvl1_lambda)


def make(W, H, u0=None, **kw):
    prm = rec.rec_default_params(W, H, **kw)
    r = rec.Reconstructor(W, H, params=prm, u0=u0)
    o = oracle.Oracle(oracle_params(prm), u0=u0)
    return r, o


def device_events(ev):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(ev.t)).cuda(),
            torch.from_numpy(np.ascontiguousarray(ev.x).view(np.int16)).cuda(),
            torch.from_numpy(np.ascontiguousarray(ev.y).view(np.int16)).cuda(),
            torch.from_numpy(np.ascontiguousarray(ev.p)).cuda())


# --------------------------------------------------------------------------
# Bit-exact steps
# --------------------------------------------------------------------------

@pytest.mark.parametrize("on_device", [False, True])
def test_scatter_bit_exact(c1, on_device):
    r, o = make(128, 128)
    for b in evgen.batches(c1.events, 500)[:3]:
        if on_device:
            r.push(*device_events(b), on_device=True)
        else:
            r.push(b.t, b.x, b.y, b.p)
        o.push_events(b)
    assert np.array_equal(r.image(rec.REC_COUNT_POS), o.get(oracle.NPOS))
    assert np.array_equal(r.image(rec.REC_COUNT_NEG), o.get(oracle.NNEG))
    assert np.array_equal(r.image(rec.REC_T_LAST), o.get(oracle.TLAST))
    st = r.solve(50, stats=True)
    assert st.t_ref_us == o.t_ref and st.events_in_batch == 1500
    assert not r.image(rec.REC_COUNT_POS).any()


@pytest.mark.parametrize("ts", [1000.0, 100.0, 10000.0, 0.0])
def test_time_planes_bit_exact(c1, ts):
    r, o = make(128, 128, time_unit_us=ts)
    for b in evgen.batches(c1.events, 500)[:4]:
        r.push(b.t, b.x, b.y, b.p)
        o.push_events(b)
        r.solve(5)
        o.solve(5)
        assert np.array_equal(r.image(rec.REC_TX), o.get(oracle.TX32))
        assert np.array_equal(r.image(rec.REC_TY), o.get(oracle.TY32))
        assert np.array_equal(r.image(rec.REC_TIME), o.get(oracle.TAU32))


@pytest.mark.parametrize("iters", [1, 2, 9, 10, 19])
def test_short_solves(c1, iters):
    """Solves of a few iterations: a single launch that rotates p into each
    pixel's frame and back (iters up to the iterations per launch) or a short
    split, with device pushes folded into the first launch; against the
    two-kernel loop bit for bit and against the oracle."""
    r, o = make(128, 128)
    rp = rec.Reconstructor(128, 128, fuse_iters=0)
    for b in evgen.batches(c1.events, 500)[:4]:
        r.push(*device_events(b), on_device=True)
        rp.push(b.t, b.x, b.y, b.p)
        o.push_events(b)
        r.solve(iters)
        rp.solve(iters)
        o.solve(iters)
        u = r.image(rec.REC_U)
        assert np.array_equal(u, rp.image(rec.REC_U))
        assert np.array_equal(r.image(rec.REC_STATE_P), rp.image(rec.REC_STATE_P))
        assert np.abs(u.astype(np.float64) - o.u).max() <= U_TOL
    r.close()
    rp.close()


def test_large_push_path_bit_exact(c1):
    """Pushes above the single-workgroup size use the multi-kernel path."""
    r, o = make(128, 128)
    ev = c1.events
    r.push(*device_events(ev), on_device=True)
    o.push_events(ev)
    assert np.array_equal(r.image(rec.REC_COUNT_POS), o.get(oracle.NPOS))
    assert np.array_equal(r.image(rec.REC_T_LAST), o.get(oracle.TLAST))


# --------------------------------------------------------------------------
# Reconstruction parity
# --------------------------------------------------------------------------

@pytest.mark.parametrize("fuse", [0, 8])
def test_dvs128_stream_parity(c1, fuse):
    """128x128, 20 blocks of 500 events, 50 iterations each, lambda 90:
    max |u_gpu - u_oracle| <= 1e-4 after every block."""
    r, o = make(128, 128, fuse_iters=fuse)
    worst = 0.0
    for b in evgen.batches(c1.events, 500)[:20]:
        r.push(b.t, b.x, b.y, b.p)
        o.push_events(b)
        r.solve(50)
        o.solve(50)
        d = np.abs(r.image(rec.REC_U).astype(np.float64) - o.u).max()
        worst = max(worst, d)
        assert d <= U_TOL, d
    print(f"fuse={fuse} worst max-abs {worst:.3e}")


def test_gap_parity(c1):
    r, o = make(128, 128, gap_every=10)
    for b in evgen.batches(c1.events, 500)[:3]:
        r.push(b.t, b.x, b.y, b.p)
        o.push_events(b)
        st = r.solve(50, stats=True)
        g_o, e_o = o.solve(50, gap_every=10)
        g, e = r.gap_history()
        assert len(g) == 5 and st.gap_samples == 5
        assert np.allclose(g, g_o, rtol=1e-3, atol=0)
        assert np.allclose(e, e_o, rtol=1e-6, atol=0)
        assert (g >= 0).all() and (np.diff(g) <= 0).all()
        assert st.gap == g[-1]


# --------------------------------------------------------------------------
# Fused loop == two-kernel loop
# --------------------------------------------------------------------------

SHAPES = [(128, 128), (240, 180), (67, 45), (1, 1), (1, 37), (29, 1), (200, 7), (5, 130)]


def _random_stream(W, H, n, seed):
    rng = np.random.default_rng(seed)
    t = evgen.T0_US + np.sort(rng.integers(0, 200_000, n)).astype(np.int64)
    x = rng.integers(0, W, n).astype(np.uint16)
    y = rng.integers(0, H, n).astype(np.uint16)
    p = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    return t, x, y, p


@pytest.mark.parametrize("W,H", SHAPES)
def test_fused_equals_plain_bitwise(W, H):
    t, x, y, p = _random_stream(W, H, 4 * max(1, W * H // 8), seed=W * 1000 + H)
    n = len(t)
    runs = []
    cfgs = [dict(fuse_iters=0), dict(fuse_iters=8), dict(fuse_iters=5, tile_rows=4, tile_waves=4),
            dict(fuse_iters=3, tile_rows=2, tile_waves=8), dict(fuse_iters=1, tile_rows=8, tile_waves=1),
            dict(fuse_iters=15, tile_rows=8, tile_waves=4), dict(fuse_iters=-1),
            dict(fuse_iters=12, tile_rows=2, tile_waves=16, gap_every=5),
            dict(fuse_iters=6, tile_rows=6, tile_waves=8), dict(fuse_iters=7, tile_rows=5, tile_waves=8),
            dict(fuse_iters=9, tile_rows=3, tile_waves=16), dict(fuse_iters=6, tile_rows=4, tile_waves=8),
            dict(fuse_iters=0, gap_every=7),
            # the automatic shapes of larger frames (64 x 64 tiles)
            dict(fuse_iters=10, tile_rows=8, tile_waves=8),
            dict(fuse_iters=13, tile_rows=4, tile_waves=16),
            # 32-column tiles (two lane rows per wavefront)
            dict(fuse_iters=8, tile_rows=2, tile_waves=8, tile_cols=32),
            dict(fuse_iters=15, tile_rows=1, tile_waves=16, tile_cols=32),
            dict(fuse_iters=5, tile_rows=4, tile_waves=4, tile_cols=32),
            dict(fuse_iters=3, tile_rows=1, tile_waves=8, tile_cols=32),
            dict(fuse_iters=11, tile_rows=3, tile_waves=8, tile_cols=32),
            dict(fuse_iters=13, tile_rows=2, tile_waves=16, tile_cols=32, gap_every=6),
            dict(fuse_iters=6, tile_rows=2, tile_waves=4, tile_cols=32),
            dict(fuse_iters=9, tile_rows=4, tile_waves=8, tile_cols=32)]
    for cfg in cfgs:
        r = rec.Reconstructor(W, H, **cfg)
        for a in range(0, n, n // 4):
            r.push(t[a:a + n // 4], x[a:a + n // 4], y[a:a + n // 4], p[a:a + n // 4])
            r.solve(23)
        runs.append((r.image(rec.REC_U), r.image(rec.REC_STATE_P)))
        r.close()
    for (u, pp), cfg in zip(runs[1:], cfgs[1:]):
        assert np.array_equal(u, runs[0][0]), cfg
        assert np.array_equal(pp, runs[0][1]), cfg


@pytest.mark.parametrize("cfg", [dict(fuse_iters=-1), dict(fuse_iters=5, tile_rows=2, tile_waves=8,
                                                              tile_cols=32)])
def test_gap_samples_fused_equal_plain(c1, cfg):
    """Gap samples taken between fused launches (p held in the tangent frame,
    rotated back by the gap kernel) equal the two-kernel loop's bit for bit."""
    hist = []
    for kw in (dict(fuse_iters=0), cfg):
        r = rec.Reconstructor(128, 128, gap_every=7, **kw)
        for b in evgen.batches(c1.events, 500)[:3]:
            r.push(b.t, b.x, b.y, b.p)
            r.solve(30)
        hist.append(r.gap_history())
        r.close()
    assert len(hist[0][0]) == 4
    assert np.array_equal(hist[0][0], hist[1][0]) and np.array_equal(hist[0][1], hist[1][1])


def test_repeat_run_deterministic(c1):
    outs = []
    for _ in range(2):
        r = rec.Reconstructor(128, 128)
        for b in evgen.batches(c1.events, 500)[:5]:
            r.push(b.t, b.x, b.y, b.p)
            r.solve(50)
        outs.append(r.image(rec.REC_U))
        r.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("W,H", [(1, 1), (1, 37), (29, 1), (67, 45)])
def test_small_and_ragged_parity(W, H):
    t, x, y, p = _random_stream(W, H, 3 * W * H + 5, seed=W + 7 * H)
    r, o = make(W, H)
    n = len(t)
    for a in range(0, n, max(1, n // 3)):
        sl = slice(a, a + max(1, n // 3))
        r.push(t[sl], x[sl], y[sl], p[sl])
        o.push(t[sl], x[sl], y[sl], p[sl])
        r.solve(50)
        o.solve(50)
        assert np.abs(r.image(rec.REC_U).astype(np.float64) - o.u).max() <= U_TOL


@pytest.fixture(scope="module")
def davis():
    """The benchmark's 240x180 stream (2 s at 1e6 events/s plus 1 % noise)."""
    s, bs, nb, iters = evgen.davis240(seed=2)
    return s.events, bs, iters


def test_davis240_benchmark_path_parity(davis):
    """The first 40 blocks of the benchmark stream through the benchmark's
    path (device-resident pushes folded into the first fused launch, default
    tile and launch split): u after every block within 1e-4 of the FP64
    oracle."""
    ev, bs, iters = davis
    r, o = make(240, 180)
    worst = 0.0
    for b in evgen.batches(ev, bs)[:40]:
        r.push(*device_events(b), on_device=True)
        o.push_events(b)
        r.solve(iters)
        o.solve(iters)
        worst = max(worst, float(np.abs(r.image(rec.REC_U).astype(np.float64) - o.u).max()))
    print(f"240x180 benchmark path, 40 blocks: max-abs {worst:.3e}")
    assert worst <= U_TOL


def test_davis240_full_stream_properties(davis):
    """All ~2000 blocks of the benchmark stream (the oracle cannot follow the
    whole stream in test time): every block's events are consumed, the image
    stays in [u_min, u_max], the dual field stays in its ball, and the gap
    sampled at the end of the blocks is finite and non-negative."""
    ev, bs, iters = davis
    r = rec.Reconstructor(240, 180, gap_every=iters)
    t, x, y, p = device_events(ev)
    blocks = evgen.batches(ev, bs)
    a = 0
    for i, b in enumerate(blocks):
        n = len(b)
        r.push(t[a:a + n], x[a:a + n], y[a:a + n], p[a:a + n], on_device=True)
        check = i % 250 == 249 or i == len(blocks) - 1
        st = r.solve(iters, stats=check)
        if check:
            assert st.iters_run == iters and st.events_in_batch == n
            assert np.isfinite(st.gap) and st.gap >= -1e-9 * abs(st.energy)
        a += n
    assert a == len(ev)
    st = r.solve(iters, stats=True)  # an empty block smooths and consumes nothing
    assert st.events_in_batch == 0
    u = r.image(rec.REC_U)
    assert np.isfinite(u).all() and u.min() >= 1.0 and u.max() <= np.float32(np.e)
    pp = r.image(rec.REC_STATE_P).astype(np.float64)
    tx = r.image(rec.REC_TX).astype(np.float64)
    ty = r.image(rec.REC_TY).astype(np.float64)
    s = np.sqrt(1.0 + tx * tx + ty * ty)
    assert (np.sqrt((pp * pp).sum(axis=0)) <= s * (1 + 1e-6)).all()
    print(f"240x180 full stream: {a} events in {len(blocks)} blocks, final gap {st.gap:.3e}, "
          f"energy {st.energy:.6e}")
    r.close()


def test_binding_rejects_host_and_mistyped_tensors():
    """Tensors that would hand the device a host pointer or a wrong element
    size are refused in the binding, before any launch."""
    import torch
    r = rec.Reconstructor(16, 16)
    t = torch.arange(5, dtype=torch.int64) + evgen.T0_US
    x = torch.zeros(5, dtype=torch.int16)
    pol = torch.ones(5, dtype=torch.int8)
    with pytest.raises(ValueError):
        r.push(t, x, x, pol)                           # CPU tensors
    with pytest.raises(ValueError):
        r.push(t.cuda().to(torch.int32), x.cuda(), x.cuda(), pol.cuda())
    r.push(t.cuda(), x.cuda(), x.cuda(), pol.cuda())   # well-formed
    r.solve(5)
    assert np.isfinite(r.image(rec.REC_U)).all()
    r.close()
    inp = evgen.diff_inputs(3, 1, 8, 8)
    th = torch.tensor([90.0, 0.2, 0.2], dtype=torch.float64)
    c = {k: torch.from_numpy(v) for k, v in inp.items()}
    with pytest.raises(ValueError):
        rec.unrolled(c["u0"], c["npos"], c["nneg"], c["tx"], c["ty"], th, 3)


@pytest.mark.parametrize("W,H", [(65535, 2), (2, 65535)])
def test_largest_width_and_height(W, H):
    """The largest frame side the ABI accepts (65535), with the other side 2:
    thousands of tiles along one axis; fused and two-kernel loops give the
    same bits and stay within the tolerance of the FP64 oracle."""
    t, x, y, p = _random_stream(W, H, 20000, seed=W + H)
    r, o = make(W, H)
    r0 = rec.Reconstructor(W, H, fuse_iters=0)
    for a in (0, 10000):
        sl = slice(a, a + 10000)
        print(f"largest side W={W} H={H} block at {a}", flush=True)
        r.push(t[sl], x[sl], y[sl], p[sl])
        r0.push(t[sl], x[sl], y[sl], p[sl])
        o.push(t[sl], x[sl], y[sl], p[sl])
        r.solve(50)
        r0.solve(50)
        o.solve(50)
        u = r.image(rec.REC_U)
        assert np.array_equal(u, r0.image(rec.REC_U))
        assert np.abs(u.astype(np.float64) - o.u).max() <= U_TOL
    r.close()
    r0.close()


def test_empty_block_and_known_initial_image(c1):
    spec = c1.spec
    u0 = np.exp(evgen.ref0(spec)).astype(np.float32)
    r = rec.Reconstructor(128, 128, u0=u0)
    o = oracle.Oracle(oracle.Params(128, 128), u0=u0.astype(np.float64))
    r.solve(50)
    o.solve(50)
    assert np.abs(r.image(rec.REC_U) - o.u).max() <= U_TOL
    b = c1.events.slice(0, 500)
    u_prev = r.image(rec.REC_U).astype(np.float64)
    r.push(b.t, b.x, b.y, b.p)
    o.push_events(b)
    r.solve(50)
    o.solve(50)
    assert np.abs(r.image(rec.REC_U) - o.u).max() <= U_TOL
    # f is the GPU's own previous image times exp(Delta+ n+ - Delta- n-),
    # formed in FP64 and rounded once (eqn. intensity_update)
    n_pos = np.zeros((128, 128))
    n_neg = np.zeros((128, 128))
    np.add.at(n_pos, (b.y.astype(int), b.x.astype(int)), (b.p > 0).astype(float))
    np.add.at(n_neg, (b.y.astype(int), b.x.astype(int)), (b.p < 0).astype(float))
    f_ref = u_prev * np.exp(0.2 * n_pos - 0.2 * n_neg)
    assert np.allclose(r.image(rec.REC_F), f_ref, rtol=1.2e-7, atol=0)


# --------------------------------------------------------------------------
# Error handling through the ABI
# --------------------------------------------------------------------------

def test_host_push_errors_are_immediate_and_atomic():
    r = rec.Reconstructor(8, 5)
    t = np.array([10, 11, 11, 15], np.int64)
    x = np.array([0, 7, 3, 2], np.uint16)
    y = np.array([0, 4, 1, 2], np.uint16)
    p = np.array([1, -1, 1, 1], np.int8)
    with pytest.raises(rec.RecError) as e:
        r.push(t, x, y, np.array([1, 2, 1, 1], np.int8))
    assert e.value.code == rec.REC_EINVAL
    with pytest.raises(rec.RecError) as e:
        r.push(t, np.array([0, 8, 3, 2], np.uint16), y, p)
    assert e.value.code == rec.REC_ERANGE
    r.push(t, x, y, p)
    with pytest.raises(rec.RecError) as e:
        r.push(t[:1], x[:1], y[:1], p[:1])
    assert e.value.code == rec.REC_EORDER
    assert r.image(rec.REC_COUNT_POS).sum() == 3 and r.image(rec.REC_COUNT_NEG).sum() == 1


def test_device_push_errors_are_deferred_and_atomic():
    import torch
    r = rec.Reconstructor(8, 5)
    t = torch.tensor([10, 11, 11, 15], dtype=torch.int64, device="cuda")
    x = torch.tensor([0, 7, 3, 2], dtype=torch.int16, device="cuda")
    y = torch.tensor([0, 4, 1, 2], dtype=torch.int16, device="cuda")
    p = torch.tensor([1, -1, 1, 1], dtype=torch.int8, device="cuda")
    r.push(t, x, torch.tensor([0, 4, 9, 2], dtype=torch.int16, device="cuda"), p, on_device=True)
    with pytest.raises(rec.RecError) as e:
        r.sync()
    assert e.value.code == rec.REC_ERANGE
    r.sync()  # reported once
    r.push(t, x, y, torch.tensor([1, -1, 0, 1], dtype=torch.int8, device="cuda"), on_device=True)
    with pytest.raises(rec.RecError) as e:
        r.sync()
    assert e.value.code == rec.REC_EINVAL
    assert not r.image(rec.REC_COUNT_POS).any()
    r.push(t, x, y, p, on_device=True)
    r.push(t[:2], x[:2], y[:2], p[:2], on_device=True)  # goes back in time
    with pytest.raises(rec.RecError) as e:
        r.sync()
    assert e.value.code == rec.REC_EORDER
    assert r.image(rec.REC_COUNT_POS).sum() == 3
    # a later host push learns the device time and checks against it
    with pytest.raises(rec.RecError) as e:
        r.push(np.array([12], np.int64), np.array([1], np.uint16), np.array([1], np.uint16),
               np.array([1], np.int8))
    assert e.value.code == rec.REC_EORDER


# --------------------------------------------------------------------------
# Device pushes folded into the first fused launch
# --------------------------------------------------------------------------

def test_folded_pushes_match_scattered_pushes(c1):
    """Device-pointer pushes and host pushes of at most max_events events are
    binned by the solve's first launch; host pushes larger than max_events
    are split and scattered by kernels of their own.  All three give the
    same image, time planes and latest timestamps, bit for bit."""
    a = rec.Reconstructor(128, 128)
    b = rec.Reconstructor(128, 128)
    s = rec.Reconstructor(128, 128, max_events=128)
    for blk in evgen.batches(c1.events, 500)[:6]:
        a.push(*device_events(blk), on_device=True)
        b.push(blk.t, blk.x, blk.y, blk.p)
        s.push(blk.t, blk.x, blk.y, blk.p)
        sa = a.solve(50, stats=True)
        for other in (b, s):
            so = other.solve(50, stats=True)
            assert (sa.t_ref_us, sa.events_in_batch) == (so.t_ref_us, so.events_in_batch)
    for plane in (rec.REC_U, rec.REC_F, rec.REC_TX, rec.REC_TY, rec.REC_STATE_P, rec.REC_T_LAST,
                  rec.REC_TIME):
        assert np.array_equal(a.image(plane), b.image(plane)), plane
        assert np.array_equal(a.image(plane), s.image(plane)), plane


def test_host_pushes_through_the_staging_ring(c1):
    """A small staging ring (max_events 256: two pushes of 100 events per
    half) is reused while earlier pushes of the half are still recorded
    (they are scattered first) and while earlier solves are still queued
    (nothing synchronises between them); every block matches the oracle."""
    r, o = make(128, 128, max_events=256)
    blocks = evgen.batches(c1.events.slice(0, 2100), 100)
    assert len(blocks) == 21
    for i, blk in enumerate(blocks):
        r.push(blk.t, blk.x, blk.y, blk.p)
        o.push_events(blk)
        if i % 7 == 6:
            r.solve(20)
            o.solve(20)
    st = r.solve(20, stats=True)
    o.solve(20)
    assert st.events_in_batch == 0 and st.t_ref_us == o.t_ref
    assert np.array_equal(r.image(rec.REC_T_LAST), o.get(oracle.TLAST))
    assert np.array_equal(r.image(rec.REC_TX), o.get(oracle.TX32))
    assert np.abs(r.image(rec.REC_U).astype(np.float64) - o.u).max() <= U_TOL


def _dev(t, x, y, p):
    import torch
    return (torch.tensor(t, dtype=torch.int64, device="cuda"),
            torch.tensor(x, dtype=torch.int16, device="cuda"),
            torch.tensor(y, dtype=torch.int16, device="cuda"),
            torch.tensor(p, dtype=torch.int8, device="cuda"))


def test_folded_push_errors_all_or_nothing():
    """Folded pushes are validated in order, each all-or-nothing, with the
    codes of the host check; the first error is reported at the next sync."""
    W, H = 70, 40
    pushes = [
        ([100, 101, 105], [1, 69, 3], [0, 39, 7], [1, -1, 1]),        # ok
        ([106, 107, 108], [2, 3, 4], [1, 1, 1], [1, 0, 1]),           # bad polarity
        ([106, 110, 110], [5, 6, 7], [2, 2, 2], [-1, 1, 1]),          # ok (ties allowed)
        ([109, 111, 112], [8, 9, 10], [3, 3, 3], [1, 1, 1]),          # goes back in time
        ([120, 121, 122], [11, 70, 12], [4, 4, 4], [1, 1, 1]),        # x out of range
        ([130, 131, 132], [13, 14, 15], [5, 5, 5], [1, -1, -1]),      # ok
    ]
    r = rec.Reconstructor(W, H)
    o = oracle.Oracle(oracle_params(r.prm))
    codes = []
    for t, x, y, p in pushes[:4]:
        r.push(*_dev(t, x, y, p), on_device=True)
        codes.append(o.push(np.array(t, np.int64), np.array(x, np.uint16), np.array(y, np.uint16),
                            np.array(p, np.int8)))
    assert codes == [0, oracle.EINVAL, 0, oracle.EORDER]
    r.solve(30)
    o.solve(30)
    with pytest.raises(rec.RecError) as e:
        r.sync()
    assert e.value.code == rec.REC_EINVAL
    for t, x, y, p in pushes[4:]:
        r.push(*_dev(t, x, y, p), on_device=True)
        o.push(np.array(t, np.int64), np.array(x, np.uint16), np.array(y, np.uint16),
               np.array(p, np.int8))
    r.solve(30)
    o.solve(30)
    with pytest.raises(rec.RecError) as e:
        r.sync()
    assert e.value.code == rec.REC_ERANGE
    assert np.array_equal(r.image(rec.REC_T_LAST), o.get(oracle.TLAST))
    assert np.array_equal(r.image(rec.REC_TX), o.get(oracle.TX32))
    assert np.abs(r.image(rec.REC_U).astype(np.float64) - o.u).max() <= U_TOL


@pytest.mark.parametrize("fuse", [-1, 0])
def test_host_push_sizes_at_the_staging_limit(c1, fuse):
    """Host pushes of exactly max_events events (one record filling a half
    of the staging ring), of max_events + 1 (split: a full record and a
    single event, scattered at once), of single events and of max_events - 1,
    in the fused loop (records folded into the first launch) and in the
    unfused one (every record scattered): the oracle's result after every
    solve."""
    cap = 64
    r, o = make(128, 128, max_events=cap, fuse_iters=fuse)
    ev = c1.events.slice(0, 2000)
    sizes = [cap, cap + 1, 1, cap - 1, 1, 1, cap, 2 * cap + 1, cap]
    a = 0
    for k, n in enumerate(sizes):
        r.push(ev.t[a:a + n], ev.x[a:a + n], ev.y[a:a + n], ev.p[a:a + n])
        o.push(ev.t[a:a + n], ev.x[a:a + n], ev.y[a:a + n], ev.p[a:a + n])
        a += n
        if k % 3 == 2:
            st = r.solve(30, stats=True)
            o.solve(30)
            assert st.t_ref_us == o.t_ref
            assert np.array_equal(r.image(rec.REC_T_LAST), o.get(oracle.TLAST)), k
            assert np.abs(r.image(rec.REC_U).astype(np.float64) - o.u).max() <= U_TOL, k


def test_mixed_device_and_host_pushes(c1):
    """Device and host pushes alternating within blocks (a host push after a
    device push first learns the stream state, which scatters the recorded
    device push; the pushes after it are recorded in order, host records
    beside device arrays): the oracle's result after every solve."""
    r, o = make(128, 128)
    ev = c1.events.slice(0, 2400)
    a = 0
    for blk in range(4):
        for k, n in enumerate((150, 90, 160, 200)):
            sl = slice(a, a + n)
            a += n
            part = evgen.Events(ev.t[sl], ev.x[sl], ev.y[sl], ev.p[sl], np.zeros(n, np.uint8))
            if (k + blk) % 2 == 0:
                r.push(*device_events(part), on_device=True)
            else:
                r.push(part.t, part.x, part.y, part.p)
            o.push_events(part)
        st = r.solve(40, stats=True)
        o.solve(40)
        assert st.t_ref_us == o.t_ref and st.events_in_batch == 600
        assert np.array_equal(r.image(rec.REC_T_LAST), o.get(oracle.TLAST)), blk
        assert np.array_equal(r.image(rec.REC_TX), o.get(oracle.TX32)), blk
        assert np.abs(r.image(rec.REC_U).astype(np.float64) - o.u).max() <= U_TOL, blk


def test_many_pushes_per_solve(c1):
    """More device pushes than the first launch folds: the earlier ones are
    scattered, the rest folded; the result matches the oracle."""
    r, o = make(128, 128)
    for blk in evgen.batches(c1.events.slice(0, 3000), 100)[:7]:
        r.push(*device_events(blk), on_device=True)
        o.push_events(blk)
    st = r.solve(50, stats=True)
    o.solve(50)
    assert st.events_in_batch == 700 and st.t_ref_us == o.t_ref
    assert np.array_equal(r.image(rec.REC_T_LAST), o.get(oracle.TLAST))
    assert np.abs(r.image(rec.REC_U).astype(np.float64) - o.u).max() <= U_TOL


# --------------------------------------------------------------------------
# Reduced-precision storage of p and (tx, ty), FP32 arithmetic
# --------------------------------------------------------------------------

@pytest.mark.parametrize("storage,bound", [(rec.REC_STORE_F16, 2e-3), (rec.REC_STORE_BF16, 2e-2)])
def test_reduced_storage_error_vs_oracle(c1, storage, bound):
    """16-bit storage of the dual field and the time differences: the error
    against the FP64 oracle after every block of the 128x128 stream stays
    below the stated bound (FP16 2e-3, BF16 2e-2 max-abs on u in [1, e])."""
    r, o = make(128, 128, storage=storage)
    worst = 0.0
    for b in evgen.batches(c1.events, 500)[:20]:
        r.push(b.t, b.x, b.y, b.p)
        o.push_events(b)
        r.solve(50)
        o.solve(50)
        worst = max(worst, float(np.abs(r.image(rec.REC_U).astype(np.float64) - o.u).max()))
    print(f"storage={storage} max-abs error vs FP64 oracle over 20 blocks: {worst:.3e}")
    assert worst <= bound


@pytest.fixture(scope="module")
def hd720_oracle():
    """First 10 blocks of the 1280x720 stream (20000 events, 100 iterations
    each) and the FP64 oracle's image after every block."""
    s, bs, _, iters = evgen.hd720(duration_us=15_000)
    blocks = evgen.batches(s.events, bs)[:10]
    o = oracle.Oracle(oracle.Params(1280, 720))
    us = []
    for b in blocks:
        o.push_events(b)
        o.solve(iters)
        us.append(o.u)
    o.close()
    return blocks, iters, us


@pytest.mark.parametrize("storage,bound", [(rec.REC_STORE_F32, 1e-4), (rec.REC_STORE_F16, 2e-3),
                                           (rec.REC_STORE_BF16, 2e-2)])
def test_hd720_precision_vs_oracle(hd720_oracle, storage, bound):
    """1280x720 at 2e7 events/s, 100 iterations per block: max-abs and mean-abs
    error of u against the FP64 oracle over the first 10 blocks, per storage
    of the dual field and time differences."""
    blocks, iters, us = hd720_oracle
    r = rec.Reconstructor(1280, 720, storage=storage)
    worst, mean = 0.0, 0.0
    for b, uo in zip(blocks, us):
        r.push(*device_events(b), on_device=True)
        r.solve(iters)
        d = np.abs(r.image(rec.REC_U).astype(np.float64) - uo)
        worst = max(worst, float(d.max()))
        mean = max(mean, float(d.mean()))
    r.close()
    print(f"hd720 storage={storage}: max-abs {worst:.3e}, worst mean-abs {mean:.3e} "
          f"over 10 blocks")
    assert worst <= bound


@pytest.mark.parametrize("storage", [rec.REC_STORE_F16, rec.REC_STORE_BF16])
def test_reduced_storage_tile_independent(storage):
    """With the same iterations per launch, the 16-bit form gives the same
    bits whatever the tile shape (rounding happens only at launch ends)."""
    W, H = 150, 97
    t, x, y, p = _random_stream(W, H, 4000, seed=77)
    outs = []
    for rows, waves, cols in [(2, 16, 64), (4, 16, 64), (4, 8, 64), (8, 4, 64), (8, 8, 64),
                              (2, 8, 32)]:
        r = rec.Reconstructor(W, H, storage=storage, fuse_iters=6, tile_rows=rows, tile_waves=waves,
                              tile_cols=cols)
        for a in range(0, 4000, 1000):
            r.push(*device_events(evgen.Events(t[a:a + 1000], x[a:a + 1000], y[a:a + 1000],
                                               p[a:a + 1000], np.zeros(1000, np.uint8))),
                   on_device=True)
            r.solve(31)
        outs.append((r.image(rec.REC_U), r.image(rec.REC_STATE_P), r.image(rec.REC_TX)))
        r.close()
    for u, pp, tx in outs[1:]:
        assert np.array_equal(u, outs[0][0])
        assert np.array_equal(pp, outs[0][1])
        assert np.array_equal(tx, outs[0][2])


# --------------------------------------------------------------------------
# Timestamp denoising (TV-L1 before the metric, Section 4)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def noisy():
    spec = evgen.StreamSpec(96, 72, 21, duration_us=60_000, speed_px_s=400.0, omega_rad_s=3.0,
                            noise_frac=0.05)
    return evgen.generate(spec).events


@pytest.mark.parametrize("fuse", [-1, 0])
def test_denoised_time_differences_and_image(noisy, fuse):
    r, o = make(96, 72, tvl1_iters=5, tvl1_lambda=1.0, fuse_iters=fuse)
    n = len(noisy)
    for a in range(0, n - n % 4, n // 4):
        b = noisy.slice(a, a + n // 4)
        r.push(*device_events(b), on_device=True)
        o.push_events(b)
        r.solve(50)
        o.solve(50)
        tx, ty = r.image(rec.REC_TX), r.image(rec.REC_TY)
        assert np.allclose(tx, o.get(oracle.TX32), rtol=1e-6, atol=1e-9)
        assert np.allclose(ty, o.get(oracle.TY32), rtol=1e-6, atol=1e-9)
        assert np.abs(r.image(rec.REC_U).astype(np.float64) - o.u).max() <= U_TOL


@pytest.mark.parametrize("on_device", [False, True])
@pytest.mark.parametrize("iters", [1, 5, 14, 15, 20])
def test_denoised_time_differences_exact(noisy, iters, on_device):
    """Up to 14 iterations the denoising runs as one tiled launch, beyond as
    one launch per half-step; both repeat the oracle's FP64 operations in
    order, so the rounded time differences equal the oracle's bit for bit.
    Device pushes are binned by the one-launch denoiser itself."""
    r, o = make(96, 72, tvl1_iters=iters, tvl1_lambda=1.0)
    n = len(noisy)
    for a in range(0, n - n % 2, n // 2):
        b = noisy.slice(a, a + n // 2)
        if on_device:
            r.push(*device_events(b), on_device=True)
        else:
            r.push(b.t, b.x, b.y, b.p)
        o.push_events(b)
        r.solve(3)
        o.solve(3)
        for which, plane in ((rec.REC_TX, oracle.TX32), (rec.REC_TY, oracle.TY32)):
            g, ref = r.image(which), o.get(plane)
            print(f"tvl1 iters={iters}: max |d| {np.abs(g - ref).max():.3e}")
            assert np.array_equal(g, ref)
    r.close()


@pytest.mark.parametrize("W,H", [(320, 240), (40, 30)])
def test_denoised_time_differences_exact_tile_heights(W, H):
    """The one-launch denoiser takes one row per lane (64 x 16 tiles) when
    those tiles fit on the compute units at once and two rows otherwise:
    320 x 240 at 5 iterations needs 420 one-row tiles (so two rows run),
    40 x 30 a handful.  Both equal the oracle bit for bit."""
    spec = evgen.StreamSpec(W, H, 23, duration_us=20_000, speed_px_s=400.0, omega_rad_s=3.0,
                            noise_frac=0.05)
    ev = evgen.generate(spec).events
    r, o = make(W, H, tvl1_iters=5, tvl1_lambda=1.0)
    n = len(ev)
    for a in range(0, n - n % 2, n // 2):
        b = ev.slice(a, a + n // 2)
        r.push(*device_events(b), on_device=True)
        o.push_events(b)
        r.solve(3)
        o.solve(3)
        for which, plane in ((rec.REC_TX, oracle.TX32), (rec.REC_TY, oracle.TY32)):
            assert np.array_equal(r.image(which), o.get(plane))
    r.close()


def test_denoising_flattens_noise_spikes(noisy):
    """Uniform noise events put isolated, out-of-sequence timestamps into the
    surface; the denoised surface has far fewer large time differences."""
    raw = rec.Reconstructor(96, 72)
    den = rec.Reconstructor(96, 72, tvl1_iters=50, tvl1_lambda=1.0)
    for r in (raw, den):
        r.push(noisy.t, noisy.x, noisy.y, noisy.p)
        r.solve(1)
    big_raw = (np.abs(raw.image(rec.REC_TX)) > 5.0).sum()
    big_den = (np.abs(den.image(rec.REC_TX)) > 5.0).sum()
    assert big_den < 0.5 * big_raw


# --------------------------------------------------------------------------
# Batched solves of several streams
# --------------------------------------------------------------------------

BATCH_SHAPES = [(128, 128), (240, 180), (67, 45), (346, 260), (1, 37), (200, 7), (128, 128),
                (240, 180)]


@pytest.mark.parametrize("mode,tune", [(rec.REC_BATCH_SERIAL, 0), (rec.REC_BATCH_STREAMS, 0),
                                       (rec.REC_BATCH_GRAPH, 0), (rec.REC_BATCH_STREAMS, 50),
                                       (rec.REC_BATCH_GRAPH, 50)])
def test_batch_equals_individual_solves(mode, tune):
    """A batched solve gives each stream the same bits as solving it alone,
    whatever the class geometries (one class per sensor size, each with its
    own autotuned tile and iterations per launch) and however the class
    chains are issued; the autotuner leaves state alone.  In graph mode the
    captured solves are replayed over several blocks (two descriptor
    buffers, folded and scattered pushes, two iteration counts) with the
    program's own eager work and readbacks between replays, and every
    replay is checked.  Untuned, all sizes share one geometry; tuned, the
    sizes may get several.  Pushes: device pointers (folded), host pushes
    above max_events (split and scattered at once) and host pushes of 100
    events through a staging ring of one such push per half (when the ring
    comes back to a half whose push is still recorded, the recorded pushes
    are scattered; the last one or two of a block are folded)."""
    rng = np.random.default_rng(4)
    steps = 6
    streams = []
    for i, (W, H) in enumerate(BATCH_SHAPES):
        n = int(rng.integers(200, 3000))
        streams.append(_random_stream(W, H, steps * n, seed=W * 31 + H + i))
    recs = [rec.Reconstructor(W, H, max_events=128) for (W, H) in BATCH_SHAPES]
    u_before = [r.image(rec.REC_U) for r in recs]
    batch = rec.Batch(recs, tune_iters=tune)
    if not tune:
        # several classes: geometries set per sensor size (32- and 64-column
        # tiles, different iterations per launch)
        assert len(batch.config()) == 1
        for (W, H), geo in zip(BATCH_SHAPES, [(1, 16, 32, 10), (2, 8, 32, 8), (8, 8, 64, 6),
                                              (4, 16, 64, 13)]):
            batch.set_geometry(W, H, *geo)
    cfg = batch.config()
    print(f"mode {mode} tune {tune}: classes {cfg}", flush=True)
    assert 1 <= len(cfg) <= len(set(BATCH_SHAPES))
    assert len(cfg) == 5 or tune
    assert sum(c["streams"] for c in cfg) == len(BATCH_SHAPES)
    for c in cfg:
        assert c["rows"] * c["waves"] * (64 // c["cols"]) > 2 * c["kiters"]
        assert (c["tuned_us"] > 0) == (tune > 0)
    for r, u in zip(recs, u_before):
        assert np.array_equal(r.image(rec.REC_U), u)
    batch.set_mode(mode)
    solo = [rec.Reconstructor(W, H, max_events=128) for (W, H) in BATCH_SHAPES]
    for step in range(steps):
        iters = 50 if step == 4 else 37
        for (t, x, y, p), r, s in zip(streams, recs, solo):
            n = len(t) // steps
            sl = slice(step * n, (step + 1) * n)
            ev = evgen.Events(t[sl], x[sl], y[sl], p[sl], np.zeros(n, np.uint8))
            if step == 3:
                # scattered pushes: no class folds events into its first launch
                r.push(ev.t, ev.x, ev.y, ev.p)
                s.push(ev.t, ev.x, ev.y, ev.p)
            elif step == 5:
                for a in range(0, n, 100):
                    r.push(ev.t[a:a + 100], ev.x[a:a + 100], ev.y[a:a + 100], ev.p[a:a + 100])
                    s.push(ev.t[a:a + 100], ev.x[a:a + 100], ev.y[a:a + 100], ev.p[a:a + 100])
            else:
                r.push(*device_events(ev), on_device=True)
                s.push(*device_events(ev), on_device=True)
        batch.solve(iters)
        for s in solo:
            s.solve(iters)
        for i, (r, s) in enumerate(zip(recs, solo)):
            assert np.array_equal(r.image(rec.REC_U), s.image(rec.REC_U)), (step, i)
            assert np.array_equal(r.image(rec.REC_STATE_P), s.image(rec.REC_STATE_P)), (step, i)
            assert np.array_equal(r.image(rec.REC_T_LAST), s.image(rec.REC_T_LAST)), (step, i)
    batch.close()


@pytest.mark.parametrize("mode", [rec.REC_BATCH_STREAMS, rec.REC_BATCH_GRAPH])
def test_batch_host_pushes_beyond_one_copy_launch(mode):
    """16 cameras, each with four host pushes per block: with the descriptor
    upload that is 65 copies, more than one copy launch takes, so a batched
    solve launches two.  Every camera gets the same bits as its own solve."""
    shapes = [(48 + 3 * i, 40 - i) for i in range(16)]
    streams = [_random_stream(W, H, 3 * 4 * 30, seed=5 * W + H) for (W, H) in shapes]
    recs = [rec.Reconstructor(W, H) for (W, H) in shapes]
    solo = [rec.Reconstructor(W, H) for (W, H) in shapes]
    batch = rec.Batch(recs, tune_iters=0)
    batch.set_mode(mode)
    for blk in range(3):
        for (t, x, y, p), r, o in zip(streams, recs, solo):
            for k in range(4):
                sl = slice((4 * blk + k) * 30, (4 * blk + k + 1) * 30)
                r.push(t[sl], x[sl], y[sl], p[sl])
                o.push(t[sl], x[sl], y[sl], p[sl])
        batch.solve(25)
        for o in solo:
            o.solve(25)
        for i, (r, o) in enumerate(zip(recs, solo)):
            assert np.array_equal(r.image(rec.REC_U), o.image(rec.REC_U)), (blk, i)
            assert np.array_equal(r.image(rec.REC_T_LAST), o.image(rec.REC_T_LAST)), (blk, i)
    batch.close()


@pytest.mark.parametrize("storage", [rec.REC_STORE_F16, rec.REC_STORE_BF16])
def test_batch_16bit_storage_equals_individual_solves(storage):
    """16-bit storage of p and tx, ty in a batch (64- and 32-column classes):
    the same bits as each stream solved alone with the same storage and the
    same iterations per launch (16-bit storage rounds p at the end of every
    launch, so unlike FP32 its bits depend on where the launches split a
    solve, though not on the tile shape)."""
    shapes = [(128, 128), (240, 180), (67, 45)]
    streams = [_random_stream(W, H, 3 * 800, seed=W + 7 * H) for (W, H) in shapes]
    recs = [rec.Reconstructor(W, H, storage=storage) for (W, H) in shapes]
    batch = rec.Batch(recs, tune_iters=0)
    batch.set_geometry(240, 180, 2, 8, 32, 7)
    cfg = batch.config()
    assert len(cfg) == 2
    k_of = {(c["width"], c["height"]): c["kiters"] for c in cfg}
    k_def = [c["kiters"] for c in cfg if (c["width"], c["height"]) != (240, 180)][0]
    solo = [rec.Reconstructor(W, H, storage=storage, fuse_iters=k_of.get((W, H), k_def))
            for (W, H) in shapes]
    for step in range(3):
        for (t, x, y, p), r, s in zip(streams, recs, solo):
            sl = slice(step * 800, (step + 1) * 800)
            ev = evgen.Events(t[sl], x[sl], y[sl], p[sl], np.zeros(800, np.uint8))
            r.push(*device_events(ev), on_device=True)
            s.push(*device_events(ev), on_device=True)
        batch.solve(30)
        for s in solo:
            s.solve(30)
    for r, s in zip(recs, solo):
        assert np.array_equal(r.image(rec.REC_U), s.image(rec.REC_U))
        assert np.array_equal(r.image(rec.REC_STATE_P), s.image(rec.REC_STATE_P))
    batch.close()


def test_batch_geometry_checks():
    """Geometries outside the batched launch's set, halos that leave no
    interior and sizes not in the batch are refused and change nothing."""
    recs = [rec.Reconstructor(64, 32), rec.Reconstructor(40, 40)]
    batch = rec.Batch(recs, tune_iters=0)
    before = batch.config()
    for args in [(64, 32, 3, 3, 64, 4), (64, 32, 8, 8, 48, 4), (64, 32, 1, 16, 64, 4),
                 (64, 32, 8, 8, 64, 32), (64, 32, 1, 16, 32, 16), (64, 32, 8, 8, 64, 0),
                 (65, 32, 8, 8, 64, 6)]:
        with pytest.raises(rec.RecError) as e:
            batch.set_geometry(*args)
        assert e.value.code == rec.REC_EINVAL
    assert batch.config() == before
    batch.set_geometry(40, 40, 2, 8, 32, 15)
    assert len(batch.config()) == 2
    batch.close()


def test_batch_rejects_mixed_contexts():
    a = rec.Reconstructor(64, 32)
    b = rec.Reconstructor(64, 32, storage=rec.REC_STORE_F16)
    c = rec.Reconstructor(64, 32, fuse_iters=0)
    for group in ([a, b], [a, c], [a, a]):
        with pytest.raises(rec.RecError) as e:
            rec.Batch(group, tune_iters=0)
        assert e.value.code == rec.REC_EINVAL
