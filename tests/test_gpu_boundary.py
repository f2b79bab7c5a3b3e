"""Boundary behaviour of the C ABI on the GPU: ownership of device event
arrays, the numeric and state error codes, and the latest-timestamp plane
read into device memory."""
import ctypes

import numpy as np
import pytest

import evgen
import oracle
from paper_1607_06283_amd import rec

from gpu_helpers import U_TOL, device_events, make

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def c1():
    s, _, _, _ = evgen.dvs128(seed=1, n_batches=4)
    return s


@pytest.mark.parametrize("reader", ["image_u", "gap_history", "image_u_device"])
def test_device_arrays_released_after_synchronising_call(c1, reader):
    """rec_get_image and rec_gap_history scatter recorded device-pointer
    pushes before they return, so the caller may reuse the event arrays
    afterwards: push, read u, overwrite the arrays with other (valid)
    events, solve -- the image is that of the original events."""
    import torch
    r, o = make(128, 128)
    blocks = evgen.batches(c1.events, 500)
    for k in range(3):
        b = blocks[k]
        t, x, y, p = device_events(b)
        r.push(t, x, y, p, on_device=True)
        o.push_events(b)
        if reader == "image_u":
            r.image(rec.REC_U)
        elif reader == "gap_history":
            r.gap_history()
        else:
            r.image(rec.REC_U, device=True)
        # overwrite in place with events of another block: a library that
        # still held the pointers would read these instead
        other = blocks[3]
        t.copy_(torch.from_numpy(np.ascontiguousarray(other.t)).cuda())
        x.copy_(torch.from_numpy(np.ascontiguousarray(other.x).view(np.int16)).cuda())
        y.copy_(torch.from_numpy(np.ascontiguousarray(other.y).view(np.int16)).cuda())
        p.copy_(torch.from_numpy(np.ascontiguousarray(other.p)).cuda())
        torch.cuda.synchronize()
        st = r.solve(50, stats=True)
        o.solve(50)
        assert st.events_in_batch == len(b) and st.t_ref_us == o.t_ref
        assert np.array_equal(r.image(rec.REC_T_LAST), o.get(oracle.TLAST))
        assert np.abs(r.image(rec.REC_U).astype(np.float64) - o.u).max() <= U_TOL
    r.close()


def test_latest_timestamps_on_device_resolve_never_fired_pixels(c1):
    """The int64 plane read into device memory resolves pixels that never
    fired to the stream's first timestamp, as the host readback does."""
    r, o = make(128, 128)
    b = c1.events.slice(0, 300)
    r.push(*device_events(b), on_device=True)
    o.push_events(b)
    r.solve(10)
    dev = r.image(rec.REC_T_LAST, device=True).cpu().numpy()
    host = r.image(rec.REC_T_LAST)
    assert np.array_equal(dev, host) and np.array_equal(host, o.get(oracle.TLAST))
    assert (host >= int(b.t[0])).all()
    r.close()


def test_numeric_error_reported_by_solve_with_stats():
    """A finite initial image near the FP32 maximum: the block's events
    multiply it past FP32's range, so the data image holds infinities and
    the sampled gap and energy are not finite: rec_solve with stats returns
    REC_ENUMERIC (through the plain C entry points)."""
    W, H = 32, 24
    prm = rec.rec_default_params(W, H, gap_every=10)
    import torch
    nbytes = rec.rec_workspace_bytes(prm)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    u0 = np.full(W * H, 3.0e38, np.float32)
    rc, ctx = rec.rec_init(prm, ws.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream, u0)
    assert rc == rec.REC_OK
    n = 50
    t = evgen.T0_US + np.arange(n, dtype=np.int64)
    x = (np.arange(n) % W).astype(np.uint16)
    y = (np.arange(n) % H).astype(np.uint16)
    pol = np.ones(n, np.int8)
    assert rec.rec_push_events(ctx, t, x, y, pol, n, 0) == rec.REC_OK
    rc, st = rec.rec_solve(ctx, 20, want_stats=True)
    assert rc == rec.REC_ENUMERIC
    assert not (np.isfinite(st.gap) and np.isfinite(st.energy))
    assert rec.rec_destroy(ctx) == rec.REC_OK


def test_destroy_of_a_context_held_by_a_batch_is_refused():
    """rec_destroy returns REC_ESTATE and releases nothing while a live batch
    holds the context; after rec_batch_destroy it succeeds."""
    a = rec.Reconstructor(64, 32)
    b = rec.Reconstructor(40, 30)
    batch = rec.Batch([a, b], tune_iters=0)
    assert rec.rec_destroy(a.ctx) == rec.REC_ESTATE
    with pytest.raises(rec.RecError) as e:
        a.close()
    assert e.value.code == rec.REC_ESTATE
    # the context still works
    ev = evgen.Events(evgen.T0_US + np.arange(10, dtype=np.int64),
                      np.arange(10, dtype=np.uint16), np.arange(10, dtype=np.uint16),
                      np.ones(10, np.int8), np.zeros(10, np.uint8))
    a.push(*device_events(ev), on_device=True)
    batch.solve(20)
    assert np.isfinite(a.image(rec.REC_U)).all()
    batch.close()
    a.close()
    b.close()
    assert a.ctx is None and b.ctx is None


@pytest.mark.parametrize("storage,on_device", [(rec.REC_STORE_F32, False), (rec.REC_STORE_F32, True),
                                               (rec.REC_STORE_F16, False)])
def test_checkpoint_resume_gives_the_same_bits(c1, storage, on_device):
    """A stream checkpointed after a solve (u, p, latest timestamps, t_ref)
    and imported into a fresh context continues with the same bits as the
    original context, block after block; a context given the state of a
    stream with no events behaves like a new one."""
    import torch
    blocks = evgen.batches(c1.events, 500)[:4]
    a = rec.Reconstructor(128, 128, storage=storage)
    for b in blocks[:2]:
        a.push(*device_events(b), on_device=True)
        a.solve(50)
    ck = a.state()
    assert ck["t_ref"] == int(blocks[1].t[-1])
    r = rec.Reconstructor(128, 128, storage=storage)
    if on_device:
        r.set_state(torch.from_numpy(ck["u"]).cuda(), torch.from_numpy(ck["p"]).cuda(),
                    torch.from_numpy(ck["t_last"]).cuda(), ck["t_ref"])
    else:
        r.set_state(ck["u"], ck["p"], ck["t_last"], ck["t_ref"])
    assert r.times() == (int(ck["t_last"].min()), ck["t_ref"], True)
    assert a.times()[0] == int(blocks[0].t[0]) == int(ck["t_last"].min())
    for b in blocks[2:]:
        for q in (a, r):
            q.push(*device_events(b), on_device=True)
            q.solve(37)
        for plane in (rec.REC_U, rec.REC_STATE_P, rec.REC_T_LAST, rec.REC_TX, rec.REC_F):
            assert np.array_equal(a.image(plane), r.image(plane)), plane
    # a stream with no event: same as a new context
    fresh, empty = rec.Reconstructor(128, 128, storage=storage), rec.Reconstructor(128, 128, storage=storage)
    empty.set_state(np.full((128, 128), np.exp(0.5), np.float32), None, None, rec.NO_EVENT)
    assert empty.times() == (0, 0, False)
    for q in (fresh, empty):
        q.push(*device_events(blocks[0]), on_device=True)
        q.solve(20)
    assert np.array_equal(fresh.image(rec.REC_U), empty.image(rec.REC_U))
    assert np.array_equal(fresh.image(rec.REC_T_LAST), empty.image(rec.REC_T_LAST))
    for q in (a, r, fresh, empty):
        q.close()


def test_set_state_checks():
    """Bad values, timestamps after t_ref and pending pushes are refused
    before anything changes."""
    r = rec.Reconstructor(16, 8)
    u = np.full((8, 16), 1.5, np.float32)
    tl = np.full((8, 16), evgen.T0_US, np.int64)
    for bad_u, bad_p, bad_t, code in [
            (np.where(np.arange(128).reshape(8, 16) == 5, 0.0, u), None, tl, rec.REC_EINVAL),
            (u, np.full((3, 8, 16), np.nan, np.float32), tl, rec.REC_EINVAL),
            (u, None, tl + 1, rec.REC_EORDER)]:
        with pytest.raises(rec.RecError) as e:
            r.set_state(bad_u, bad_p, bad_t, evgen.T0_US)
        assert e.value.code == code
    assert np.array_equal(r.image(rec.REC_U), np.full((8, 16), np.exp(0.5), np.float32))
    r.push(np.array([evgen.T0_US], np.int64), np.array([3], np.uint16), np.array([2], np.uint16),
           np.array([1], np.int8))
    with pytest.raises(rec.RecError) as e:
        r.set_state(u, None, tl, evgen.T0_US)
    assert e.value.code == rec.REC_ESTATE
    r.close()


FAULT_SCRIPT = r"""
import sys
import numpy as np
sys.path.insert(0, {root!r})
import torch
from paper_1607_06283_amd import rec
torch.cuda.set_device(0)
r = rec.Reconstructor(64, 32)
t = np.arange(100, dtype=np.int64) + 10**10
x = (np.arange(100) % 64).astype(np.uint16)
y = (np.arange(100) % 32).astype(np.uint16)
p = np.where(np.arange(100) % 2 == 0, 1, -1).astype(np.int8)
r.push(t, x, y, p)
rc, _ = rec.rec_solve(r.ctx, 50, False)
print("solve", rc, rec.rec_strerror(rc), flush=True)
"""


def test_injected_launch_failure_is_reported():
    """With REC_FAULT_AFTER=n every launch after the process's first n fails
    without being issued: the solve returns REC_EDEVICE (the host-side
    error path; no kernel runs, so the GPU is left alone)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, REC_FAULT_AFTER="2")  # init and the push launch, then failures
    out = subprocess.run([sys.executable, "-c", FAULT_SCRIPT.format(root=root)], env=env,
                         capture_output=True, text=True, timeout=240)
    print(out.stdout, out.stderr[-2000:])
    assert out.returncode == 0
    assert f"solve {rec.REC_EDEVICE} HIP runtime error" in out.stdout
