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
