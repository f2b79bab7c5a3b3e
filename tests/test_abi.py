"""The C-ABI library on the CPU: it loads, exports every declared symbol, and
its host-side validation works without touching a GPU."""
import math
import os
import re

import numpy as np
import pytest

from paper_1607_06283_amd import rec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rec.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rec_[a-z_]+)\s*\(", src)))


def test_exports_match_header():
    lib = rec.load()
    names = declared_functions()
    assert set(names) == set(rec.EXPORTS)
    for n in names:
        getattr(lib, n)


def test_struct_sizes_match_header_layout():
    # rec_params: 2 int32, 9 double, 8 int32, 1 double, tile_cols, 3 int32 reserved
    import ctypes
    assert ctypes.sizeof(rec.rec_params) == 136
    assert rec.rec_params.tvl1_lambda.offset == 112
    assert rec.rec_params.tile_cols.offset == 120
    assert ctypes.sizeof(rec.rec_stats) == 40
    assert ctypes.sizeof(rec.rec_profile_t) == 72


def test_default_params():
    p = rec.rec_default_params(128, 128)
    assert p.width == 128 and p.height == 128
    assert p.lambda_ == 90.0 and p.delta_pos == 0.2 and p.delta_neg == 0.2
    assert p.u_min == 1.0 and abs(p.u_max - math.e) < 1e-15
    assert abs(p.tau * p.sigma * (8 + 4 * math.sqrt(2)) - 1.0) < 1e-12
    assert p.time_unit_us == 1000.0 and p.iters == 50
    assert rec.rec_check_params(p) == rec.REC_OK
    assert rec.rec_workspace_bytes(p) >= 128 * 128 * 60


@pytest.mark.parametrize("field,value", [
    ("width", 0), ("height", -3), ("width", 70000), ("lambda_", 0.0), ("lambda_", float("nan")),
    ("delta_pos", -0.1), ("u_min", 0.0), ("u_max", 0.5), ("tau", 0.6), ("sigma", 0.0),
    ("time_unit_us", -1.0), ("time_unit_us", float("inf")), ("u_init", 0.0), ("iters", -1),
    ("gap_every", -2), ("fuse_iters", 40), ("max_events", 0), ("tile_rows", 3),
    ("storage", 3), ("storage", -1), ("tvl1_iters", -1), ("tvl1_iters", 20000),
])
def test_bad_params_rejected(field, value):
    p = rec.rec_default_params(64, 48)
    setattr(p, field, value)
    if field == "tile_rows":
        p.tile_waves = 4
    assert rec.rec_check_params(p) == rec.REC_EINVAL
    assert rec.rec_workspace_bytes(p) == 0


def test_reduced_storage_needs_fused_loop():
    p = rec.rec_default_params(64, 48)
    for st in (rec.REC_STORE_BF16, rec.REC_STORE_F16):
        p.storage = st
        p.fuse_iters = -1
        assert rec.rec_check_params(p) == rec.REC_OK
        p.fuse_iters = 0
        assert rec.rec_check_params(p) == rec.REC_EINVAL
        p.fuse_iters = -1
        p.tile_rows, p.tile_waves = 16, 4   # no 16-bit variant of this tile
        assert rec.rec_check_params(p) == rec.REC_EINVAL
        p.tile_rows, p.tile_waves = 4, 16
        assert rec.rec_check_params(p) == rec.REC_OK
        p.tile_rows, p.tile_waves = 0, 0


def test_tile_cols_params():
    p = rec.rec_default_params(64, 48)
    assert p.tile_cols == 0
    p.tile_cols = 32                      # only together with tile_rows / tile_waves
    assert rec.rec_check_params(p) == rec.REC_EINVAL
    p.tile_rows, p.tile_waves = 2, 8
    assert rec.rec_check_params(p) == rec.REC_OK
    for cols in (16, 48, 128, -32):
        p.tile_cols = cols
        assert rec.rec_check_params(p) == rec.REC_EINVAL
    p.tile_cols = 32
    p.tile_rows, p.tile_waves = 6, 8      # no 32-column variant of this tile
    assert rec.rec_check_params(p) == rec.REC_EINVAL
    p.tile_rows, p.tile_waves = 1, 16
    assert rec.rec_check_params(p) == rec.REC_OK
    p.storage = rec.REC_STORE_BF16        # 16-bit storage: 2x8 only
    assert rec.rec_check_params(p) == rec.REC_EINVAL
    p.tile_rows, p.tile_waves = 2, 8
    assert rec.rec_check_params(p) == rec.REC_OK
    p.tile_cols = 64
    assert rec.rec_check_params(p) == rec.REC_EINVAL   # 2x8 of 64 columns: FP32 only


def test_denoising_params():
    p = rec.rec_default_params(32, 32)
    assert p.tvl1_iters == 0 and p.tvl1_lambda == 1.0
    p.tvl1_iters = 5
    assert rec.rec_check_params(p) == rec.REC_OK
    base = rec.rec_workspace_bytes(rec.rec_default_params(32, 32))
    assert rec.rec_workspace_bytes(p) >= base + 5 * 8 * 32 * 32  # FP64 planes only when on
    p.tvl1_lambda = 0.0
    assert rec.rec_check_params(p) == rec.REC_EINVAL


def test_step_size_bound():
    """tau sigma ||L_g||^2 <= 1 with ||L_g||^2 <= 8 + 4 sqrt 2 (Section 3.2)."""
    p = rec.rec_default_params(8, 8)
    p.tau = 0.2
    p.sigma = 1.0 / (0.2 * (8 + 4 * math.sqrt(2)))
    assert rec.rec_check_params(p) == rec.REC_OK
    p.sigma *= 1.001
    assert rec.rec_check_params(p) == rec.REC_EINVAL


def _ev(t, x, y, p):
    return (np.array(t, np.int64), np.array(x, np.uint16), np.array(y, np.uint16),
            np.array(p, np.int8))


def test_event_validation_codes():
    t, x, y, p = _ev([5, 6, 6, 9], [0, 3, 2, 1], [0, 1, 2, 2], [1, -1, 1, -1])
    assert rec.rec_check_events(t, x, y, p, 4, 3) == rec.REC_OK
    assert rec.rec_check_events(t, x, y, p, 4, 3, t_prev=5) == rec.REC_OK
    assert rec.rec_check_events(t, x, y, p, 4, 3, t_prev=6) == rec.REC_EORDER
    assert rec.rec_check_events(t, x, y, p, 3, 3) == rec.REC_ERANGE
    assert rec.rec_check_events(t, x, y, p, 4, 2) == rec.REC_ERANGE
    bad = p.copy()
    bad[2] = 0
    assert rec.rec_check_events(t, x, y, bad, 4, 3) == rec.REC_EINVAL
    tt = t.copy()
    tt[2] = 4
    assert rec.rec_check_events(tt, x, y, p, 4, 3) == rec.REC_EORDER
    assert rec.rec_check_events(t[:0], x[:0], y[:0], p[:0], 4, 3) == rec.REC_OK


def _check_events_reference(t, x, y, p, W, H, t_prev):
    """The validation rule event by event: the first event that fails a check
    decides, with its first failing check (polarity, then position, then
    order against the previous timestamp)."""
    prev = t_prev
    for i in range(len(t)):
        if p[i] not in (1, -1):
            return rec.REC_EINVAL
        if x[i] >= W or y[i] >= H:
            return rec.REC_ERANGE
        if t[i] < prev:
            return rec.REC_EORDER
        prev = t[i]
    return rec.REC_OK


def test_event_validation_matches_the_sequential_rule():
    """Streams spanning several of the validator's 512-event blocks, with one
    or two planted faults (at block boundaries among other places, an event
    failing several checks at once, an order fault across two blocks): the
    code of the sequential rule every time."""
    rng = np.random.default_rng(11)
    W, H = 70, 40
    sizes = [1, 511, 512, 513, 1024, 1500, 2049]
    cases = 0
    for n in sizes:
        for trial in range(12):
            t = np.sort(rng.integers(0, 10 * n, n)).astype(np.int64)
            x = rng.integers(0, W, n).astype(np.uint16)
            y = rng.integers(0, H, n).astype(np.uint16)
            p = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
            assert rec.rec_check_events(t, x, y, p, W, H) == rec.REC_OK
            picks = [int(i) for i in rng.integers(0, n, 2)] + [min(n - 1, 511), min(n - 1, 512)]
            for i in rng.choice(picks, size=1 + trial % 2, replace=False):
                kind = (trial + int(i)) % 5
                if kind == 0:
                    p[i] = (0, 2, -2, 127, -128)[trial % 5]
                elif kind == 1:
                    x[i] = W + trial
                elif kind == 2:
                    y[i] = H
                elif kind == 3 and i > 0:
                    t[i] = t[i - 1] - 1
                else:  # several checks fail at once
                    p[i] = 0
                    x[i] = W
                    if i > 0:
                        t[i] = t[i - 1] - 5
            for t_prev in (-(2 ** 63), int(t[0]), int(t[0]) + 1):
                want = _check_events_reference(t, x, y, p, W, H, t_prev)
                assert rec.rec_check_events(t, x, y, p, W, H, t_prev=t_prev) == want, (n, trial)
                cases += 1
    assert cases == len(sizes) * 12 * 3


def test_strerror_covers_codes():
    for c in range(0, -8, -1):
        assert rec.rec_strerror(c) != "unknown status code"
    assert rec.rec_strerror(-99) == "unknown status code"


def test_init_rejects_without_touching_device():
    """Invalid parameters, a NULL or misaligned workspace and a short workspace
    are refused before any device call."""
    p = rec.rec_default_params(16, 16)
    rc, h = rec.rec_init(p, None, 0, None)
    assert rc == rec.REC_EINVAL and h is None
    rc, h = rec.rec_init(p, 0x1001, 1 << 20, None)
    assert rc == rec.REC_EINVAL
    rc, h = rec.rec_init(p, 0x10000, 16, None)
    assert rc == rec.REC_ENOMEM
    p.lambda_ = -1.0
    rc, h = rec.rec_init(p, 0x10000, 1 << 30, None)
    assert rc == rec.REC_EINVAL


def test_null_context_calls():
    assert rec.rec_push_events(None, None, None, None, None, 1, 0) == rec.REC_EINVAL
    assert rec.rec_solve(None, 5)[0] == rec.REC_EINVAL
    assert rec.rec_sync(None) == rec.REC_EINVAL
    assert rec.rec_destroy(None) == rec.REC_OK
    assert rec.rec_get_times(None)[0] == rec.REC_EINVAL
    u = np.ones(4, np.float32)
    assert rec.rec_set_state(None, u, None, None, rec.NO_EVENT, 0) == rec.REC_EINVAL
    assert rec.rec_batch_classes(None) == rec.REC_EINVAL
    assert rec.rec_batch_set_mode(None, rec.REC_BATCH_GRAPH) == rec.REC_EINVAL
    assert rec.rec_batch_set_geometry(None, 64, 32, 8, 8, 64, 6) == rec.REC_EINVAL
    assert rec.rec_batch_solve(None, 10) == rec.REC_EINVAL
    assert rec.rec_batch_destroy(None) == rec.REC_OK
    import ctypes
    c = rec.rec_batch_class()
    assert rec.load().rec_batch_config(None, 0, ctypes.byref(c)) == rec.REC_EINVAL
    assert ctypes.sizeof(rec.rec_batch_class) == 40


def _diff_desc(**kw):
    d = rec.rec_diff_desc_make(70, 37, 2, 30, 7)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_diff_desc_layout_and_workspace():
    import ctypes
    assert ctypes.sizeof(rec.rec_diff_desc) == 56
    assert ctypes.sizeof(rec.rec_diff_inputs) == 64
    assert ctypes.sizeof(rec.rec_diff_grads) == 32
    d = _diff_desc()
    a = lambda x: (x + 255) // 256 * 256
    plane = a(70 * 37 * 2 * 4)
    C = math.ceil(30 / 7)
    blocks = 2 * 10 * 2  # ceil(70/64) x ceil(37/4) x images
    want = plane * (1 + 4 * (C + 1) + 4 * (7 - 1) + 7 + 5) + a(blocks * 3 * 8)
    assert rec.rec_diff_workspace_bytes(d) == want


@pytest.mark.parametrize("field,value", [
    ("width", 0), ("height", 70000), ("batch", 0), ("iters", -1), ("ckpt_every", 0),
    ("ckpt_every", 31), ("unfused", 2), ("tau", 0.0), ("sigma", float("nan")),
    ("tau", 0.5), ("u_min", 0.0), ("u_max", 0.5),
])
def test_diff_bad_desc(field, value):
    d = _diff_desc(**{field: value})
    assert rec.rec_diff_workspace_bytes(d) == 0
    inp = rec.rec_diff_inputs(0x1000, None, 0x1000, 0x1000, 0x1000, 0x1000, None, 0x1000)
    assert rec.rec_diff_forward(d, inp, 0x1000, None, 0x10000, 1 << 30, None) == rec.REC_EINVAL


def test_diff_rejects_without_touching_device():
    d = _diff_desc()
    n = rec.rec_diff_workspace_bytes(d)
    inp = rec.rec_diff_inputs(0x1000, None, 0x1000, 0x1000, 0x1000, 0x1000, None, 0x1000)
    missing = rec.rec_diff_inputs(0x1000, None, 0x1000, None, 0x1000, 0x1000, None, 0x1000)
    assert rec.rec_diff_forward(d, missing, 0x1000, None, 0x10000, n, None) == rec.REC_EINVAL
    assert rec.rec_diff_forward(d, inp, None, None, 0x10000, n, None) == rec.REC_EINVAL
    assert rec.rec_diff_forward(d, inp, 0x1000, None, 0x10001, n, None) == rec.REC_EINVAL
    assert rec.rec_diff_forward(d, inp, 0x1000, None, 0x10000, n - 1, None) == rec.REC_ENOMEM
    g = rec.rec_diff_grads(None, None, None, None)
    assert rec.rec_diff_backward(d, inp, None, None, g, 0x10000, n - 1, None) == rec.REC_ENOMEM
    assert rec.rec_diff_backward(d, inp, None, None, g, None, n, None) == rec.REC_EINVAL


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built library every entry raises: there is no CPU path to
    fall back to."""
    monkeypatch.setattr(rec, "_lib", None)
    monkeypatch.setattr(rec, "LIB_PATH", "/nonexistent/librec.so")
    with pytest.raises(RuntimeError, match="missing"):
        rec.load()
    with pytest.raises(RuntimeError, match="missing"):
        rec.rec_default_params(64, 64)
