"""ctypes binding of ``librec.so`` (the C ABI declared in include/rec.h).

The functions below carry the C names and only marshal arguments; every step
of the reconstruction runs in the library's HIP kernels.  ``Reconstructor``
adds the PyTorch plumbing: the device workspace is a ``torch.uint8`` tensor
on the current CUDA (HIP) device and launches go to torch's current stream.

The library must have been built (``paper_1607_06283_amd.build.build()``);
importing this module without it raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librec.so")

REC_OK, REC_EINVAL, REC_ERANGE, REC_EORDER, REC_EDEVICE, REC_ENUMERIC, REC_ESTATE, REC_ENOMEM = (
    0, -1, -2, -3, -4, -5, -6, -7)
(REC_U, REC_F, REC_TIME, REC_METRIC_G, REC_STATE_P, REC_TX, REC_TY, REC_COUNT_POS,
 REC_COUNT_NEG, REC_T_LAST) = range(10)

REC_STORE_F32, REC_STORE_BF16, REC_STORE_F16 = 0, 1, 2
REC_BATCH_SERIAL, REC_BATCH_STREAMS, REC_BATCH_GRAPH = 0, 1, 2

_PLANE_DTYPE = {REC_COUNT_POS: np.int32, REC_COUNT_NEG: np.int32, REC_T_LAST: np.int64}


class rec_params(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("lambda_", ctypes.c_double),
        ("delta_pos", ctypes.c_double), ("delta_neg", ctypes.c_double),
        ("u_min", ctypes.c_double), ("u_max", ctypes.c_double),
        ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
        ("time_unit_us", ctypes.c_double),
        ("u_init", ctypes.c_double),
        ("iters", ctypes.c_int32),
        ("gap_every", ctypes.c_int32),
        ("fuse_iters", ctypes.c_int32),
        ("max_events", ctypes.c_int32),
        ("tile_rows", ctypes.c_int32),
        ("tile_waves", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("tvl1_iters", ctypes.c_int32),
        ("tvl1_lambda", ctypes.c_double),
        ("tile_cols", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


class rec_stats(ctypes.Structure):
    _fields_ = [
        ("gap", ctypes.c_double), ("energy", ctypes.c_double),
        ("iters_run", ctypes.c_int32), ("gap_samples", ctypes.c_int32),
        ("t_ref_us", ctypes.c_int64), ("events_in_batch", ctypes.c_int64),
    ]


class rec_profile_t(ctypes.Structure):
    _fields_ = [
        ("ms", ctypes.c_double * 4),
        ("launches", ctypes.c_int64 * 4),
        ("pd_pixel_iters", ctypes.c_int64),
    ]


EXPORTS = (
    "rec_default_params", "rec_check_params", "rec_workspace_bytes", "rec_check_events",
    "rec_init", "rec_push_events", "rec_solve", "rec_get_image", "rec_gap_history",
    "rec_get_times", "rec_set_state",
    "rec_sync", "rec_profile", "rec_profile_read", "rec_destroy", "rec_strerror",
    "rec_batch_workspace_bytes", "rec_batch_init", "rec_batch_solve", "rec_batch_config",
    "rec_batch_classes", "rec_batch_set_geometry", "rec_batch_set_mode", "rec_batch_destroy",
    "rec_diff_workspace_bytes", "rec_diff_forward", "rec_diff_backward",
    "rec_diff_forward_noalloc",
)


class rec_batch_class(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("streams", ctypes.c_int32),
        ("rows", ctypes.c_int32), ("waves", ctypes.c_int32), ("cols", ctypes.c_int32),
        ("kiters", ctypes.c_int32), ("tiles", ctypes.c_int32), ("tuned_us", ctypes.c_double),
    ]


class rec_diff_desc(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("iters", ctypes.c_int32), ("ckpt_every", ctypes.c_int32), ("unfused", ctypes.c_int32),
        ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
        ("u_min", ctypes.c_double), ("u_max", ctypes.c_double),
    ]


class rec_diff_inputs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("u0", "p0", "npos", "nneg", "tx", "ty", "w", "theta")]


class rec_diff_grads(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("u0", "p0", "w", "theta")]

_lib = None
_vp = ctypes.c_void_p


def load() -> ctypes.CDLL:
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1607_06283_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(rec_params)
    lib.rec_default_params.restype = None
    lib.rec_default_params.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    lib.rec_check_params.restype = ctypes.c_int
    lib.rec_check_params.argtypes = [P]
    lib.rec_workspace_bytes.restype = ctypes.c_size_t
    lib.rec_workspace_bytes.argtypes = [P]
    lib.rec_check_events.restype = ctypes.c_int
    lib.rec_check_events.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int64]
    lib.rec_init.restype = ctypes.c_int
    lib.rec_init.argtypes = [P, _vp, ctypes.c_size_t, _vp, _vp, ctypes.POINTER(_vp)]
    lib.rec_push_events.restype = ctypes.c_int
    lib.rec_push_events.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_int]
    lib.rec_solve.restype = ctypes.c_int
    lib.rec_solve.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(rec_stats)]
    lib.rec_get_image.restype = ctypes.c_int
    lib.rec_get_image.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int]
    lib.rec_gap_history.restype = ctypes.c_int
    lib.rec_gap_history.argtypes = [_vp, _vp, _vp, ctypes.c_int32]
    lib.rec_get_times.restype = ctypes.c_int
    lib.rec_get_times.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
    lib.rec_set_state.restype = ctypes.c_int
    lib.rec_set_state.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_int]
    lib.rec_sync.restype = ctypes.c_int
    lib.rec_sync.argtypes = [_vp]
    lib.rec_profile.restype = ctypes.c_int
    lib.rec_profile.argtypes = [_vp, ctypes.c_int]
    lib.rec_profile_read.restype = ctypes.c_int
    lib.rec_profile_read.argtypes = [_vp, ctypes.POINTER(rec_profile_t)]
    lib.rec_destroy.restype = ctypes.c_int
    lib.rec_destroy.argtypes = [_vp]
    lib.rec_strerror.restype = ctypes.c_char_p
    lib.rec_strerror.argtypes = [ctypes.c_int]
    lib.rec_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.rec_batch_workspace_bytes.argtypes = [_vp, ctypes.c_int32]
    lib.rec_batch_init.restype = ctypes.c_int
    lib.rec_batch_init.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_size_t, ctypes.c_int32,
                                   ctypes.POINTER(_vp)]
    lib.rec_batch_solve.restype = ctypes.c_int
    lib.rec_batch_solve.argtypes = [_vp, ctypes.c_int32]
    lib.rec_batch_config.restype = ctypes.c_int
    lib.rec_batch_config.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(rec_batch_class)]
    lib.rec_batch_classes.restype = ctypes.c_int
    lib.rec_batch_classes.argtypes = [_vp]
    lib.rec_batch_set_geometry.restype = ctypes.c_int
    lib.rec_batch_set_geometry.argtypes = [_vp] + [ctypes.c_int32] * 6
    lib.rec_batch_set_mode.restype = ctypes.c_int
    lib.rec_batch_set_mode.argtypes = [_vp, ctypes.c_int32]
    lib.rec_batch_destroy.restype = ctypes.c_int
    lib.rec_batch_destroy.argtypes = [_vp]
    D = ctypes.POINTER(rec_diff_desc)
    lib.rec_diff_workspace_bytes.restype = ctypes.c_size_t
    lib.rec_diff_workspace_bytes.argtypes = [D]
    lib.rec_diff_forward.restype = ctypes.c_int
    lib.rec_diff_forward.argtypes = [D, ctypes.POINTER(rec_diff_inputs), _vp, _vp, _vp,
                                     ctypes.c_size_t, _vp]
    lib.rec_diff_forward_noalloc.restype = ctypes.c_int
    lib.rec_diff_forward_noalloc.argtypes = [D, ctypes.POINTER(rec_diff_inputs), _vp, _vp, _vp]
    lib.rec_diff_backward.restype = ctypes.c_int
    lib.rec_diff_backward.argtypes = [D, ctypes.POINTER(rec_diff_inputs), _vp, _vp,
                                      ctypes.POINTER(rec_diff_grads), _vp, ctypes.c_size_t, _vp]
    _lib = lib
    return lib


class RecError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {rec_strerror(code)} ({code})")


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise RecError(rc, where)
    return rc


def _addr(a) -> Optional[int]:
    """Data pointer of a numpy array or torch tensor; ints pass through as
    addresses and None as NULL."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


# ---------------------------------------------------------------------------
# C functions, same names
# ---------------------------------------------------------------------------

def rec_default_params(width: int, height: int, **overrides) -> rec_params:
    p = rec_params()
    load().rec_default_params(ctypes.byref(p), int(width), int(height))
    for k, v in overrides.items():
        setattr(p, "lambda_" if k in ("lambda", "lam") else k, v)
    return p


def rec_check_params(prm: rec_params) -> int:
    return load().rec_check_params(ctypes.byref(prm))


def rec_workspace_bytes(prm: rec_params) -> int:
    return load().rec_workspace_bytes(ctypes.byref(prm))


def rec_check_events(t, x, y, p, width: int, height: int, t_prev: int = -(1 << 63)) -> int:
    n = int(len(t))
    return load().rec_check_events(_addr(t), _addr(x), _addr(y), _addr(p), n, int(width),
                                   int(height), int(t_prev))


def rec_init(prm: rec_params, workspace_ptr: int, workspace_bytes: int, stream_ptr: int,
             u0: Optional[np.ndarray] = None) -> Tuple[int, Optional[int]]:
    h = _vp()
    u = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float32)
    rc = load().rec_init(ctypes.byref(prm), workspace_ptr, int(workspace_bytes), stream_ptr,
                         _addr(u), ctypes.byref(h))
    return rc, h.value


def rec_push_events(ctx: int, t, x, y, p, n: int, on_device: int) -> int:
    return load().rec_push_events(ctx, _addr(t), _addr(x), _addr(y), _addr(p), int(n),
                                  int(on_device))


def rec_solve(ctx: int, iters: int, want_stats: bool = False) -> Tuple[int, Optional[rec_stats]]:
    st = rec_stats() if want_stats else None
    rc = load().rec_solve(ctx, int(iters), ctypes.byref(st) if st is not None else None)
    return rc, st


def rec_get_image(ctx: int, which: int, out, on_device: int) -> int:
    return load().rec_get_image(ctx, int(which), _addr(out), int(on_device))


def rec_gap_history(ctx: int, cap: int = 4096) -> Tuple[np.ndarray, np.ndarray]:
    g = np.zeros(max(cap, 1))
    e = np.zeros(max(cap, 1))
    n = _check(load().rec_gap_history(ctx, g.ctypes.data, e.ctypes.data, int(cap)),
               "rec_gap_history")
    return g[:n], e[:n]


def rec_get_times(ctx: int) -> Tuple[int, int, int, int]:
    """(status, t_first, t_ref, started)."""
    tf, tr, st = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    rc = load().rec_get_times(ctx, ctypes.byref(tf), ctypes.byref(tr), ctypes.byref(st))
    return rc, tf.value, tr.value, st.value


NO_EVENT = -(1 << 63)  # t_ref of rec_set_state for a stream that has seen no event


def rec_set_state(ctx: int, u, p, t_last, t_ref: int, on_device: int) -> int:
    return load().rec_set_state(ctx, _addr(u), _addr(p), _addr(t_last), int(t_ref),
                                int(on_device))


def rec_sync(ctx: int) -> int:
    return load().rec_sync(ctx)


def rec_profile(ctx: int, enable: bool) -> int:
    return load().rec_profile(ctx, 1 if enable else 0)


def rec_profile_read(ctx: int) -> rec_profile_t:
    out = rec_profile_t()
    _check(load().rec_profile_read(ctx, ctypes.byref(out)), "rec_profile_read")
    return out


def rec_destroy(ctx: Optional[int]) -> int:
    return load().rec_destroy(ctx)


def rec_strerror(code: int) -> str:
    return load().rec_strerror(int(code)).decode()


# ---------------------------------------------------------------------------
# Convenience wrapper: torch provides the device memory and the stream
# ---------------------------------------------------------------------------

class Reconstructor:
    """One event stream on one GPU.

    ``params`` may be a ``rec_params`` or keyword overrides of the defaults.
    """

    def __init__(self, width: int, height: int, params: Optional[rec_params] = None,
                 u0: Optional[np.ndarray] = None, device=None, stream=None, **overrides):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        self.torch = torch
        self.prm = params if params is not None else rec_default_params(width, height, **overrides)
        if params is not None and overrides:
            for k, v in overrides.items():
                setattr(self.prm, "lambda_" if k in ("lambda", "lam") else k, v)
        _check(rec_check_params(self.prm), "rec_check_params")
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        nbytes = rec_workspace_bytes(self.prm)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            rc, h = rec_init(self.prm, self.workspace.data_ptr(), nbytes,
                             self.stream.cuda_stream, u0)
        _check(rc, "rec_init")
        self.ctx = h
        self.shape = (self.prm.height, self.prm.width)
        # device event tensors pushed but not yet consumed: the library reads
        # them when the next solve runs or a synchronising call (image, sync,
        # gap history) scatters them, so they are kept alive until such a
        # call has succeeded (stream order covers the solve's own launches)
        self._pending = []

    def close(self):
        """Release the context.  Raises RecError(REC_ESTATE) and keeps it
        while a live Batch still holds it."""
        if getattr(self, "ctx", None):
            rc = rec_destroy(self.ctx)
            if rc == REC_ESTATE:
                raise RecError(rc, "rec_destroy")
            self.ctx = None
            self._pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, t, x, y, p, on_device: Optional[bool] = None) -> None:
        """Push events given as numpy arrays (host) or torch tensors (device)."""
        n = int(t.shape[0])
        if on_device is None:
            on_device = not isinstance(t, np.ndarray)
        if on_device:
            for a in (t, x, y, p):
                if isinstance(a, np.ndarray) or getattr(a, "device", None) is None or \
                        a.device.type != "cuda":
                    raise ValueError("on_device pushes need device (HIP) tensors")
                if not a.is_contiguous():
                    raise ValueError("event tensors must be contiguous")
            for a, size, name in ((t, 8, "t"), (x, 2, "x"), (y, 2, "y"), (p, 1, "p")):
                if a.element_size() != size or int(a.shape[0]) < n:
                    raise ValueError(f"{name} must hold n elements of {size} bytes")
        if not on_device:
            t = np.ascontiguousarray(t, np.int64)
            x = np.ascontiguousarray(x, np.uint16)
            y = np.ascontiguousarray(y, np.uint16)
            p = np.ascontiguousarray(p, np.int8)
        _check(rec_push_events(self.ctx, t, x, y, p, n, 1 if on_device else 0), "rec_push_events")
        if on_device:
            self._pending.append((t, x, y, p))

    def solve(self, iters: int = 0, stats: bool = False) -> Optional[rec_stats]:
        rc, st = rec_solve(self.ctx, iters, stats)
        _check(rc, "rec_solve")
        self._pending.clear()
        return st

    def image(self, which: int = REC_U, device: bool = False):
        np_ = self.shape[0] * self.shape[1]
        n = 3 * np_ if which == REC_STATE_P else np_
        dt = _PLANE_DTYPE.get(which, np.float32)
        shape = (3,) + self.shape if which == REC_STATE_P else self.shape
        if device:
            tdt = {np.int32: self.torch.int32, np.int64: self.torch.int64}.get(dt, self.torch.float32)
            out = self.torch.empty(n, dtype=tdt, device=self.device)
            _check(rec_get_image(self.ctx, which, out, 1), "rec_get_image")
            self._pending.clear()
            return out.view(*shape)
        out = np.empty(n, dtype=dt)
        _check(rec_get_image(self.ctx, which, out, 0), "rec_get_image")
        self._pending.clear()
        return out.reshape(shape)

    def gap_history(self):
        out = rec_gap_history(self.ctx)
        self._pending.clear()
        return out

    def sync(self) -> None:
        _check(rec_sync(self.ctx), "rec_sync")
        self._pending.clear()

    def times(self) -> Tuple[int, int, bool]:
        """(first, latest accepted timestamp, whether any event was accepted)."""
        rc, tf, tr, st = rec_get_times(self.ctx)
        _check(rc, "rec_get_times")
        self._pending.clear()
        return tf, tr, bool(st)

    def state(self) -> dict:
        """A checkpoint of the stream: u, p, latest timestamps and t_ref
        (host arrays), for ``set_state`` of this or another context."""
        _, t_ref, started = self.times()
        return {"u": self.image(REC_U), "p": self.image(REC_STATE_P),
                "t_last": self.image(REC_T_LAST), "t_ref": t_ref if started else NO_EVENT}

    def set_state(self, u, p, t_last, t_ref: int) -> None:
        """Import a checkpoint (numpy arrays, or device tensors)."""
        on_device = not isinstance(u, np.ndarray)
        if not on_device:
            u = np.ascontiguousarray(u, np.float32)
            p = None if p is None else np.ascontiguousarray(p, np.float32)
            t_last = None if t_last is None else np.ascontiguousarray(t_last, np.int64)
        _check(rec_set_state(self.ctx, u, p, t_last, t_ref, 1 if on_device else 0),
               "rec_set_state")


def _ctx_array(ctxs):
    arr = (_vp * len(ctxs))(*ctxs)
    return arr


def rec_batch_workspace_bytes(ctxs) -> int:
    return load().rec_batch_workspace_bytes(_ctx_array(ctxs), len(ctxs))


def rec_batch_init(ctxs, workspace_ptr: int, workspace_bytes: int, tune_iters: int):
    h = _vp()
    rc = load().rec_batch_init(_ctx_array(ctxs), len(ctxs), workspace_ptr, int(workspace_bytes),
                               int(tune_iters), ctypes.byref(h))
    return rc, h.value


def rec_batch_solve(batch: int, iters: int) -> int:
    return load().rec_batch_solve(batch, int(iters))


def rec_batch_classes(batch: int) -> int:
    return load().rec_batch_classes(batch)


def rec_batch_config(batch: int, cls: int) -> dict:
    c = rec_batch_class()
    _check(load().rec_batch_config(batch, int(cls), ctypes.byref(c)), "rec_batch_config")
    return {f: getattr(c, f) for f, _ in rec_batch_class._fields_}


def rec_batch_set_geometry(batch: int, width: int, height: int, rows: int, waves: int,
                           cols: int, kiters: int) -> int:
    return load().rec_batch_set_geometry(batch, int(width), int(height), int(rows), int(waves),
                                         int(cols), int(kiters))


def rec_batch_set_mode(batch: int, mode: int) -> int:
    return load().rec_batch_set_mode(batch, int(mode))


def rec_batch_destroy(batch: Optional[int]) -> int:
    return load().rec_batch_destroy(batch)


class Batch:
    """Several Reconstructors solved together (one launch per block of
    iterations for all of them)."""

    def __init__(self, recs, tune_iters: int = 50):
        import torch

        self.recs = list(recs)
        ctxs = [r.ctx for r in self.recs]
        nbytes = rec_batch_workspace_bytes(ctxs)
        if nbytes == 0:
            raise RecError(REC_EINVAL, "rec_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.recs[0].device)
        rc, h = rec_batch_init(ctxs, self.workspace.data_ptr(), nbytes, tune_iters)
        _check(rc, "rec_batch_init")
        self.handle = h

    def solve(self, iters: int) -> None:
        _check(rec_batch_solve(self.handle, iters), "rec_batch_solve")
        for r in self.recs:
            r._pending.clear()

    def config(self):
        """Per class: sensor size, streams, tile geometry, K, tiles, tuned time."""
        return [rec_batch_config(self.handle, c) for c in range(rec_batch_classes(self.handle))]

    def set_mode(self, mode: int) -> None:
        _check(rec_batch_set_mode(self.handle, mode), "rec_batch_set_mode")

    def set_geometry(self, width: int, height: int, rows: int, waves: int, cols: int,
                     kiters: int) -> None:
        _check(rec_batch_set_geometry(self.handle, width, height, rows, waves, cols, kiters),
               "rec_batch_set_geometry")

    def close(self):
        if getattr(self, "handle", None):
            rec_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


DEFAULT_STEP = 1.0 / math.sqrt(8.0 + 4.0 * math.sqrt(2.0))


# ---------------------------------------------------------------------------
# Differentiable unrolled solve
# ---------------------------------------------------------------------------

def rec_diff_desc_make(width: int, height: int, batch: int, iters: int, ckpt_every: int = 10,
                       tau: float = DEFAULT_STEP, sigma: float = DEFAULT_STEP,
                       u_min: float = 1.0, u_max: float = math.e,
                       unfused: bool = False) -> rec_diff_desc:
    k = max(1, min(int(ckpt_every), max(int(iters), 1)))
    return rec_diff_desc(int(width), int(height), int(batch), int(iters), k, int(bool(unfused)),
                         float(tau), float(sigma), float(u_min), float(u_max))


def rec_diff_workspace_bytes(desc: rec_diff_desc) -> int:
    return load().rec_diff_workspace_bytes(ctypes.byref(desc))


def _diff_inputs(u0, p0, npos, nneg, tx, ty, w, theta) -> rec_diff_inputs:
    return rec_diff_inputs(*[_addr(a) for a in (u0, p0, npos, nneg, tx, ty, w, theta)])


def rec_diff_forward(desc: rec_diff_desc, inputs: rec_diff_inputs, u_out, p_out, workspace_ptr,
                     workspace_bytes: int, stream_ptr) -> int:
    return load().rec_diff_forward(ctypes.byref(desc), ctypes.byref(inputs), _addr(u_out),
                                   _addr(p_out), workspace_ptr, int(workspace_bytes), stream_ptr)


def rec_diff_forward_noalloc(desc: rec_diff_desc, inputs: rec_diff_inputs, u_out, p_out,
                             stream_ptr) -> int:
    return load().rec_diff_forward_noalloc(ctypes.byref(desc), ctypes.byref(inputs),
                                           _addr(u_out), _addr(p_out), stream_ptr)


def rec_diff_backward(desc: rec_diff_desc, inputs: rec_diff_inputs, g_u, g_p,
                      grads: rec_diff_grads, workspace_ptr, workspace_bytes: int,
                      stream_ptr) -> int:
    return load().rec_diff_backward(ctypes.byref(desc), ctypes.byref(inputs), _addr(g_u),
                                    _addr(g_p), ctypes.byref(grads), workspace_ptr,
                                    int(workspace_bytes), stream_ptr)


def _unrolled_function():
    import torch

    class UnrolledPD(torch.autograd.Function):
        """(u_K, p_K) of the unrolled loop; gradients by the library's reverse
        sweep with checkpoints (rec_diff_forward / rec_diff_backward)."""

        @staticmethod
        def _prep(u0, w, theta, p0, npos, nneg, tx, ty):
            """Contiguous device tensors of the library's types (the same
            values, so forward and backward see identical inputs)."""
            dev = u0.device
            if dev.type != "cuda":
                raise ValueError("the inputs must be device (HIP) tensors")
            f32 = lambda a: None if a is None else a.detach().to(dev, torch.float32).contiguous()
            i32 = lambda a: a.detach().to(dev, torch.int32).contiguous()
            return dict(u0=f32(u0), w=f32(w), p0=f32(p0), npos=i32(npos), nneg=i32(nneg),
                        tx=f32(tx), ty=f32(ty),
                        theta=theta.detach().to(dev, torch.float64).contiguous())

        @staticmethod
        def forward(ctx, u0, w, theta, p0, npos, nneg, tx, ty, desc):
            dev = u0.device
            B, H, W = desc.batch, desc.height, desc.width
            t = UnrolledPD._prep(u0, w, theta, p0, npos, nneg, tx, ty)
            if t["u0"].shape != (B, H, W) or (t["p0"] is not None and t["p0"].shape != (B, 3, H, W)):
                raise ValueError("u0 must be [B, H, W] and p0 [B, 3, H, W]")
            for k in ("w", "npos", "nneg", "tx", "ty"):
                if t[k] is not None and t[k].shape != (B, H, W):
                    raise ValueError(f"{k} must be [B, H, W]")
            if t["theta"].shape != (3,):
                raise ValueError("theta must hold (lambda, delta_pos, delta_neg)")
            nbytes = rec_diff_workspace_bytes(desc)
            if nbytes == 0:
                raise RecError(REC_EINVAL, "rec_diff_workspace_bytes")
            ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            u_out = torch.empty((B, H, W), dtype=torch.float32, device=dev)
            p_out = torch.empty((B, 3, H, W), dtype=torch.float32, device=dev)
            inputs = _diff_inputs(t["u0"], t["p0"], t["npos"], t["nneg"], t["tx"], t["ty"],
                                  t["w"], t["theta"])
            stream = torch.cuda.current_stream(dev).cuda_stream
            with torch.cuda.device(dev):
                _check(rec_diff_forward(desc, inputs, u_out, p_out, ws.data_ptr(), nbytes,
                                        stream), "rec_diff_forward")
            # the original inputs are saved so that autograd's version check
            # rejects an in-place change between forward and backward
            ctx.save_for_backward(u0, w, theta, p0, npos, nneg, tx, ty)
            ctx.desc, ctx.ws, ctx.nbytes = desc, ws, nbytes
            return u_out, p_out

        @staticmethod
        @torch.autograd.function.once_differentiable
        def backward(ctx, g_u, g_p):
            t, desc = UnrolledPD._prep(*ctx.saved_tensors), ctx.desc
            dev = t["u0"].device
            B, H, W = desc.batch, desc.height, desc.width
            need_u0, need_w, need_th, need_p0 = ctx.needs_input_grad[:4]
            g_u = None if g_u is None else g_u.to(torch.float32).contiguous()
            g_p = None if g_p is None else g_p.to(torch.float32).contiguous()
            gu0 = torch.empty((B, H, W), dtype=torch.float32, device=dev) if need_u0 else None
            gw = torch.empty((B, H, W), dtype=torch.float32, device=dev) if need_w else None
            gp0 = torch.empty((B, 3, H, W), dtype=torch.float32, device=dev) if need_p0 else None
            gth = torch.empty(3, dtype=torch.float64, device=dev) if need_th else None
            grads = rec_diff_grads(_addr(gu0), _addr(gp0), _addr(gw), _addr(gth))
            inputs = _diff_inputs(t["u0"], t["p0"], t["npos"], t["nneg"], t["tx"], t["ty"],
                                  t["w"], t["theta"])
            stream = torch.cuda.current_stream(dev).cuda_stream
            with torch.cuda.device(dev):
                _check(rec_diff_backward(desc, inputs, g_u, g_p, grads, ctx.ws.data_ptr(),
                                         ctx.nbytes, stream), "rec_diff_backward")
            return gu0, gw, gth, gp0, None, None, None, None, None

    return UnrolledPD


_UNROLLED = None


def unrolled(u0, npos, nneg, tx, ty, theta, iters: int, w=None, p0=None, ckpt_every: int = 10,
             tau: float = DEFAULT_STEP, sigma: float = DEFAULT_STEP, u_min: float = 1.0,
             u_max: float = math.e, unfused: bool = False):
    """K = iters primal-dual iterations on a batch of blocks, differentiable
    in u0, w, theta = (lambda, delta_pos, delta_neg) and p0.

    u0, npos, nneg, tx, ty, w: [B, H, W] (w None = all 1); p0: [B, 3, H, W]
    (None = 0); theta: float64 tensor of 3 on the device.  Returns
    (u_K [B, H, W], p_K [B, 3, H, W]) as float32 device tensors."""
    global _UNROLLED
    if _UNROLLED is None:
        _UNROLLED = _unrolled_function()
    if u0.dim() != 3:
        raise ValueError("u0 must be [B, H, W]")
    B, H, W = u0.shape
    desc = rec_diff_desc_make(W, H, B, iters, ckpt_every, tau, sigma, u_min, u_max, unfused)
    return _UNROLLED.apply(u0, w, theta, p0, npos, nneg, tx, ty, desc)
