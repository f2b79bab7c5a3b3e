"""FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``oracle.c`` (plain C loops in
double precision, built with gcc -O2 without fast-math) through ctypes and
shares no code with the GPU library.  See ``oracle.c`` for the method steps
and the readings of points the paper leaves open.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_LIB_MT_PATH = os.path.join(_HERE, "liboracle_mt.so")  # same source, OpenMP over pixels

OK, EINVAL, ERANGE, EORDER = 0, -1, -2, -3
U, F, TAU, TX, TY, P1, P2, P3, TAU32, TX32, TY32, NPOS, NNEG, TLAST = range(14)

# tau = sigma = (8 + 4 sqrt 2)^(-1/2): tau * sigma * ||L_g||^2 <= 1 with the
# paper's bound ||L_g||^2 <= 8 + 4 sqrt 2 (Section 3.2).
STEP = 1.0 / math.sqrt(8.0 + 4.0 * math.sqrt(2.0))


class _P(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32),
        ("lam", ctypes.c_double),
        ("delta_pos", ctypes.c_double), ("delta_neg", ctypes.c_double),
        ("u_min", ctypes.c_double), ("u_max", ctypes.c_double),
        ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
        ("time_unit_us", ctypes.c_double),
        ("u_init", ctypes.c_double),
        ("tvl1_iters", ctypes.c_int32),
        ("tvl1_lambda", ctypes.c_double),
        ("slope_cap", ctypes.c_double),
    ]


@dataclasses.dataclass
class Params:
    width: int
    height: int
    lam: float = 90.0
    delta_pos: float = 0.2
    delta_neg: float = 0.2
    u_min: float = 1.0
    u_max: float = math.e
    tau: float = STEP
    sigma: float = STEP
    time_unit_us: float = 1000.0
    u_init: float = math.exp(0.5)
    tvl1_iters: int = 0
    tvl1_lambda: float = 1.0
    # > 0: time differences clipped to [-slope_cap, slope_cap] (the reading
    # of 16-bit storage, whose largest FP16 value is 65504); 0: none
    slope_cap: float = 0.0

    def _c(self) -> _P:
        return _P(self.width, self.height, self.lam, self.delta_pos, self.delta_neg,
                  self.u_min, self.u_max, self.tau, self.sigma, self.time_unit_us, self.u_init,
                  self.tvl1_iters, self.tvl1_lambda, self.slope_cap)


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` (gcc -O2, IEEE double, no contraction) and
    the OpenMP build of the same file, ``liboracle_mt.so``."""
    for path, extra in ((_LIB_PATH, ["-Wno-unknown-pragmas"]), (_LIB_MT_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call([
                "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                "-ffp-contract=off", "-Wall", *extra, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIB_PATH


_lib = None
_lib_mt = None
_vp = ctypes.c_void_p


def _load(threads: bool = False):
    """The single-threaded library, or with threads=True the OpenMP build
    (its thread count follows OMP_NUM_THREADS)."""
    global _lib, _lib_mt
    if threads:
        if _lib_mt is None:
            if not os.path.exists(_LIB_MT_PATH):
                build(force=False)
            _lib_mt = _declare(ctypes.CDLL(_LIB_MT_PATH))
        return _lib_mt
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = _declare(ctypes.CDLL(_LIB_PATH))
    return _lib


def _declare(lib):
    """Argument and result types of the exported functions."""
    lib.orc_create.restype = _vp
    lib.orc_create.argtypes = [ctypes.POINTER(_P), _vp]
    lib.orc_free.restype = None
    lib.orc_free.argtypes = [_vp]
    lib.orc_check_params.restype = ctypes.c_int
    lib.orc_check_params.argtypes = [ctypes.POINTER(_P)]
    lib.orc_push.restype = ctypes.c_int
    lib.orc_push.argtypes = [_vp] * 5 + [ctypes.c_int64]
    lib.orc_build.restype = None
    lib.orc_build.argtypes = [_vp]
    lib.orc_iterate.restype = None
    lib.orc_iterate.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp]
    lib.orc_solve.restype = None
    lib.orc_solve.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp]
    lib.orc_gap_energy.restype = None
    lib.orc_gap_energy.argtypes = [_vp, _vp, _vp]
    lib.orc_get.restype = ctypes.c_int
    lib.orc_get.argtypes = [_vp, ctypes.c_int, _vp]
    lib.orc_t_ref.restype = ctypes.c_int64
    lib.orc_t_ref.argtypes = [_vp]
    lib.orc_set_state.restype = ctypes.c_int
    lib.orc_set_state.argtypes = [_vp] * 5
    lib.orc_set_data.restype = ctypes.c_int
    lib.orc_set_data.argtypes = [_vp] * 4
    lib.orc_grad.restype = None
    lib.orc_grad.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
    lib.orc_div.restype = None
    lib.orc_div.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
    lib.orc_apply_Lg.restype = None
    lib.orc_apply_Lg.argtypes = [ctypes.c_int, ctypes.c_int] + [_vp] * 6
    lib.orc_apply_LgT.restype = None
    lib.orc_apply_LgT.argtypes = [ctypes.c_int, ctypes.c_int] + [_vp] * 6
    lib.orc_prox_kl.restype = ctypes.c_double
    lib.orc_prox_kl.argtypes = [ctypes.c_double] * 5
    lib.orc_project.restype = None
    lib.orc_project.argtypes = [_vp, _vp, _vp, ctypes.c_double]
    lib.orc_set_weights.restype = ctypes.c_int
    lib.orc_set_weights.argtypes = [_vp, _vp]
    lib.orc_tvl1.restype = None
    lib.orc_tvl1.argtypes = [ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_double, _vp]
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


# ---------------------------------------------------------------------------
# Operators (pure functions)
# ---------------------------------------------------------------------------

def grad(v):
    v = _f64(v)
    H, W = v.shape
    gx, gy = np.empty_like(v), np.empty_like(v)
    _load().orc_grad(W, H, _ptr(v), _ptr(gx), _ptr(gy))
    return gx, gy


def div(qx, qy):
    qx, qy = _f64(qx), _f64(qy)
    H, W = qx.shape
    out = np.empty_like(qx)
    _load().orc_div(W, H, _ptr(qx), _ptr(qy), _ptr(out))
    return out


def apply_Lg(tx, ty, u):
    tx, ty, u = _f64(tx), _f64(ty), _f64(u)
    H, W = u.shape
    a = np.empty((3, H, W))
    _load().orc_apply_Lg(W, H, _ptr(tx), _ptr(ty), _ptr(u), a[0].ctypes.data,
                         a[1].ctypes.data, a[2].ctypes.data)
    return a


def apply_LgT(tx, ty, p):
    tx, ty, p = _f64(tx), _f64(ty), _f64(p)
    H, W = tx.shape
    out = np.empty((H, W))
    _load().orc_apply_LgT(W, H, _ptr(tx), _ptr(ty), p[0].ctypes.data, p[1].ctypes.data,
                          p[2].ctypes.data, _ptr(out))
    return out


def prox_kl(ubar, beta, f, umin, umax) -> float:
    return _load().orc_prox_kl(float(ubar), float(beta), float(f), float(umin), float(umax))


def project(q, s):
    a = [ctypes.c_double(float(v)) for v in q]
    _load().orc_project(ctypes.byref(a[0]), ctypes.byref(a[1]), ctypes.byref(a[2]), float(s))
    return np.array([a[0].value, a[1].value, a[2].value])


def tvl1(f, iters: int, lam: float):
    """TV-L1 denoising of an image by Chambolle-Pock (the timestamp step of Section 4)."""
    f = _f64(f)
    H, W = f.shape
    out = np.empty_like(f)
    _load().orc_tvl1(W, H, _ptr(f), int(iters), float(lam), _ptr(out))
    return out


def check_params(p: Params) -> int:
    c = p._c()
    return _load().orc_check_params(ctypes.byref(c))


# ---------------------------------------------------------------------------
# Stateful reconstruction
# ---------------------------------------------------------------------------

class Oracle:
    """One event stream reconstructed in FP64 (mirrors the library's calls)."""

    def __init__(self, params: Params, u0: Optional[np.ndarray] = None, threads: bool = False):
        self.params = params
        self._lib = _load(threads)
        c = params._c()
        u0a = None if u0 is None else _f64(u0).reshape(params.height, params.width)
        self._h = self._lib.orc_create(ctypes.byref(c), _ptr(u0a))
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        self.shape = (params.height, params.width)

    def close(self):
        if self._h:
            self._lib.orc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, t, x, y, p) -> int:
        t = np.ascontiguousarray(t, np.int64)
        x = np.ascontiguousarray(x, np.uint16)
        y = np.ascontiguousarray(y, np.uint16)
        p = np.ascontiguousarray(p, np.int8)
        n = t.shape[0]
        if not (x.shape[0] == y.shape[0] == p.shape[0] == n):
            raise ValueError("event arrays differ in length")
        return self._lib.orc_push(self._h, _ptr(t), _ptr(x), _ptr(y), _ptr(p), n)

    def push_events(self, ev) -> int:
        return self.push(ev.t, ev.x, ev.y, ev.p)

    def build(self):
        self._lib.orc_build(self._h)

    def iterate(self, iters: int, gap_every: int = 0):
        m = iters // gap_every if gap_every > 0 else 0
        g = np.zeros(max(m, 1))
        e = np.zeros(max(m, 1))
        self._lib.orc_iterate(self._h, iters, gap_every, _ptr(g), _ptr(e))
        return g[:m], e[:m]

    def solve(self, iters: int, gap_every: int = 0):
        self.build()
        return self.iterate(iters, gap_every)

    def gap_energy(self):
        g, e = ctypes.c_double(), ctypes.c_double()
        self._lib.orc_gap_energy(self._h, ctypes.byref(g), ctypes.byref(e))
        return g.value, e.value

    def get(self, which: int) -> np.ndarray:
        dt = {TAU32: np.float32, TX32: np.float32, TY32: np.float32,
              NPOS: np.int32, NNEG: np.int32, TLAST: np.int64}.get(which, np.float64)
        out = np.empty(self.shape, dtype=dt)
        if self._lib.orc_get(self._h, which, _ptr(out)) != 0:
            raise ValueError("bad plane id")
        return out

    @property
    def u(self):
        return self.get(U)

    @property
    def p(self):
        return np.stack([self.get(P1), self.get(P2), self.get(P3)])

    @property
    def t_ref(self) -> int:
        return self._lib.orc_t_ref(self._h)

    def set_state(self, u=None, p=None):
        u = None if u is None else _f64(u)
        ps = [None, None, None] if p is None else [_f64(p[i]) for i in range(3)]
        self._lib.orc_set_state(self._h, _ptr(u), *[_ptr(a) for a in ps])

    def set_weights(self, w=None):
        w = None if w is None else _f64(w)
        self._lib.orc_set_weights(self._h, _ptr(w))

    def set_data(self, f=None, tx=None, ty=None):
        f = None if f is None else _f64(f)
        tx = None if tx is None else _f64(tx)
        ty = None if ty is None else _f64(ty)
        self._lib.orc_set_data(self._h, _ptr(f), _ptr(tx), _ptr(ty))
