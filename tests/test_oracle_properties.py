"""Property tests of the oracle's operators (CPU, FP64, hypothesis).

Randomised counterparts of the fixed pins: for arbitrary frame shapes, time
surfaces and fields, the manifold operator and its adjoint satisfy the
adjoint identity (Section 3.2, L_g^* as the adjoint of L_g); the KL prox
returns the point that satisfies the optimality conditions of the clamped
problem (eqn. update_rules); the dual projection lands in the ball of
radius sqrt(G), keeps the direction and is idempotent.
"""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle

# fixed example sequence: the same cases on every run
SETTINGS = settings(max_examples=150, deadline=None, derandomize=True, database=None)


@SETTINGS
@given(H=st.integers(1, 12), W=st.integers(1, 12), seed=st.integers(0, 2**32 - 1),
       scale=st.floats(0.0, 200.0))
def test_Lg_adjoint_identity(H, W, seed, scale):
    rng = np.random.default_rng(seed)
    tau = rng.normal(size=(H, W)) * scale
    tx = np.zeros((H, W))
    ty = np.zeros((H, W))
    tx[:, :-1] = tau[:, 1:] - tau[:, :-1]
    ty[:-1, :] = tau[1:, :] - tau[:-1, :]
    u = rng.normal(size=(H, W))
    p = rng.normal(size=(3, H, W))
    lhs = float((oracle.apply_Lg(tx, ty, u) * p).sum())
    rhs = float((u * oracle.apply_LgT(tx, ty, p)).sum())
    # Both sides add up the same products |M| |grad u| |p| in another order;
    # every entry of M is at most 1 in magnitude, which bounds the terms.
    gx = np.zeros((H, W))
    gy = np.zeros((H, W))
    gx[:, :-1] = np.abs(np.diff(u, axis=1))
    gy[:-1, :] = np.abs(np.diff(u, axis=0))
    scale = float(((gx + gy) * np.abs(p).sum(axis=0)).sum())
    assert abs(lhs - rhs) <= 1e-12 * (1.0 + scale)


@SETTINGS
@given(ubar=st.floats(-50.0, 50.0), beta=st.floats(1e-3, 300.0), f=st.floats(1e-3, 10.0),
       lo=st.floats(1e-3, 5.0), width=st.floats(1e-3, 10.0))
def test_prox_kl_satisfies_the_clamped_optimality_conditions(ubar, beta, f, lo, width):
    umin, umax = lo, lo + width
    v = oracle.prox_kl(ubar, beta, f, umin, umax)
    assert umin <= v <= umax
    # derivative of (v - ubar)^2 / 2 + beta (v - f log v)
    g = v - ubar + beta * (1.0 - f / v)
    tol = 1e-9 * (1.0 + abs(ubar) + beta + beta * f / v)
    if umin < v < umax:
        assert abs(g) <= tol
    elif v == umin and v < umax:
        assert g >= -tol  # the objective does not decrease into the box from umin
    else:
        assert g <= tol   # ... nor from umax


@SETTINGS
@given(q=st.lists(st.floats(-1e3, 1e3), min_size=3, max_size=3),
       s=st.floats(1.0, 100.0))
def test_projection_is_radial_and_idempotent(q, s):
    q = np.array(q)
    r = oracle.project(q, s)
    n = float(np.linalg.norm(q))
    assert np.linalg.norm(r) <= s * (1 + 1e-14)
    if n <= s:
        assert np.array_equal(r, q)
    else:
        # same direction, on the sphere
        assert np.allclose(r, q * (s / n), rtol=1e-13, atol=1e-300)
        assert math.isclose(np.linalg.norm(r), s, rel_tol=1e-13)
    assert np.allclose(oracle.project(r, s), r, rtol=1e-14, atol=0)
