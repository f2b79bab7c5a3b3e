"""The KL prox as the kernels evaluate it: half scale, no cancellation (CPU).

The primal step's prox (Section 3.2, update rules) is the positive root of
u^2 - a u - beta f = 0 with a = ubar - beta.  The kernels form h = a / 2,
r / 2 = sqrt(h^2 + beta f) and take r / 2 + |h| when h >= 0, else
beta f / (r / 2 + |h|).  These checks restate that form in numpy and pin it
to things other than itself: the root of the quadratic, a direct numerical
minimisation of the prox objective, and the FP32 error of the form against
the FP64 root over the whole range of a, including the branch where the
printed form (a + r) / 2 loses every digit to cancellation.
"""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar


def half_scale_root(ubar, beta, f, dtype=np.float64):
    """The kernels' evaluation order; in FP32, each step rounded once (a fused
    multiply-add is emulated by forming it in FP64 and rounding once)."""
    t = dtype
    ubar, beta, f = t(ubar), t(beta), t(f)
    hb = t(0.5) * beta
    bf = t(np.float64(beta) * np.float64(f))
    # h = fma(0.5, u, fma(0.5 ts, div, -hb)); here ubar = u + ts div is given,
    # so the inner term is taken as 0.5 (ubar - u) with u = ubar: h = 0.5 ubar - hb
    h = t(0.5 * np.float64(ubar) - np.float64(hb))
    rh = t(np.sqrt(t(np.float64(h) * np.float64(h) + np.float64(bf))))
    dh = t(rh + abs(h))
    if h >= 0:
        return dh
    return t(bf * (t(1.0) / dh))


def prox_objective(u, ubar, beta, f):
    # (u - ubar)^2 / 2 + beta (u - f log u): the primal step's prox for the KL term
    return 0.5 * (u - ubar) ** 2 + beta * (u - f * np.log(u))


CASES = [(3.0, 24.0, 1.5), (30.0, 24.0, 1.5), (-50.0, 24.0, 2.7), (24.0, 24.0, 1.0),
         (1e3, 0.5, 1.0), (-1e3, 60.0, 1e-3), (0.1, 1e-4, 2.0), (2.0, 80.0, 2.718)]


@pytest.mark.parametrize("ubar,beta,f", CASES)
def test_half_scale_root_solves_the_quadratic(ubar, beta, f):
    u = half_scale_root(ubar, beta, f)
    a = ubar - beta
    assert u > 0
    # residual of u^2 - a u - beta f = 0, relative to the size of its terms
    res = u * u - a * u - beta * f
    assert abs(res) <= 1e-12 * (u * u + abs(a * u) + beta * f)


@pytest.mark.parametrize("ubar,beta,f", CASES)
def test_half_scale_root_minimises_the_prox_objective(ubar, beta, f):
    u = half_scale_root(ubar, beta, f)
    lo, hi = u * 1e-3, u * 1e3 + 1.0
    best = minimize_scalar(prox_objective, bounds=(lo, hi), args=(ubar, beta, f),
                           method="bounded", options={"xatol": 1e-12 * u})
    assert best.fun >= prox_objective(u, ubar, beta, f) - 1e-12 * abs(best.fun)
    assert abs(best.x - u) <= 1e-5 * u


def test_fp32_half_scale_form_keeps_full_precision_where_the_printed_form_cancels():
    rng = np.random.default_rng(3)
    worst_half = 0.0
    worst_naive = 0.0
    for _ in range(4000):
        beta = float(np.float32(10 ** rng.uniform(-3, 2)))
        f = float(np.float32(10 ** rng.uniform(-3, 0.5)))
        ubar = float(np.float32(rng.choice([-1, 1]) * 10 ** rng.uniform(-3, 4)))
        a = ubar - beta
        ref = (a + np.sqrt(a * a + 4 * beta * f)) / 2 if a >= 0 else \
            2 * beta * f / (np.sqrt(a * a + 4 * beta * f) - a)
        got = float(half_scale_root(ubar, beta, f, np.float32))
        worst_half = max(worst_half, abs(got - ref) / ref)
        # the printed form in FP32
        a32 = np.float32(np.float32(ubar) - np.float32(beta))
        r32 = np.sqrt(np.float32(a32 * a32 + np.float32(4) * np.float32(beta) * np.float32(f)))
        naive = float(np.float32(0.5) * (a32 + r32))
        worst_naive = max(worst_naive, abs(naive - ref) / ref)
    eps = float(np.finfo(np.float32).eps)
    # a few roundings of the inputs' own FP32 representation and of the steps
    assert worst_half < 8 * eps
    # the printed form loses all digits for a << 0 (the kernels never use it)
    assert worst_naive > 0.5
