"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test states the passage it follows.  None of them re-types the oracle's
formulas: they check definitions (the tangent basis of eqns. 1-4), adjoint
identities, closed forms, brute-force minimisation, an independently written
textbook TV-KL Chambolle-Pock, optimality of the converged image for the
energy of eqn. (5) evaluated independently, and the gap certificate.
"""
import math

import numpy as np
import pytest
from scipy import optimize

import oracle
from oracle import Oracle, Params

RNG = np.random.default_rng(20160721)
SHAPES = [(1, 1), (1, 7), (6, 1), (5, 8), (17, 23)]


def rand_surface(shape, scale, rng=RNG):
    H, W = shape
    tx = rng.normal(0, scale, shape)
    ty = rng.normal(0, scale, shape)
    tx[:, W - 1] = 0.0  # forward differences vanish on the last column / row
    ty[H - 1, :] = 0.0
    return tx, ty


def metric(tx, ty):
    """g = [[<phi_x, phi_x>, <phi_x, phi_y>], [.., <phi_y, phi_y>]] with
    phi_x = (1, 0, t_x), phi_y = (0, 1, t_y)  (eqns. 1-2)."""
    phx = np.stack([np.ones_like(tx), np.zeros_like(tx), tx], -1)
    phy = np.stack([np.zeros_like(ty), np.ones_like(ty), ty], -1)
    g = np.empty(tx.shape + (2, 2))
    g[..., 0, 0] = (phx * phx).sum(-1)
    g[..., 0, 1] = g[..., 1, 0] = (phx * phy).sum(-1)
    g[..., 1, 1] = (phy * phy).sum(-1)
    return g, phx, phy


def fwd_diff(v):
    """Forward differences, zero on the last column / row (numpy slicing)."""
    gx = np.zeros_like(v)
    gy = np.zeros_like(v)
    gx[:, :-1] = v[:, 1:] - v[:, :-1]
    gy[:-1, :] = v[1:, :] - v[:-1, :]
    return gx, gy


# --------------------------------------------------------------------------
# Operators
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", SHAPES)
def test_grad_div_adjoint(shape):
    """<grad u, p> = -<u, div p> (div defined as minus the adjoint, Chambolle 2004)."""
    u = RNG.normal(size=shape)
    qx, qy = RNG.normal(size=shape), RNG.normal(size=shape)
    gx, gy = oracle.grad(u)
    lhs = (gx * qx).sum() + (gy * qy).sum()
    rhs = -(u * oracle.div(qx, qy)).sum()
    assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))


@pytest.mark.parametrize("shape", SHAPES)
def test_grad_is_forward_difference(shape):
    """L_x, L_y: first-order forward differences (Section 3.1, Discrete Energy)."""
    u = RNG.normal(size=shape)
    gx, gy = oracle.grad(u)
    ex, ey = fwd_diff(u)
    assert np.array_equal(gx, ex) and np.array_equal(gy, ey)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("scale", [0.0, 0.3, 5.0, 150.0])
def test_Lg_adjoint(shape, scale):
    """<L_g u, p> = <u, L_g^* p> for random time surfaces (Section 3.2)."""
    tx, ty = rand_surface(shape, scale)
    u = RNG.normal(size=shape)
    p = RNG.normal(size=(3,) + shape)
    lhs = (oracle.apply_Lg(tx, ty, u) * p).sum()
    rhs = (u * oracle.apply_LgT(tx, ty, p)).sum()
    assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs) + np.abs(p).sum())


@pytest.mark.parametrize("scale", [0.0, 0.5, 3.0, 80.0])
def test_Lg_is_manifold_gradient(scale):
    """eqn. (4): grad_g f = (g^11 f_x + g^12 f_y) phi_x + (g^21 f_x + g^22 f_y) phi_y,
    with g^{ij} from a numerical inverse of the metric of eqn. (2)."""
    shape = (9, 11)
    tx, ty = rand_surface(shape, scale)
    u = RNG.normal(size=shape)
    ux, uy = fwd_diff(u)
    g, phx, phy = metric(tx, ty)
    gi = np.linalg.inv(g)
    A = gi[..., 0, 0] * ux + gi[..., 0, 1] * uy
    B = gi[..., 1, 0] * ux + gi[..., 1, 1] * uy
    expect = A[..., None] * phx + B[..., None] * phy
    got = np.moveaxis(oracle.apply_Lg(tx, ty, u), 0, -1)
    assert np.allclose(got, expect, rtol=1e-11, atol=1e-13)
    # |grad_g u|^2 in the ambient space equals grad u^T g^-1 grad u, and
    # G = det g = 1 + t_x^2 + t_y^2 (Section 3.1).
    n2 = (got ** 2).sum(-1)
    q = ux * (gi[..., 0, 0] * ux + gi[..., 0, 1] * uy) + uy * (gi[..., 1, 0] * ux + gi[..., 1, 1] * uy)
    assert np.allclose(n2, q, rtol=1e-10, atol=1e-14)
    # (det of the 2x2 cancels ~(t_x t_y)^2, hence the looser tolerance)
    assert np.allclose(np.linalg.det(g), 1 + tx ** 2 + ty ** 2, rtol=1e-8)


def test_flat_surface_gives_plain_gradient():
    """t = const: g is the identity and TV_g is the standard TV (Section 3.1)."""
    u = RNG.normal(size=(7, 9))
    z = np.zeros_like(u)
    a = oracle.apply_Lg(z, z, u)
    gx, gy = fwd_diff(u)
    assert np.array_equal(a[0], gx) and np.array_equal(a[1], gy) and not a[2].any()


@pytest.mark.parametrize("slope", [0.0, 0.7, 4.0, 30.0])
def test_ramp_surface_closed_form(slope):
    """Ramp t = a x (Fig. 2b): t_x = a, t_y = 0, so at interior pixels
    sqrt(G) |L_g u| = sqrt(u_x^2 + (1 + a^2) u_y^2): regularisation across the
    ramp is weaker than along it (the anisotropy of Fig. 2)."""
    H, W = 8, 10
    t = slope * np.tile(np.arange(W, dtype=float), (H, 1))
    tx, ty = fwd_diff(t)
    u = RNG.normal(size=(H, W))
    ux, uy = fwd_diff(u)
    a = oracle.apply_Lg(tx, ty, u)
    lhs = np.sqrt(1 + tx ** 2 + ty ** 2) * np.sqrt((a ** 2).sum(0))
    rhs = np.sqrt(ux ** 2 + (1 + slope ** 2) * uy ** 2)
    inner = (slice(0, H - 1), slice(0, W - 1))
    assert np.allclose(lhs[inner], rhs[inner], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("scale", [0.0, 1.0, 20.0])
def test_operator_norm_bound(scale):
    """||L_g||^2 <= 8 + 4 sqrt 2 (Section 3.2); power iteration on L_g^* L_g."""
    shape = (12, 13)
    tx, ty = rand_surface(shape, scale)
    v = RNG.normal(size=shape)
    lam = 0.0
    for _ in range(400):
        w = oracle.apply_LgT(tx, ty, oracle.apply_Lg(tx, ty, v))
        lam = np.linalg.norm(w)
        v = w / lam
    assert lam <= 8.0 + 1e-9
    assert lam <= 8.0 + 4.0 * math.sqrt(2.0)
    if scale == 0.0:
        assert lam > 7.0  # the flat case approaches the discrete Laplacian's bound 8


# --------------------------------------------------------------------------
# Proximal maps
# --------------------------------------------------------------------------

def _kl_objective(v, ubar, beta, f):
    return 0.5 * (v - ubar) ** 2 + beta * (v - f * math.log(v))


def test_prox_kl_brute_force():
    """prox_{tau D}: minimiser over [u_min, u_max] of (v - ubar)^2 / 2 +
    beta (v - f log v) (eqn. update_rules), found by bounded scalar search."""
    umin, umax = 1.0, math.e
    cases = [(RNG.uniform(-5, 8), RNG.uniform(1e-3, 200), RNG.uniform(0.05, 8)) for _ in range(300)]
    cases += [(1.5, 24.35, 1.5), (0.0, 124.0, 2.0), (10.0, 0.01, 1.2), (-3.0, 50.0, 0.3)]
    for ubar, beta, f in cases:
        got = oracle.prox_kl(ubar, beta, f, umin, umax)
        res = optimize.minimize_scalar(_kl_objective, bounds=(umin, umax), method="bounded",
                                       args=(ubar, beta, f), options={"xatol": 1e-12})
        # compare objective values (robust near flat minima) and the argmin
        assert _kl_objective(got, ubar, beta, f) <= res.fun + 1e-11 * (1 + abs(res.fun))
        assert abs(got - res.x) <= 1e-5


def test_prox_kl_special_cases():
    umin, umax = 0.5, 4.0
    for f in [0.7, 1.3, 3.9]:
        # f = ubar is a fixed point of the prox for any beta
        for beta in [1e-3, 1.0, 100.0]:
            assert abs(oracle.prox_kl(f, beta, f, umin, umax) - f) <= 1e-13 * f
    # beta -> 0: the prox is the projection onto [u_min, u_max]
    for ubar in [-1.0, 0.6, 2.0, 7.0]:
        assert abs(oracle.prox_kl(ubar, 1e-14, 1.0, umin, umax) - min(max(ubar, umin), umax)) <= 1e-12


def test_prox_kl_matches_quadratic_formula():
    """Where it does not cancel, the printed closed form 1/2 (a + sqrt(a^2 + 4 beta f))
    agrees with the oracle's cancellation-free form."""
    for _ in range(200):
        ubar, beta, f = RNG.uniform(0, 5), RNG.uniform(0, 2), RNG.uniform(0.5, 3)
        a = ubar - beta
        paper = 0.5 * (a + math.sqrt(a * a + 4 * beta * f))
        paper = min(max(paper, 1e-3), 1e3)
        assert abs(oracle.prox_kl(ubar, beta, f, 1e-3, 1e3) - paper) <= 1e-13 * paper


def test_projection():
    """prox_{sigma R^*}: p / max(1, |p| / sqrt(G)) (eqn. update_rules)."""
    for _ in range(200):
        s = RNG.uniform(0.5, 50)
        q = RNG.normal(size=3) * RNG.uniform(0.01, 3) * s
        r = oracle.project(q, s)
        n = np.linalg.norm(q)
        if n <= s:
            assert np.array_equal(r, q)
        else:
            assert abs(np.linalg.norm(r) - s) <= 1e-12 * s
            assert np.allclose(r / np.linalg.norm(r), q / n, atol=1e-14)
        assert np.linalg.norm(r) <= s * (1 + 1e-15)
        assert np.allclose(oracle.project(r, s), r, rtol=1e-15, atol=0)


# --------------------------------------------------------------------------
# Whole iteration
# --------------------------------------------------------------------------

def _oracle_on_data(f, tx, ty, u0, **kw):
    H, W = f.shape
    o = Oracle(Params(W, H, **kw), u0=u0)
    o.set_data(f=f, tx=tx, ty=ty)
    return o


@pytest.mark.parametrize("scale", [0.0, 2.0, 60.0])
def test_constant_image_is_fixed_point(scale):
    """f = u0 = c and p = 0 is a saddle point for any time surface."""
    shape = (9, 10)
    tx, ty = rand_surface(shape, scale)
    c = 1.9
    f = np.full(shape, c)
    o = _oracle_on_data(f, tx, ty, f)
    o.iterate(30)
    assert np.allclose(o.u, c, rtol=0, atol=1e-13)
    assert np.abs(o.p).max() <= 1e-13


def textbook_tv_kl(f, u0, lam, tau, sigma, umin, umax, iters):
    """Chambolle-Pock 2011 for min TV(u) + lam sum(u - f log u), u in [umin, umax],
    written independently with numpy slicing (2-component dual, unit ball).
    The primal prox solves v^2 - (ubar - tau lam) v - tau lam f = 0."""
    u = u0.copy()
    px = np.zeros_like(u)
    py = np.zeros_like(u)
    for _ in range(iters):
        d = np.zeros_like(u)
        d[:, :-1] += px[:, :-1]
        d[:, 1:] -= px[:, :-1]
        d[:-1, :] += py[:-1, :]
        d[1:, :] -= py[:-1, :]
        ubar = u + tau * d
        b = ubar - tau * lam
        un = np.clip(0.5 * (b + np.sqrt(b * b + 4 * tau * lam * f)), umin, umax)
        ut = 2 * un - u
        gx, gy = fwd_diff(ut)
        qx, qy = px + sigma * gx, py + sigma * gy
        m = np.maximum(1.0, np.sqrt(qx ** 2 + qy ** 2))
        px, py = qx / m, qy / m
        u = un
    return u, px, py


@pytest.mark.parametrize("lam", [0.5, 8.0, 90.0])
def test_flat_manifold_reduces_to_textbook_tv_kl(lam):
    """t = const: TV_g is the standard TV and sqrt(G) = 1 (Section 3.1), so
    the iterates equal textbook TV-KL primal-dual; the third dual component
    stays zero."""
    shape = (17, 23)
    f = np.exp(RNG.uniform(0, 1, shape))
    u0 = np.exp(RNG.uniform(0, 1, shape))
    z = np.zeros(shape)
    o = _oracle_on_data(f, z, z, u0, lam=lam)
    o.iterate(60)
    u, px, py = textbook_tv_kl(f, u0, lam, oracle.STEP, oracle.STEP, 1.0, math.e, 60)
    assert np.allclose(o.u, u, rtol=0, atol=1e-12)
    p = o.p
    assert np.allclose(p[0], px, atol=1e-12) and np.allclose(p[1], py, atol=1e-12)
    assert not p[2].any()


def energy_eq5(u, f, tx, ty, lam):
    """Discrete energy of eqn. (5), written from the manifold gradient of
    eqn. (4) (numerical metric inverse), not from the oracle's operators."""
    ux, uy = fwd_diff(u)
    g, phx, phy = metric(tx, ty)
    gi = np.linalg.inv(g)
    A = gi[..., 0, 0] * ux + gi[..., 0, 1] * uy
    B = gi[..., 1, 0] * ux + gi[..., 1, 1] * uy
    grad_g = A[..., None] * phx + B[..., None] * phy
    G = np.linalg.det(g)
    reg = np.sqrt(G * (grad_g ** 2).sum(-1)).sum()
    data = lam * ((u - f * np.log(u)) * np.sqrt(G)).sum()
    return reg + data


@pytest.mark.parametrize("scale", [0.0, 1.5, 12.0])
def test_converged_image_minimises_eq5(scale):
    """After many iterations the image is a minimiser of eqn. (5): no feasible
    perturbation lowers the independently evaluated energy, and the oracle's
    gap certifies it."""
    shape = (6, 7)
    rng = np.random.default_rng(7)
    tx, ty = rand_surface(shape, scale, rng)
    f = np.exp(rng.uniform(-0.2, 1.2, shape))
    lam = 1.5
    o = _oracle_on_data(f, tx, ty, np.full(shape, 1.6), lam=lam)
    o.iterate(60000)
    u = o.u
    e0 = energy_eq5(u, f, tx, ty, lam)
    g, e = o.gap_energy()
    assert abs(e - e0) <= 1e-10 * abs(e0)
    assert -1e-12 * e0 <= g <= 5e-6 * e0  # (>= 0 up to rounding at convergence)
    # the gap bounds the suboptimality: E(v) >= E* >= E(u) - gap for every feasible v
    for k in range(400):
        step = 10.0 ** rng.uniform(-6, -1)
        d = rng.normal(size=shape) * step
        v = np.clip(u + d, 1.0, math.e)
        assert energy_eq5(v, f, tx, ty, lam) >= e0 - g - 1e-10 * e0


def test_tiny_brute_force_minimum():
    """2x2 image: direct numerical minimisation of eqn. (5) over the box
    reaches the energy of the oracle's converged iterate."""
    shape = (2, 2)
    rng = np.random.default_rng(3)
    tx, ty = rand_surface(shape, 2.0, rng)
    f = np.array([[1.2, 2.5], [2.0, 1.05]])
    lam = 0.8
    o = _oracle_on_data(f, tx, ty, np.full(shape, 1.5), lam=lam)
    o.iterate(50000)
    e_or = energy_eq5(o.u, f, tx, ty, lam)
    best = np.inf
    for start in range(6):
        x0 = rng.uniform(1.0, math.e, 4)
        res = optimize.minimize(lambda v: energy_eq5(v.reshape(shape), f, tx, ty, lam), x0,
                                method="Powell", bounds=[(1.0, math.e)] * 4,
                                options={"xtol": 1e-12, "ftol": 1e-15, "maxfev": 200000})
        best = min(best, res.fun)
    assert e_or <= best + 1e-9 * abs(best)
    assert best <= e_or + 1e-6 * abs(e_or)


def test_large_lambda_gives_clamped_data():
    """lambda -> infinity: the data term dominates and u -> clamp(f)."""
    shape = (8, 9)
    tx, ty = rand_surface(shape, 3.0)
    f = np.exp(RNG.uniform(-0.3, 1.3, shape))
    o = _oracle_on_data(f, tx, ty, np.full(shape, 1.5), lam=1e8)
    o.iterate(5)
    assert np.allclose(o.u, np.clip(f, 1.0, math.e), rtol=0, atol=1e-6)


@pytest.mark.parametrize("scale", [0.0, 5.0])
def test_mirrored_time_surface_same_image(scale):
    """The metric sees only squares and products of (t_x, t_y) (eqn. 2), so
    t -> c - t (latest timestamp vs time since the last event) gives the same
    images; only the third dual component changes sign."""
    shape = (10, 12)
    tx, ty = rand_surface(shape, scale)
    f = np.exp(RNG.uniform(0, 1, shape))
    a = _oracle_on_data(f, tx, ty, np.full(shape, 1.4))
    b = _oracle_on_data(f, -tx, -ty, np.full(shape, 1.4))
    a.iterate(40)
    b.iterate(40)
    assert np.allclose(a.u, b.u, rtol=0, atol=1e-13)
    pa, pb = a.p, b.p
    assert np.allclose(pa[:2], pb[:2], atol=1e-13) and np.allclose(pa[2], -pb[2], atol=1e-13)
