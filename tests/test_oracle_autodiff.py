"""Pins of the FP64 autograd reference of the unrolled loop (CPU).

Its forward is pinned to the C oracle (separate code, same iteration of
Section 3.2 with per-pixel data weights); its gradients are pinned to
central finite differences of the C oracle, so a wrong sign, index or
dropped term in either the forward or the derivative chain fails here."""
import math

import numpy as np
import pytest
import torch

import evgen
import oracle
from oracle import autodiff

LAM, DPOS, DNEG = 90.0, 0.2, 0.25


def oracle_forward(inp, lam, dpos, dneg, iters, p0=None, w=None, u0=None):
    """u_K, p_K of every image by the C oracle (f formed here in FP64)."""
    u0 = inp["u0"] if u0 is None else u0
    B, H, W = u0.shape
    us, ps = [], []
    for b in range(B):
        o = oracle.Oracle(oracle.Params(W, H, lam=lam, delta_pos=dpos, delta_neg=dneg))
        u = u0[b].astype(np.float64)
        f = u * np.exp(dpos * inp["npos"][b] - dneg * inp["nneg"][b])
        o.set_state(u, None if p0 is None else p0[b].astype(np.float64))
        o.set_data(f, inp["tx"][b].astype(np.float64), inp["ty"][b].astype(np.float64))
        if w is not None:
            o.set_weights(w[b].astype(np.float64))
        o.iterate(iters)
        us.append(o.u)
        ps.append(o.p)
        o.close()
    return np.stack(us), np.stack(ps)


def ref_forward(inp, lam, dpos, dneg, iters, p0=None, w=None):
    t = lambda a: torch.from_numpy(np.asarray(a))
    return autodiff.unrolled(t(inp["u0"]), t(inp["npos"]), t(inp["nneg"]), t(inp["tx"]),
                             t(inp["ty"]), None if w is None else t(w), lam, dpos, dneg, iters,
                             p0=None if p0 is None else t(p0))


@pytest.fixture(scope="module")
def small():
    return evgen.diff_inputs(11, 2, 12, 10)


def test_forward_matches_c_oracle(small):
    rng = np.random.default_rng(3)
    p0 = 0.05 * rng.standard_normal((2, 3, 12, 10))
    u, p = ref_forward(small, LAM, DPOS, DNEG, 25, p0=p0, w=small["w"])
    uo, po = oracle_forward(small, LAM, DPOS, DNEG, 25, p0=p0, w=small["w"])
    np.testing.assert_allclose(u.numpy(), uo, rtol=0, atol=1e-12)
    np.testing.assert_allclose(p.numpy(), po, rtol=0, atol=1e-12)


def test_weights_one_is_the_paper_model(small):
    u1, _ = ref_forward(small, LAM, DPOS, DNEG, 10, w=np.ones_like(small["w"]))
    u2, _ = ref_forward(small, LAM, DPOS, DNEG, 10)
    assert torch.equal(u1, u2)
    # lambda w is what enters: doubling w equals doubling lambda
    u3, _ = ref_forward(small, 2 * LAM, DPOS, DNEG, 10)
    u4, _ = ref_forward(small, LAM, DPOS, DNEG, 10, w=2 * np.ones_like(small["w"]))
    np.testing.assert_allclose(u3.numpy(), u4.numpy(), rtol=0, atol=1e-13)


def _loss_weights(shape, seed=5):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape), rng.standard_normal(shape[:1] + (3,) + shape[1:])


def _oracle_loss(inp, gu, gp, lam, dpos, dneg, iters, p0, w, u0=None):
    u, p = oracle_forward(inp, lam, dpos, dneg, iters, p0=p0, w=w, u0=u0)
    return float((gu * u).sum() + (gp * p).sum())


def test_gradients_match_finite_differences(small):
    """d/d(lambda, dpos, dneg) and directional derivatives along w, u0, p0 of
    J = <gu, u_K> + <gp, p_K> against central differences of the C oracle."""
    iters = 20
    rng = np.random.default_rng(7)
    B, H, W = small["u0"].shape
    p0 = 0.05 * rng.standard_normal((B, 3, H, W))
    gu, gp = _loss_weights((B, H, W))
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    u0 = t(small["u0"]).requires_grad_()
    w = t(small["w"]).requires_grad_()
    p0t = t(p0).requires_grad_()
    th = torch.tensor([LAM, DPOS, DNEG], dtype=torch.float64, requires_grad=True)
    u, p = autodiff.unrolled(u0, t(small["npos"]), t(small["nneg"]), t(small["tx"]),
                             t(small["ty"]), w, th[0], th[1], th[2], iters, p0=p0t)
    J = (t(gu) * u).sum() + (t(gp) * p).sum()
    J.backward()

    def J_at(lam=LAM, dpos=DPOS, dneg=DNEG, w_=None, u0_=None, p0_=None):
        return _oracle_loss(small, gu, gp, lam, dpos, dneg, iters,
                            p0 if p0_ is None else p0_, small["w"] if w_ is None else w_,
                            u0=u0_)

    for k, (name, val) in enumerate([("lam", LAM), ("dpos", DPOS), ("dneg", DNEG)]):
        h = 1e-6 * max(abs(val), 1.0)
        fd = (J_at(**{name: val + h}) - J_at(**{name: val - h})) / (2 * h)
        assert abs(th.grad[k].item() - fd) <= 1e-6 * max(abs(fd), 1e-3), (name, th.grad[k], fd)

    base_w = small["w"].astype(np.float64)
    base_u = small["u0"].astype(np.float64)
    for what, grad, base in (("w", w.grad, base_w), ("u0", u0.grad, base_u),
                             ("p0", p0t.grad, p0)):
        v = rng.standard_normal(base.shape)
        h = 1e-6
        if what == "w":
            jp, jm = J_at(w_=base + h * v), J_at(w_=base - h * v)
        elif what == "u0":
            jp, jm = J_at(u0_=base + h * v), J_at(u0_=base - h * v)
        else:
            jp, jm = J_at(p0_=base + h * v), J_at(p0_=base - h * v)
        fd = (jp - jm) / (2 * h)
        an = float((grad.numpy() * v).sum())
        assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-3), (what, an, fd)


def test_zero_iterations_is_identity(small):
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    u0 = t(small["u0"]).requires_grad_()
    u, p = autodiff.unrolled(u0, t(small["npos"]), t(small["nneg"]), t(small["tx"]),
                             t(small["ty"]), None, LAM, DPOS, DNEG, 0)
    assert torch.equal(u, u0) and not p.any()


def test_no_nan_gradients_at_branch_edges():
    """Clamped pixels, zero dual fields and a flat manifold: the untaken
    branches must not leak NaN into the gradient."""
    H, W = 6, 5
    u0 = torch.full((1, H, W), math.e, dtype=torch.float64, requires_grad=True)
    z = torch.zeros((1, H, W), dtype=torch.float64)
    npos = torch.full((1, H, W), 3, dtype=torch.int32)
    u, p = autodiff.unrolled(u0, npos, torch.zeros_like(npos), z, z, None, LAM, DPOS, DNEG, 5)
    u.sum().backward()
    assert torch.isfinite(u0.grad).all()
    assert (u == math.e).all()           # f > e everywhere: clamped at the top
    assert not u0.grad.any()             # and so no dependence on u0
