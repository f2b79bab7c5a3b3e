"""FP64 PyTorch reference of the unrolled primal-dual loop, differentiated
by autograd.

TEST INFRASTRUCTURE ONLY (like the rest of this package): the tests and
the CPU baseline of the benchmark use it; the GPU library never does.

The function below unrolls K Chambolle-Pock iterations (Section 3.2,
eqn. cont_iterates) of the reconstruction on the event manifold for a batch
of images with a fixed block of data:

    f      = u0 * exp(dpos * n+ - dneg * n-)           (eqn. intensity_update)
    ubar   = u - tau L_g^* p
    u+     = clamp(prox_{tau D}(ubar), u_min, u_max)    (KL prox, Section 3.2)
    p+     = proj_{|.| <= s}(p + sigma L_g (2 u+ - u))
    L_g u  = M (D_x u, D_y u),  M = (1/G) [[1+ty^2, -tx ty], [-tx ty, 1+tx^2], [tx, ty]]
    s      = sqrt(G), G = 1 + tx^2 + ty^2                (eqn. (3), Section 3.1)

with the data term lambda * w * (u - f log u) * sqrt(G) per pixel.  The
per-pixel weights w are not in the paper (w = 1 is its model); they are the
weights a learned reconstruction would train.  Autograd supplies the
derivatives with respect to u0, p0, w, lambda, dpos and dneg; the code is
written so that no branch that is not taken produces a non-finite value
(autograd multiplies such values by zero and would get NaN).

The operators are written here from the definitions, independently of the C
oracle; the tests pin this forward to the C oracle and its gradients to
central finite differences of the C oracle.
"""
from __future__ import annotations

import math
from typing import Optional, Tuple

import torch

STEP = 1.0 / math.sqrt(8.0 + 4.0 * math.sqrt(2.0))


def _dx(u: torch.Tensor) -> torch.Tensor:
    """Forward difference along x, zero on the last column."""
    z = torch.zeros_like(u[..., :1])
    return torch.cat([u[..., 1:] - u[..., :-1], z], dim=-1)


def _dy(u: torch.Tensor) -> torch.Tensor:
    """Forward difference along y, zero on the last row."""
    z = torch.zeros_like(u[..., :1, :])
    return torch.cat([u[..., 1:, :] - u[..., :-1, :], z], dim=-2)


def _dxT(q: torch.Tensor) -> torch.Tensor:
    """Adjoint of _dx: (D_x^T q)[j] = q[j-1] - q[j], with q taken as zero on
    the last column (where D_x vanishes) and before the first."""
    q = torch.cat([q[..., :-1], torch.zeros_like(q[..., :1])], dim=-1)
    prev = torch.cat([torch.zeros_like(q[..., :1]), q[..., :-1]], dim=-1)
    return prev - q


def _dyT(q: torch.Tensor) -> torch.Tensor:
    q = torch.cat([q[..., :-1, :], torch.zeros_like(q[..., :1, :])], dim=-2)
    prev = torch.cat([torch.zeros_like(q[..., :1, :]), q[..., :-1, :]], dim=-2)
    return prev - q


def metric(tx: torch.Tensor, ty: torch.Tensor):
    """Entries of M and the ball radius s = sqrt(G) per pixel."""
    G = 1.0 + tx * tx + ty * ty
    m11 = (1.0 + ty * ty) / G
    m12 = -(tx * ty) / G
    m22 = (1.0 + tx * tx) / G
    m31 = tx / G
    m32 = ty / G
    return (m11, m12, m22, m31, m32), torch.sqrt(G)


def apply_Lg(m, u: torch.Tensor) -> torch.Tensor:
    m11, m12, m22, m31, m32 = m
    gx, gy = _dx(u), _dy(u)
    return torch.stack([m11 * gx + m12 * gy, m12 * gx + m22 * gy, m31 * gx + m32 * gy], dim=-3)


def apply_LgT(m, p: torch.Tensor) -> torch.Tensor:
    m11, m12, m22, m31, m32 = m
    p1, p2, p3 = p.unbind(dim=-3)
    qx = m11 * p1 + m12 * p2 + m31 * p3
    qy = m12 * p1 + m22 * p2 + m32 * p3
    return _dxT(qx) + _dyT(qy)


def prox_kl(ubar, beta, f, u_min, u_max):
    """argmin_u (u - ubar)^2 / 2 + beta (u - f log u), clamped: the positive
    root of u^2 - (ubar - beta) u - beta f = 0 in its two cancellation-free
    forms (a = ubar - beta, r = sqrt(a^2 + 4 beta f)):
    a >= 0: (a + r) / 2;  a < 0: 2 beta f / (r - a)."""
    a = ubar - beta
    c = 4.0 * beta * f
    pos = a >= 0
    ap = torch.where(pos, a, torch.zeros_like(a))
    an = torch.where(pos, torch.zeros_like(a), a)
    up = 0.5 * (ap + torch.sqrt(ap * ap + c))
    un = 0.5 * c / (torch.sqrt(an * an + c) - an)
    return torch.clamp(torch.where(pos, up, un), u_min, u_max)


def project(p: torch.Tensor, s: torch.Tensor) -> torch.Tensor:
    """Projection onto the ball |p| <= s (per pixel, over the 3 components)."""
    n2 = (p * p).sum(dim=-3)
    scale = s / torch.sqrt(torch.maximum(n2, s * s))
    return p * scale.unsqueeze(-3)


def data_image(u0, npos, nneg, dpos, dneg):
    """f = u0 exp(dpos n+ - dneg n-)."""
    return u0 * torch.exp(dpos * npos.to(u0.dtype) - dneg * nneg.to(u0.dtype))


def unrolled(u0: torch.Tensor, npos: torch.Tensor, nneg: torch.Tensor, tx: torch.Tensor,
             ty: torch.Tensor, w: Optional[torch.Tensor], lam, dpos, dneg, iters: int,
             tau: float = STEP, sigma: float = STEP, u_min: float = 1.0,
             u_max: float = math.e, p0: Optional[torch.Tensor] = None
             ) -> Tuple[torch.Tensor, torch.Tensor]:
    """K = iters iterations from (u0, p0); returns (u_K, p_K).

    Shapes: u0, npos, nneg, tx, ty, w: [..., H, W]; p0: [..., 3, H, W]
    (zero if None); lam, dpos, dneg: scalars (floats or 0-dim tensors).
    Everything is promoted to float64."""
    dt = torch.float64
    u0 = u0.to(dt)
    tx, ty = tx.to(dt), ty.to(dt)
    w = torch.ones_like(u0) if w is None else w.to(dt)
    lam = torch.as_tensor(lam, dtype=dt)
    dpos = torch.as_tensor(dpos, dtype=dt)
    dneg = torch.as_tensor(dneg, dtype=dt)
    m, s = metric(tx, ty)
    f = data_image(u0, npos, nneg, dpos, dneg)
    beta = tau * lam * w * s
    u = u0
    p = torch.zeros(u0.shape[:-2] + (3,) + u0.shape[-2:], dtype=dt) if p0 is None else p0.to(dt)
    for _ in range(iters):
        ubar = u - tau * apply_LgT(m, p)
        un = prox_kl(ubar, beta, f, u_min, u_max)
        p = project(p + sigma * apply_Lg(m, 2.0 * un - u), s)
        u = un
    return u, p
