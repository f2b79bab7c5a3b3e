"""Helpers shared by the GPU test modules (not collected by pytest)."""
import numpy as np

import oracle
from paper_1607_06283_amd import rec

U_TOL = 1e-4
# The dual field p lives in a ball of radius s = sqrt(G) per pixel.  The
# primal-dual map is nonexpansive (Chambolle-Pock, in the norm
# |u|^2 / tau + |p|^2 / sigma), so FP32 rounding cannot be amplified from one
# iteration to the next: after n iterations the FP32 iterate is within the
# sum of the per-iteration rounding errors of the exact one.  One iteration
# of a pixel's dual update (difference of the extrapolated image, metric
# weighting, step, norm and projection) rounds at most 16 times on values of
# size s, each with relative error 2^-24.  Unlike u, which the strongly
# convex data term pins down, p is not unique where the image is flat, so
# nothing pulls the rounding back: the bound is the linear one.
P_OPS_PER_ITER = 16


def p_tol(n_iters: int) -> float:
    """Bound on max |p_gpu - p_oracle| / s after n_iters FP32 iterations."""
    return n_iters * P_OPS_PER_ITER * 2.0 ** -24


def oracle_params(prm: rec.rec_params) -> oracle.Params:
    return oracle.Params(prm.width, prm.height, lam=prm.lambda_, delta_pos=prm.delta_pos,
                         delta_neg=prm.delta_neg, u_min=prm.u_min, u_max=prm.u_max, tau=prm.tau,
                         sigma=prm.sigma, time_unit_us=prm.time_unit_us, u_init=prm.u_init,
                         tvl1_iters=prm.tvl1_iters, tvl1_lambda=prm.tvl1_lambda)


def make(W, H, u0=None, **kw):
    prm = rec.rec_default_params(W, H, **kw)
    r = rec.Reconstructor(W, H, params=prm, u0=u0)
    o = oracle.Oracle(oracle_params(prm), u0=u0)
    return r, o


def device_events(ev):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(ev.t)).cuda(),
            torch.from_numpy(np.ascontiguousarray(ev.x).view(np.int16)).cuda(),
            torch.from_numpy(np.ascontiguousarray(ev.y).view(np.int16)).cuda(),
            torch.from_numpy(np.ascontiguousarray(ev.p)).cuda())


def radius(o: oracle.Oracle) -> np.ndarray:
    """Ball radius sqrt(G) of every pixel from the oracle's FP64 time differences."""
    tx, ty = o.get(oracle.TX), o.get(oracle.TY)
    return np.sqrt(1.0 + tx * tx + ty * ty)


def u_p_errors(r, o):
    """(max |u - u_o|, max |p - p_o| / s) of a library context against the oracle."""
    du = float(np.abs(r.image(rec.REC_U).astype(np.float64) - o.u).max())
    dp = np.abs(r.image(rec.REC_STATE_P).astype(np.float64) - o.p).max(axis=0)
    return du, float((dp / radius(o)).max())
