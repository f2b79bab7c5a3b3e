"""Helpers shared by the GPU test modules (not collected by pytest)."""
import numpy as np

import oracle
from paper_1607_06283_amd import rec

U_TOL = 1e-4
# The dual field p lives in a ball of radius s = sqrt(G) per pixel and is
# stored and updated in FP32 like u; its rounding errors scale with that
# radius.  The Chambolle-Pock map is nonexpansive in the norm
# |u|^2 / tau + |p|^2 / sigma (tau = sigma here), so FP32 rounding
# perturbs p no more than it perturbs u, relative to their ranges: u's bound
# of 1e-4 on [1, e] becomes 1e-4 * s per pixel for p.
P_RTOL = 1e-4


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
