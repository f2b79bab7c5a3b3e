"""The forward of the differentiable solve that allocates nothing
(rec_diff_forward_noalloc: data image and ping-pong states in a static
device array) against the workspace form rec_diff_forward, through the C ABI:
same bits of u_K and p_K on two calls in a row, the second smaller, and the
size limit rejected before any device work."""
import numpy as np
import pytest

import evgen
from paper_1607_06283_amd import rec

pytestmark = pytest.mark.gpu

SCRATCH_PIXELS = 1 << 20


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def _both(torch, B, H, W, iters, seed, unfused=False):
    """u_K, p_K of the workspace form and of the allocation-free form."""
    inp = {k: torch.from_numpy(v).cuda() for k, v in evgen.diff_inputs(seed, B, H, W).items()}
    theta = torch.tensor([90.0, 0.2, 0.25], dtype=torch.float64, device="cuda")
    d = rec.rec_diff_desc_make(W, H, B, iters, ckpt_every=10, unfused=unfused)
    ins = rec._diff_inputs(inp["u0"], None, inp["npos"], inp["nneg"], inp["tx"], inp["ty"],
                           inp["w"], theta)
    stream = torch.cuda.current_stream().cuda_stream
    nbytes = rec.rec_diff_workspace_bytes(d)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    u_ws = torch.full((B, H, W), np.nan, dtype=torch.float32, device="cuda")
    p_ws = torch.full((B, 3, H, W), np.nan, dtype=torch.float32, device="cuda")
    u_na = torch.full_like(u_ws, np.nan)
    p_na = torch.full_like(p_ws, np.nan)
    print(f"no-alloc forward B={B} H={H} W={W} iters={iters} unfused={unfused}", flush=True)
    assert rec.rec_diff_forward(d, ins, u_ws, p_ws, ws.data_ptr(), nbytes, stream) == rec.REC_OK
    assert rec.rec_diff_forward_noalloc(d, ins, u_na, p_na, stream) == rec.REC_OK
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (u_ws, p_ws, u_na, p_na)]


def test_noalloc_forward_equals_workspace_forward():
    torch = _torch()
    # a batch near the array's limit, then a smaller ragged one: the second
    # call must not see anything of the first
    for B, H, W, iters, seed in [(11, 260, 346, 23, 1), (2, 37, 70, 9, 2)]:
        assert B * H * W <= SCRATCH_PIXELS
        u_ws, p_ws, u_na, p_na = _both(torch, B, H, W, iters, seed)
        assert np.isfinite(u_ws).all() and np.isfinite(p_ws).all()
        assert np.array_equal(u_na, u_ws) and np.array_equal(p_na, p_ws)


def test_noalloc_unfused_and_zero_iterations():
    torch = _torch()
    u_ws, p_ws, u_na, p_na = _both(torch, 1, 33, 65, 5, 3, unfused=True)
    assert np.array_equal(u_na, u_ws) and np.array_equal(p_na, p_ws)
    u_ws, p_ws, u_na, p_na = _both(torch, 1, 33, 65, 0, 4)
    assert np.array_equal(u_na, u_ws) and np.array_equal(p_na, p_ws)


def test_noalloc_rejects_inputs_beyond_the_limit():
    torch = _torch()
    H, W = 1024, 1025  # one column past 2^20 pixels
    d = rec.rec_diff_desc_make(W, H, 1, 3)
    dummy = torch.zeros(1, dtype=torch.float32, device="cuda")
    th = torch.zeros(3, dtype=torch.float64, device="cuda")
    ins = rec._diff_inputs(dummy, None, dummy, dummy, dummy, dummy, None, th)
    stream = torch.cuda.current_stream().cuda_stream
    assert rec.rec_diff_forward_noalloc(d, ins, dummy, None, stream) == rec.REC_ENOMEM
    d_ok = rec.rec_diff_desc_make(1024, 1024, 1, 3)
    assert rec.rec_diff_forward_noalloc(d_ok, ins, None, None, stream) == rec.REC_EINVAL
