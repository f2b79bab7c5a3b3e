"""Differentiable unrolled solve on the GPU (rec_diff_forward / _backward
through the torch.autograd.Function) against the FP64 autograd reference
and central finite differences of the FP64 C oracle."""
import math

import numpy as np
import pytest

import evgen
import oracle
from oracle import autodiff
from paper_1607_06283_amd import rec

pytestmark = pytest.mark.gpu

LAM, DPOS, DNEG = 90.0, 0.2, 0.25
GRAD_RTOL = 1e-3


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(inp):
    torch = _torch()
    return {k: torch.from_numpy(v).cuda() for k, v in inp.items()}


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _gpu_grads(inp, iters, ckpt, p0=None, seed=5, use_w=True, unfused=False, gu=None, gp=None):
    """Forward + backward on the GPU of J = <gu, u_K> + <gp, p_K>."""
    torch = _torch()
    d = _dev(inp)
    B, H, W = inp["u0"].shape
    rng = np.random.default_rng(seed)
    if gu is None:
        gu = rng.standard_normal((B, H, W))
        gp = rng.standard_normal((B, 3, H, W))
    u0 = d["u0"].clone().requires_grad_()
    w = d["w"].clone().requires_grad_() if use_w else None
    th = torch.tensor([LAM, DPOS, DNEG], dtype=torch.float64, device="cuda", requires_grad=True)
    p0t = None if p0 is None else torch.from_numpy(p0.astype(np.float32)).cuda().requires_grad_()
    print(f"gpu diff B={B} H={H} W={W} iters={iters} ckpt={ckpt} unfused={unfused}", flush=True)
    u, p = rec.unrolled(u0, d["npos"], d["nneg"], d["tx"], d["ty"], th, iters, w=w, p0=p0t,
                        ckpt_every=ckpt, unfused=unfused)
    J = (torch.from_numpy(gu).cuda() * u.double()).sum() + \
        (torch.from_numpy(gp).cuda() * p.double()).sum()
    J.backward()
    torch.cuda.synchronize()
    out = dict(u=u.detach().cpu().numpy(), p=p.detach().cpu().numpy(),
               u0=u0.grad.cpu().numpy(), theta=th.grad.cpu().numpy(), gu=gu, gp=gp)
    if use_w:
        out["w"] = w.grad.cpu().numpy()
    if p0t is not None:
        out["p0"] = p0t.grad.cpu().numpy()
    return out


def _ref_grads(inp, iters, gu, gp, p0=None, use_w=True):
    import torch
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    u0 = t(inp["u0"]).requires_grad_()
    w = t(inp["w"]).requires_grad_() if use_w else None
    th = torch.tensor([LAM, DPOS, DNEG], dtype=torch.float64, requires_grad=True)
    p0t = None if p0 is None else t(p0.astype(np.float32)).requires_grad_()
    u, p = autodiff.unrolled(u0, t(inp["npos"]), t(inp["nneg"]), t(inp["tx"]), t(inp["ty"]),
                             w, th[0], th[1], th[2], iters, p0=p0t)
    ((t(gu) * u).sum() + (t(gp) * p).sum()).backward()
    out = dict(u=u.detach().numpy(), p=p.detach().numpy(), u0=u0.grad.numpy(),
               theta=th.grad.numpy())
    if use_w:
        out["w"] = w.grad.numpy()
    if p0t is not None:
        out["p0"] = p0t.grad.numpy()
    return out


@pytest.fixture(scope="module")
def ragged():
    # 70 columns (one full 64-wide tile and a ragged one), 37 rows (ragged
    # against 4-row workgroups), two images
    return evgen.diff_inputs(21, 2, 37, 70)


@pytest.mark.parametrize("ckpt", [7, 30])
def test_gradients_match_fp64_autograd(ragged, ckpt):
    rng = np.random.default_rng(9)
    p0 = 0.05 * rng.standard_normal((2, 3, 37, 70))
    g = _gpu_grads(ragged, 30, ckpt, p0=p0)
    r = _ref_grads(ragged, 30, g["gu"], g["gp"], p0=p0)
    assert np.abs(g["u"] - r["u"]).max() <= 1e-4
    for k in ("u0", "w", "p0"):
        e = _rel(g[k], r[k])
        print(f"  d/d{k}: relative error {e:.2e}")
        assert e <= GRAD_RTOL, k
    for i, name in enumerate(("lambda", "dpos", "dneg")):
        e = abs(g["theta"][i] - r["theta"][i]) / abs(r["theta"][i])
        print(f"  d/d{name}: {g['theta'][i]:.6e} vs {r['theta'][i]:.6e} ({e:.2e})")
        assert e <= GRAD_RTOL, name


def test_checkpoint_interval_and_form_do_not_change_bits(ragged):
    """Recomputed segments reproduce the forward bit for bit, and the fused
    register-tile kernels run the same per-pixel arithmetic as the one-launch-
    per-half-step form, so every checkpoint interval and both forms give the
    same bits."""
    outs = [_gpu_grads(ragged, 24, k, unfused=uf) for uf in (True, False)
            for k in (1, 5, 7, 24)]
    for o in outs[1:]:
        for key in ("u", "p", "u0", "w", "theta"):
            assert np.array_equal(o[key], outs[0][key]), key


@pytest.mark.slow
def test_full_size_fused_equals_unfused_and_fp64():
    """The differentiation workload's size (16 x 346x260, 100 iterations,
    checkpoints every 10) in the fused form the benchmark times: bit-equal to
    the two-kernel form; and, with the loss on two sampled images (the
    images are independent), the gradients against FP64 autograd of those
    two images.  Inputs keep f inside (1, e), away from the clamp's kinks."""
    inp = evgen.diff_inputs(500, 16, 260, 346, levels=(0.35, 0.65), max_count=1)
    iters = 100
    B, H, W = inp["u0"].shape
    rng = np.random.default_rng(8)
    gu = np.zeros((B, H, W))
    gp = np.zeros((B, 3, H, W))
    pick = [0, 9]
    for b in pick:
        gu[b] = rng.standard_normal((H, W))
        gp[b] = rng.standard_normal((3, H, W))
    gf = _gpu_grads(inp, iters, 10, gu=gu, gp=gp)
    gx = _gpu_grads(inp, iters, 10, gu=gu, gp=gp, unfused=True)
    for key in ("u", "p", "u0", "w", "theta"):
        assert np.array_equal(gf[key], gx[key]), key
    sub = {k: v[pick] for k, v in inp.items()}
    r = _ref_grads(sub, iters, gu[pick], gp[pick])
    assert np.abs(gf["u"][pick] - r["u"]).max() <= 1e-4
    for k in ("u0", "w"):
        e = _rel(gf[k][pick], r[k])
        print(f"  full size d/d{k}: relative error {e:.2e}")
        assert e <= GRAD_RTOL, k
    for i, name in enumerate(("lambda", "dpos", "dneg")):
        e = abs(gf["theta"][i] - r["theta"][i]) / abs(r["theta"][i])
        print(f"  full size d/d{name}: {gf['theta'][i]:.6e} vs {r['theta'][i]:.6e} ({e:.2e})")
        assert e <= GRAD_RTOL, name


def test_fused_large_tile_shape_equals_unfused():
    """Above 250k pixels the fused forward uses 64-row tiles; ragged
    segments (10, 10, 3) and reverse chunks (5, 5, 3)."""
    inp = evgen.diff_inputs(33, 2, 301, 455)
    a = _gpu_grads(inp, 23, 10)
    b = _gpu_grads(inp, 23, 10, unfused=True)
    for key in ("u", "p", "u0", "w", "theta"):
        assert np.array_equal(a[key], b[key]), key


def test_scalar_gradients_match_finite_differences(ragged):
    """dJ/d(lambda, dpos, dneg) vs central differences of the FP64 C oracle."""
    iters = 20
    g = _gpu_grads(ragged, iters, 10, use_w=False)
    B, H, W = ragged["u0"].shape

    def J(lam, dpos, dneg):
        tot = 0.0
        for b in range(B):
            o = oracle.Oracle(oracle.Params(W, H, lam=lam, delta_pos=dpos, delta_neg=dneg))
            u = ragged["u0"][b].astype(np.float64)
            o.set_state(u)
            o.set_data(u * np.exp(dpos * ragged["npos"][b] - dneg * ragged["nneg"][b]),
                       ragged["tx"][b].astype(np.float64), ragged["ty"][b].astype(np.float64))
            o.iterate(iters)
            tot += (g["gu"][b] * o.u).sum() + (g["gp"][b] * o.p).sum()
            o.close()
        return tot

    base = [LAM, DPOS, DNEG]
    for i, name in enumerate(("lambda", "dpos", "dneg")):
        h = 1e-6 * max(abs(base[i]), 1.0)
        up, dn = list(base), list(base)
        up[i] += h
        dn[i] -= h
        fd = (J(*up) - J(*dn)) / (2 * h)
        e = abs(g["theta"][i] - fd) / abs(fd)
        print(f"  d/d{name}: gpu {g['theta'][i]:.6e} fd {fd:.6e} ({e:.2e})")
        assert e <= GRAD_RTOL, name


def test_forward_equals_stream_solve_bitwise():
    """With w = 1 and p0 = 0 the unrolled forward is the library's solve of
    the first block: same f, same metric, p in the same tangent frame
    between the first and the last iteration, same bits."""
    torch = _torch()
    spec = evgen.StreamSpec(96, 70, 31, duration_us=30_000)
    ev = evgen.generate(spec).events
    blk = ev.slice(0, 3000)
    r = rec.Reconstructor(96, 70, fuse_iters=0)
    r.push(blk.t, blk.x, blk.y, blk.p)
    npos, nneg = r.image(rec.REC_COUNT_POS), r.image(rec.REC_COUNT_NEG)
    r.solve(25)
    u_ref, tx, ty = r.image(rec.REC_U), r.image(rec.REC_TX), r.image(rec.REC_TY)
    u0 = torch.full((1, 70, 96), r.prm.u_init, dtype=torch.float32, device="cuda")
    th = torch.tensor([r.prm.lambda_, r.prm.delta_pos, r.prm.delta_neg], dtype=torch.float64,
                      device="cuda")
    c = lambda a: torch.from_numpy(np.ascontiguousarray(a)[None]).cuda()
    u, p = rec.unrolled(u0, c(npos), c(nneg), c(tx), c(ty), th, 25, ckpt_every=10,
                        tau=r.prm.tau, sigma=r.prm.sigma, u_min=r.prm.u_min, u_max=r.prm.u_max)
    assert np.array_equal(u[0].cpu().numpy(), u_ref)
    assert np.array_equal(p[0].cpu().numpy(), r.image(rec.REC_STATE_P))
    r.close()


def test_log_intensity_loss_through_autograd(ragged):
    """The training loss 1/2 sum (log u_K - L)^2 differentiated end to end by
    torch (its own log and square, the library's reverse sweep)."""
    T = _torch()
    d = _dev(ragged)
    L = np.log(ragged["u0"].astype(np.float64)) + 0.05
    iters = 25
    th = T.tensor([LAM, DPOS, DNEG], dtype=T.float64, device="cuda", requires_grad=True)
    w = d["w"].clone().requires_grad_()
    u, _ = rec.unrolled(d["u0"], d["npos"], d["nneg"], d["tx"], d["ty"], th, iters, w=w)
    loss = 0.5 * ((T.log(u.double()) - T.from_numpy(L).cuda()) ** 2).sum()
    loss.backward()
    t = lambda a: T.from_numpy(np.asarray(a, np.float64))
    thr = T.tensor([LAM, DPOS, DNEG], dtype=T.float64, requires_grad=True)
    wr = t(ragged["w"]).requires_grad_()
    ur, _ = autodiff.unrolled(t(ragged["u0"]), t(ragged["npos"]), t(ragged["nneg"]),
                              t(ragged["tx"]), t(ragged["ty"]), wr, thr[0], thr[1], thr[2], iters)
    lr = 0.5 * ((T.log(ur) - t(L)) ** 2).sum()
    lr.backward()
    assert abs(loss.item() - lr.item()) <= 1e-4 * abs(lr.item())
    assert _rel(th.grad.cpu().numpy(), thr.grad.numpy()) <= GRAD_RTOL
    assert _rel(w.grad.cpu().numpy(), wr.grad.numpy()) <= GRAD_RTOL


@pytest.mark.parametrize("B,H,W", [(1, 1, 1), (1, 1, 70), (2, 37, 1), (3, 5, 3)])
def test_degenerate_shapes(B, H, W):
    """Single pixels, single rows and columns: both forms give the same bits
    and match FP64 autograd (iterations 7, checkpoints every 3)."""
    inp = evgen.diff_inputs(B * 100 + H * 10 + W, B, H, W)
    a = _gpu_grads(inp, 7, 3)
    b = _gpu_grads(inp, 7, 3, unfused=True)
    for key in ("u", "p", "u0", "w", "theta"):
        assert np.array_equal(a[key], b[key]), key
    r = _ref_grads(inp, 7, a["gu"], a["gp"])
    assert np.abs(a["u"] - r["u"]).max() <= 1e-4
    for k in ("u0", "w"):
        # a lone pixel's dJ/dw is ~1e-12 (FP32 rounding noise): absolute floor
        err = np.linalg.norm(a[k].astype(np.float64) - r[k])
        assert err <= GRAD_RTOL * np.linalg.norm(r[k]) + 1e-6 * np.sqrt(r[k].size), k
    # lambda and the thresholds: compare where the reference gradient is not ~0
    for i in range(3):
        if abs(r["theta"][i]) > 1e-6:
            assert abs(a["theta"][i] - r["theta"][i]) <= GRAD_RTOL * abs(r["theta"][i]) + 1e-6


def test_zero_iterations_pass_gradients_through(ragged):
    g = _gpu_grads(ragged, 0, 1, p0=np.zeros((2, 3, 37, 70)))
    assert np.array_equal(g["u"], ragged["u0"])
    assert np.allclose(g["u0"], g["gu"].astype(np.float32), rtol=0, atol=0)
    assert np.allclose(g["p0"], g["gp"].astype(np.float32), rtol=0, atol=0)
    assert not g["w"].any() and not g["theta"].any()


def test_bad_descriptors_rejected():
    torch = _torch()
    d = _dev(evgen.diff_inputs(1, 1, 8, 8))
    th = torch.tensor([LAM, DPOS, DNEG], dtype=torch.float64, device="cuda")
    with pytest.raises(rec.RecError):
        rec.unrolled(d["u0"], d["npos"], d["nneg"], d["tx"], d["ty"], th, 5, tau=1.0, sigma=1.0)


@pytest.mark.slow
def test_diff16_event_blocks_against_fp64_autograd():
    """The differentiation workload itself: 16 blocks of 2000 events from
    346x260 streams (seeds 500-515), u0 = exp(L_gt(t0)), 100 unrolled
    iterations, checkpoints every 10, loss 1/2 sum (log u - L_gt(t_end))^2.
    The block data (counts, time differences) come from the FP64 oracle's
    scatter and build.  The GPU solves all 16 images; the loss is taken on
    two sampled images (the images are independent, so the other images
    contribute nothing), whose gradients are compared with FP64 autograd
    (norm-relative 1e-3 for u0 and w, 1e-3 for lambda, Delta+, Delta-).
    These inputs put part of the image on the clamp's kinks: the fraction
    of clamped pixels and the pixels where the FP32 and FP64 iterations end
    on different sides of a clamp are reported."""
    torch = _torch()
    K, CK, W, H, NB = 100, 10, 346, 260, 16
    blocks = evgen.diff_blocks(500, NB, W, H, 2000)
    npos, nneg, tx, ty, u0, Lend = [], [], [], [], [], []
    for spec, blk, L0, L1 in blocks:
        o = oracle.Oracle(oracle.Params(W, H))
        o.push_events(blk)
        npos.append(o.get(oracle.NPOS))
        nneg.append(o.get(oracle.NNEG))
        o.build()
        tx.append(o.get(oracle.TX32))
        ty.append(o.get(oracle.TY32))
        o.close()
        u0.append(np.exp(L0).astype(np.float32))
        Lend.append(L1)
    inp = {"u0": np.stack(u0), "npos": np.stack(npos), "nneg": np.stack(nneg),
           "tx": np.stack(tx), "ty": np.stack(ty), "w": np.ones((NB, H, W), np.float32)}
    Lend = np.stack(Lend)
    pick = [3, 12]
    mask = np.zeros(NB)
    mask[pick] = 1.0
    d = _dev(inp)
    u0t = d["u0"].clone().requires_grad_()
    wt = d["w"].clone().requires_grad_()
    th = torch.tensor([90.0, 0.2, 0.2], dtype=torch.float64, device="cuda", requires_grad=True)
    print("diff16 event blocks: GPU forward + backward", flush=True)
    u, _ = rec.unrolled(u0t, d["npos"], d["nneg"], d["tx"], d["ty"], th, K, w=wt, ckpt_every=CK)
    m = torch.from_numpy(mask).cuda()[:, None, None]
    loss = 0.5 * (m * (torch.log(u.double()) - torch.from_numpy(Lend).cuda()) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    g = dict(u=u.detach().cpu().numpy()[pick], u0=u0t.grad.cpu().numpy()[pick],
             w=wt.grad.cpu().numpy()[pick], theta=th.grad.cpu().numpy())
    print("diff16 event blocks: FP64 autograd of the two sampled images", flush=True)
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    sub = {k: v[pick] for k, v in inp.items()}
    u0r = t(sub["u0"]).requires_grad_()
    wr = t(sub["w"]).requires_grad_()
    thr = torch.tensor([90.0, 0.2, 0.2], dtype=torch.float64, requires_grad=True)
    ur, _ = autodiff.unrolled(u0r, t(sub["npos"]), t(sub["nneg"]), t(sub["tx"]), t(sub["ty"]),
                              wr, thr[0], thr[1], thr[2], K)
    lr = 0.5 * ((torch.log(ur) - t(Lend[pick])) ** 2).sum()
    lr.backward()
    ref = ur.detach().numpy()
    clamped = (ref <= 1.0 + 1e-12) | (ref >= math.e - 1e-12)
    gpu_clamped = (g["u"] <= np.float32(1.0)) | (g["u"] >= np.float32(math.e))
    flips = int((clamped != gpu_clamped).sum())
    print(f"  clamp active at the end on {clamped.mean():.2%} of pixels; "
          f"FP32/FP64 on different sides: {flips} pixels")
    assert np.abs(g["u"] - ref).max() <= 1e-4
    assert abs(loss.item() - lr.item()) <= 1e-4 * abs(lr.item())
    for k, rg in (("u0", u0r.grad.numpy()), ("w", wr.grad.numpy())):
        e = _rel(g[k], rg)
        print(f"  d/d{k}: relative error {e:.2e}")
        assert e <= GRAD_RTOL, k
    for i, name in enumerate(("lambda", "dpos", "dneg")):
        rv = thr.grad.numpy()[i]
        e = abs(g["theta"][i] - rv) / abs(rv)
        print(f"  d/d{name}: {g['theta'][i]:.6e} vs {rv:.6e} ({e:.2e})")
        assert e <= GRAD_RTOL, name
