"""Surrogate kernels (HIP) against the FP64 oracle (GPU).

Inputs that enter the BF16 matrix cores are made BF16-representable on the
host, so the oracle sees exactly what the kernels see; the remaining
difference is FP32 accumulation (tolerance 2e-5 relative to the output scale).
The whole U-Net, with BF16 activations between layers, is compared by the
relative error of each parameter gradient (bound 3e-2) and its cosine
similarity.
"""
import ctypes as ct
import sys

import numpy as np
import pytest

from oracle import lbm
from oracle import surrogate as OS
from tests import cases

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(9090)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bf16_round(a):
    """Round FP32 values to BF16 (nearest even); returns (float64 values, int16 bits)."""
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    bits = u.astype(np.uint16)
    vals = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return vals, bits.view(np.int16)


def dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda:0")


def host(t):
    return t.cpu().numpy()


def _lib():
    from paper_2607_06794_amd import _lib as L

    return L, L.load()


def _stream():
    import torch

    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _conv(x1, c1, up1, x2, c2, w, b, D, H, W, cout, relu, y=None, yf=None):
    L, _ = _lib()
    cv = L.LbConv()
    cv.x1, cv.c1, cv.up1 = x1.data_ptr(), c1, up1
    cv.x2, cv.c2 = (x2.data_ptr() if x2 is not None else None), c2
    cv.w = w.data_ptr()
    cv.b = b.data_ptr() if b is not None else None
    cv.y = y.data_ptr() if y is not None else None
    cv.yf = yf.data_ptr() if yf is not None else None
    cv.D, cv.H, cv.W, cv.cout, cv.relu = D, H, W, cout, relu
    return cv


@pytest.mark.parametrize("D,H,W,c1,c2,cout,up", [(3, 5, 7, 8, 0, 8, 0), (4, 6, 10, 16, 0, 72, 0),
                                                   (4, 6, 8, 32, 16, 40, 1), (6, 10, 22, 64, 32, 128, 1)])
def test_conv_forward_and_gradients(D, H, W, c1, c2, cout, up):
    import torch

    L, lib = _lib()
    say(f"[gpu] conv D={D} H={H} W={W} c1={c1} c2={c2} cout={cout} up={up}")
    cin = c1 + c2
    sh1 = (D // 2, H // 2, W // 2, c1) if up else (D, H, W, c1)
    x1, x1b = bf16_round(RNG.normal(size=sh1))
    x2, x2b = bf16_round(RNG.normal(size=(D, H, W, c2))) if c2 else (np.zeros((D, H, W, 0)), None)
    w, wb = bf16_round(RNG.normal(size=(27, cin, cout)) / np.sqrt(27 * cin))
    b = RNG.normal(size=cout).astype(np.float32)
    xin = np.concatenate([OS.up2(x1) if up else x1, x2], axis=-1)
    # forward (FP32 output, ReLU off, then on)
    yf = torch.zeros(D * H * W * cout, dtype=torch.float32, device="cuda:0")
    y = torch.zeros(D * H * W * cout, dtype=torch.int16, device="cuda:0")
    tx1, tw, tb = dev(x1b), dev(wb), dev(b)
    tx2 = dev(x2b) if c2 else None
    cv = _conv(tx1, c1, up, tx2, c2, tw, tb, D, H, W, cout, 1, y=y, yf=yf)
    L.check(lib.lb_conv3d_forward(ct.byref(cv), _stream()))
    ref = np.maximum(OS.conv3d(xin, w, b.astype(np.float64)), 0.0)
    got = host(yf).reshape(D, H, W, cout)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 2e-5 * scale
    # gradients with the ReLU mask of this output; dy BF16-representable
    dyv, _ = bf16_round(RNG.normal(size=(D, H, W, cout)))
    tdy = dev(dyv.astype(np.float32))
    ybits = host(y).reshape(D, H, W, cout)
    yv = (ybits.astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
    g = dyv * (yv > 0)
    dx = torch.zeros(D * H * W * cin, dtype=torch.float32, device="cuda:0")
    L.check(lib.lb_conv3d_backward_data(ct.byref(cv), tdy.data_ptr(), dx.data_ptr(), _stream()))
    dref = OS.conv3d_dgrad(g, w)
    assert np.abs(host(dx).reshape(D, H, W, cin) - dref).max() <= 2e-5 * np.abs(dref).max()
    dw = torch.zeros(27 * cin * cout, dtype=torch.float32, device="cuda:0")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda:0")
    L.check(lib.lb_conv3d_backward_weights(ct.byref(cv), tdy.data_ptr(), dw.data_ptr(), db.data_ptr(), _stream()))
    wref, bref = OS.conv3d_wgrad(xin, g)
    assert np.abs(host(dw).reshape(27, cin, cout) - wref).max() <= 2e-5 * np.abs(wref).max()
    assert np.abs(host(db) - bref).max() <= 2e-5 * np.abs(bref).max()


def test_pooling_and_plumbing():
    import torch

    L, lib = _lib()
    D, H, W, C = 4, 6, 10, 16
    x, xb = bf16_round(RNG.normal(size=(D, H, W, C)))
    y = torch.zeros(D * H * W * C // 8, dtype=torch.int16, device="cuda:0")
    L.check(lib.lb_pool2(dev(xb).data_ptr(), D, H, W, C, y.data_ptr(), _stream()))
    yv = (host(y).astype(np.uint16).astype(np.uint32) << 16).view(np.float32).reshape(D // 2, H // 2, W // 2, C)
    ref = OS.pool2(x)
    assert np.abs(yv - ref).max() <= np.abs(ref).max() * 2 ** -8
    gc = RNG.normal(size=(D // 2, H // 2, W // 2, C)).astype(np.float32)
    skip = RNG.normal(size=(D, H, W, 24)).astype(np.float32)
    g = torch.zeros(D * H * W * C, dtype=torch.float32, device="cuda:0")
    L.check(lib.lb_pool2_backward(dev(gc).data_ptr(), dev(skip).data_ptr(), 24, 8, D, H, W, C, g.data_ptr(), _stream()))
    assert np.allclose(host(g).reshape(D, H, W, C), OS.pool2_back(gc) + skip[..., 8:24], rtol=1e-6, atol=1e-7)
    gc2 = torch.zeros(D * H * W * C // 8, dtype=torch.float32, device="cuda:0")
    L.check(lib.lb_up2_backward(dev(skip).data_ptr(), 24, C, D, H, W, gc2.data_ptr(), _stream()))
    assert np.allclose(host(gc2).reshape(D // 2, H // 2, W // 2, C), OS.up2_back(skip[..., :C]), rtol=1e-5, atol=1e-6)


def test_loss_and_adam():
    import torch

    L, lib = _lib()
    P = 1000
    out = RNG.normal(size=(P, 8)).astype(np.float32) * 0.1
    xin = RNG.normal(size=(P, 8)).astype(np.float32) + 1.0
    xin[:, 6] = (RNG.uniform(size=P) > 0.2).astype(np.float32)
    tgt = RNG.normal(size=(P, 8)).astype(np.float32) + 1.0
    scratch = torch.zeros(lib.lb_sur_loss_scratch_bytes() // 4 + 16, dtype=torch.float32, device="cuda:0")
    grad = torch.zeros(P * 8, dtype=torch.float32, device="cuda:0")
    res = (ct.c_double * 4)()
    L.check(lib.lb_sur_loss(dev(out).data_ptr(), dev(xin).data_ptr(), dev(tgt).data_ptr(), P, 0.5, grad.data_ptr(),
                            scratch.data_ptr(), res, _stream()))
    pred = xin[:, :6].astype(np.float64) + out[:, :6]
    Lr, gr = OS.loss(pred, tgt[:, :6].astype(np.float64), xin[:, 6].astype(np.float64), 0.5)
    assert res[3] == pytest.approx(Lr, rel=1e-10)
    assert np.allclose(host(grad).reshape(P, 8)[:, :6], gr, rtol=1e-5, atol=1e-9)
    assert np.all(host(grad).reshape(P, 8)[:, 6:] == 0)
    p = RNG.normal(size=500).astype(np.float32)
    gg = RNG.normal(size=500).astype(np.float32)
    tp, tg = dev(p), dev(gg)
    tm, tv = dev(np.zeros(500, np.float32)), dev(np.zeros(500, np.float32))
    tb = torch.zeros(500, dtype=torch.int16, device="cuda:0")
    pr, mr, vr = p.astype(np.float64), np.zeros(500), np.zeros(500)
    for step in (1, 2, 3):
        L.check(lib.lb_adam(tp.data_ptr(), tg.data_ptr(), tm.data_ptr(), tv.data_ptr(), tb.data_ptr(), 500, step, 1e-2,
                            0.9, 0.999, 1e-8, _stream()))
        pr, mr, vr = OS.adam(pr, gg.astype(np.float64), mr, vr, step, lr=1e-2)
    assert np.allclose(host(tp), pr, rtol=1e-5, atol=1e-6)


def test_restrict_and_lift_match_oracle():
    import torch

    from paper_2607_06794_amd.sim import Lattice

    L, lib = _lib()
    c = cases.cap_case(shape=(16, 24, 40), footprint=(26.0, 10.0), height=8.0, stripe=(30, 14))
    lat = Lattice(cases.lattice_params(c, "f64"), c["rho"], c["mat"])
    lat.step(20)
    D, H, W = 10, 14, 24  # larger than the lattice's 8 x 12 x 20 coarse extent
    cf = torch.zeros(D * H * W * 8, dtype=torch.float32, device="cuda:0")
    L.check(lib.lb_sur_restrict(lat._ctx, D, H, W, cf.data_ptr(), None, _stream()))
    _, f = lat.export()
    ref = OS.restrict(f, c["mat"], (D, H, W))
    got = host(cf).reshape(D, H, W, 8)
    assert np.abs(got[..., :7] - ref).max() <= 1e-6 * max(1.0, np.abs(ref).max())
    assert np.all(got[..., 7] == 0)
    # lift a perturbed canvas and compare the populations (FP64 storage)
    coarse = ref.copy()
    coarse[..., 0] *= 1.0 + 0.01 * RNG.normal(size=coarse.shape[:3])
    cc = np.zeros((D, H, W, 8), np.float32)
    cc[..., :7] = coarse
    L.check(lib.lb_sur_lift(lat._ctx, dev(cc).data_ptr(), D, H, W, _stream()))
    _, f2 = lat.export()
    want = OS.lift(cc[..., :7].astype(np.float64), c["mat"])
    fl = (c["mat"] == lbm.FLUID)[None, None]
    assert np.abs(np.where(fl, f2 - want, 0)).max() <= 1e-12
    lat.close()


def test_unet_gradients_match_oracle():
    from paper_2607_06794_amd.surrogate import UNet

    D, H, W = 8, 16, 16
    ch = (8, 16, 16, 16)
    say(f"[gpu] unet canvas {D}x{H}x{W} ch={ch}")
    P = OS.init_params(21, cin=7, ch=ch, cout=6)
    P["out"] = (RNG.normal(size=P["out"][0].shape) * 0.05, RNG.normal(size=6) * 0.05)
    net = UNet(D, H, W, ch=ch)
    for name, (w, b) in P.items():
        wv, _ = bf16_round(w)
        P[name] = (wv, b.astype(np.float32).astype(np.float64))
        net.set_layer(name, wv, P[name][1])
    x = np.zeros((D, H, W, 8))
    x[..., :7] = RNG.normal(size=(D, H, W, 7))
    xv, xb = bf16_round(x)
    tx = dev(xb.reshape(-1))
    out = net.forward(tx)
    pred_ref, cache = OS.unet_forward(xv[..., :7], P, ch=ch)
    got = host(out).reshape(D, H, W, 8)[..., :6] + xv[..., :6]
    err = np.abs(got - pred_ref).max() / np.abs(pred_ref - xv[..., :6]).max()
    say(f"[gpu] unet forward rel err {err:.2e}")
    assert err < 3e-2
    gy = RNG.normal(size=(D, H, W, 6))
    g8 = np.zeros((D, H, W, 8), np.float32)
    g8[..., :6] = gy
    net.zero_grad()
    net.backward(dev(g8.reshape(-1)))
    G = OS.unet_backward(gy, P, cache, ch=ch)
    for name, (gw, gb) in G.items():
        ww, bb = net.get_layer_grad(name)
        ww = ww[:, : gw.shape[1], : gw.shape[2]]
        bb = bb[: gb.shape[0]]
        rel = np.linalg.norm(ww - gw) / np.linalg.norm(gw)
        cos = float((ww * gw).sum() / (np.linalg.norm(ww) * np.linalg.norm(gw)))
        say(f"[gpu] grad {name}: rel {rel:.2e} cos {cos:.6f}")
        assert rel < 3e-2 and cos > 0.999, name
        assert np.linalg.norm(bb - gb) <= 3e-2 * np.linalg.norm(gb) + 1e-6, name
