"""Surrogate kernels (HIP) against the FP64 oracle (GPU).

Inputs that enter the BF16 matrix cores are made BF16-representable on the
host, so the oracle sees exactly what the kernels see; the remaining
difference is FP32 accumulation (tolerance 2e-5 relative to the output scale).
The whole U-Net's parameter gradients are compared with the oracle's
backward pass run on the activations the GPU computed (BF16 values and the
same ReLU masks); the remaining difference is the rounding of each layer's
incoming gradient to BF16 (bound 2e-2 relative, cosine > 0.9998).  Each
single layer is checked at 2e-5 above.
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


def _conv(x1, c1, up1, x2, c2, w, b, D, H, W, cout, relu, y=None, yf=None, wt=None):
    L, _ = _lib()
    cv = L.LbConv()
    cv.x1, cv.c1, cv.up1 = x1.data_ptr(), c1, up1
    cv.x2, cv.c2 = (x2.data_ptr() if x2 is not None else None), c2
    cv.w = w.data_ptr()
    cv.wt = wt.data_ptr() if wt is not None else None
    cv.b = b.data_ptr() if b is not None else None
    cv.y = y.data_ptr() if y is not None else None
    cv.yf = yf.data_ptr() if yf is not None else None
    cv.D, cv.H, cv.W, cv.cout, cv.relu = D, H, W, cout, relu
    return cv


# Tile shapes follow N (output channels forward, input channels for the input
# gradient): <= 32, <= 64, > 64 (and > 128: two column tiles).  The larger
# cases span several work-groups with ragged last tiles and several
# weight-gradient position chunks; layers of few tiles split K (the forward
# when given FP32 scratch, checked both ways), the last case has enough tiles
# not to.
@pytest.mark.parametrize("D,H,W,c1,c2,cout,up", [(3, 5, 7, 8, 0, 8, 0), (4, 6, 10, 16, 0, 72, 0),
                                                   (4, 6, 8, 32, 16, 40, 1), (6, 10, 22, 64, 32, 128, 1),
                                                   (8, 16, 40, 32, 0, 32, 0), (6, 12, 34, 128, 64, 64, 1),
                                                   (8, 16, 42, 64, 32, 136, 1), (16, 32, 64, 32, 0, 32, 0),
                                                   (8, 8, 16, 16, 24, 32, 1), (4, 8, 8, 8, 0, 8, 0),
                                                   (8, 16, 24, 64, 32, 24, 1), (6, 8, 16, 32, 32, 64, 1),
                                                   (2, 8, 8, 24, 0, 48, 0)])
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
    twt = torch.zeros(27 * cin * cout, dtype=torch.int16, device="cuda:0")
    L.check(lib.lb_conv_pack_weights(tw.data_ptr(), cin, cout, twt.data_ptr(), _stream()))
    assert int((host(twt).reshape(cout, 27, cin) != wb.reshape(27, cin, cout).transpose(2, 0, 1)).sum()) == 0
    cv = _conv(tx1, c1, up, tx2, c2, tw, tb, D, H, W, cout, 1, y=y, yf=yf, wt=twt)
    L.check(lib.lb_conv3d_forward(ct.byref(cv), _stream()))
    ref = np.maximum(OS.conv3d(xin, w, b.astype(np.float64)), 0.0)
    got = host(yf).reshape(D, H, W, cout)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 2e-5 * scale
    # again with FP32 scratch: split K where the layer has few tiles
    acc = torch.zeros(D * H * W * cout, dtype=torch.float32, device="cuda:0")
    yf2 = torch.zeros_like(yf)
    y2 = torch.zeros_like(y)
    cv2 = _conv(tx1, c1, up, tx2, c2, tw, tb, D, H, W, cout, 1, y=y2, yf=yf2, wt=twt)
    cv2.acc = acc.data_ptr()
    L.check(lib.lb_conv3d_forward(ct.byref(cv2), _stream()))
    assert np.abs(host(yf2).reshape(D, H, W, cout) - ref).max() <= 2e-5 * scale
    # gradients with the ReLU mask of this output; dy BF16-representable
    dyv, _ = bf16_round(RNG.normal(size=(D, H, W, cout)))
    tdy = dev(dyv.astype(np.float32))
    ybits = host(y).reshape(D, H, W, cout)
    yv = (ybits.astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
    g = dyv * (yv > 0)
    tg = torch.zeros(D * H * W * cout, dtype=torch.int16, device="cuda:0")
    L.check(lib.lb_relu_grad(tdy.data_ptr(), y.data_ptr(), D * H * W * cout, 1, tg.data_ptr(), _stream()))
    gbits = bf16_round(np.where(yv > 0, dyv, 0.0))[1]  # +0 where masked, as the kernel writes
    assert int((host(tg).reshape(D, H, W, cout) != gbits).sum()) == 0
    dx = torch.zeros(D * H * W * cin, dtype=torch.float32, device="cuda:0")
    L.check(lib.lb_conv3d_backward_data(ct.byref(cv), tg.data_ptr(), dx.data_ptr(), _stream()))
    dref = OS.conv3d_dgrad(g, w)
    assert np.abs(host(dx).reshape(D, H, W, cin) - dref).max() <= 2e-5 * np.abs(dref).max()
    dw = torch.zeros(27 * cin * cout, dtype=torch.float32, device="cuda:0")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda:0")
    L.check(lib.lb_conv3d_backward_weights(ct.byref(cv), tg.data_ptr(), dw.data_ptr(), db.data_ptr(), _stream()))
    wref, bref = OS.conv3d_wgrad(xin, g)
    assert np.abs(host(dw).reshape(27, cin, cout) - wref).max() <= 2e-5 * np.abs(wref).max()
    assert np.abs(host(db) - bref).max() <= 2e-5 * np.abs(bref).max()


def test_pooling_and_plumbing():
    import torch

    L, lib = _lib()
    D, H, W, C = 4, 6, 10, 16
    x, xb = bf16_round(RNG.normal(size=(D, H, W, C)))
    y = torch.zeros(D * H * W * C // 8, dtype=torch.int16, device="cuda:0")
    tx = dev(xb)  # device tensors stay referenced until the kernels have run
    L.check(lib.lb_pool2(tx.data_ptr(), D, H, W, C, y.data_ptr(), _stream()))
    yv = (host(y).astype(np.uint16).astype(np.uint32) << 16).view(np.float32).reshape(D // 2, H // 2, W // 2, C)
    ref = OS.pool2(x)
    assert np.abs(yv - ref).max() <= np.abs(ref).max() * 2 ** -8
    gc = RNG.normal(size=(D // 2, H // 2, W // 2, C)).astype(np.float32)
    skip = RNG.normal(size=(D, H, W, 24)).astype(np.float32)
    g = torch.zeros(D * H * W * C, dtype=torch.float32, device="cuda:0")
    tgc, tskip = dev(gc), dev(skip)
    L.check(lib.lb_pool2_backward(tgc.data_ptr(), tskip.data_ptr(), 24, 8, D, H, W, C, g.data_ptr(), _stream()))
    assert np.allclose(host(g).reshape(D, H, W, C), OS.pool2_back(gc) + skip[..., 8:24], rtol=1e-6, atol=1e-7)
    gc2 = torch.zeros(D * H * W * C // 8, dtype=torch.float32, device="cuda:0")
    L.check(lib.lb_up2_backward(tskip.data_ptr(), 24, C, D, H, W, gc2.data_ptr(), _stream()))
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
    tout, txin, ttgt = dev(out), dev(xin), dev(tgt)
    scale = np.array([0.5, 2.0, 0.01, 0.02, 0.03, 1.0], np.float32)
    L.check(lib.lb_sur_loss(tout.data_ptr(), txin.data_ptr(), ttgt.data_ptr(), P, scale.ctypes.data_as(ct.c_void_p),
                            0.5, grad.data_ptr(), scratch.data_ptr(), res, _stream()))
    s64 = scale.astype(np.float64)
    pred = xin[:, :6].astype(np.float64) + s64 * out[:, :6]
    Lr, gr = OS.loss(pred, tgt[:, :6].astype(np.float64), xin[:, 6].astype(np.float64), 0.5, s64)
    assert res[3] == pytest.approx(Lr, rel=1e-10)
    # dloss/dout = scale * dloss/dpred
    assert np.allclose(host(grad).reshape(P, 8)[:, :6], gr * s64, rtol=1e-5, atol=1e-9)
    assert np.all(host(grad).reshape(P, 8)[:, 6:] == 0)
    mom = (ct.c_double * 7)()
    L.check(lib.lb_sur_moments(txin.data_ptr(), ttgt.data_ptr(), P, scratch.data_ptr(), mom, _stream()))
    d = (tgt[:, :6].astype(np.float64) - xin[:, :6]) ** 2 * xin[:, 6:7]
    assert np.allclose(np.array(mom[:6]), d.sum(axis=0), rtol=1e-10) and mom[6] == pytest.approx(xin[:, 6].sum())
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
    c["body_force"] = (2e-6, -1e-6, -3e-6)
    p = cases.oracle_params(c)
    lat = Lattice(cases.lattice_params(c, "f64"), c["rho"], c["mat"])
    lat.step(20)
    D, H, W = 10, 14, 24  # larger than the lattice's 8 x 12 x 20 coarse extent
    cf = torch.zeros(D * H * W * 8, dtype=torch.float32, device="cuda:0")
    L.check(lib.lb_sur_restrict(lat._ctx, D, H, W, cf.data_ptr(), None, _stream()))
    run = lbm.Run(c["rho"], c["mat"], p)
    run.step(20)
    ref = OS.restrict(run.f, c["mat"], (D, H, W), p)
    got = host(cf).reshape(D, H, W, 8)
    assert np.abs(got - ref).max() <= 1e-6 * max(1.0, np.abs(ref).max())
    # lift a perturbed canvas and compare the populations (FP64 storage)
    coarse = ref.copy()
    coarse[..., 0] *= 1.0 + 0.01 * RNG.normal(size=coarse.shape[:3])
    coarse[2:4, 3:5, 4:7, 7] = 0.0  # cells without fluid: renormalised stencil and the block fallback
    cc = coarse.astype(np.float32)
    tcc = dev(cc)
    L.check(lib.lb_sur_lift(lat._ctx, tcc.data_ptr(), D, H, W, _stream()))
    _, f2 = lat.export()
    want = OS.lift(cc.astype(np.float64), c["mat"], p)
    fl = (c["mat"] == lbm.FLUID)[None, None]
    assert np.abs(np.where(fl, f2 - want, 0)).max() <= 1e-12
    # a canvas outside the admissible states: negative densities of either
    # component and speeds past the lift's limit in some cells
    bad = ref.copy()
    bad[1:3, 2:5, 3:9, 0] = -0.05
    bad[4:6, 1:3, 10:14, 1] = -0.2
    bad[2:5, 6:9, 2:12, 2] = 0.4
    bad[0:3, 0:4, 12:18, 3:5] = -0.12
    cc = bad.astype(np.float32)
    L.check(lib.lb_sur_lift(lat._ctx, dev(cc).data_ptr(), D, H, W, _stream()))
    _, f3 = lat.export()
    want = OS.lift(cc.astype(np.float64), c["mat"], p)
    assert np.abs(np.where(fl, f3 - want, 0)).max() <= 1e-12
    r = np.where(fl[0, 0], f3.sum(axis=1), 1.0)
    assert np.all(r >= -1e-12) and np.isfinite(f3).all()
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
    # the oracle's forward with its activations stored in BF16 as the
    # network's are (round to nearest even after each ReLU and pooling)
    pred_ref, cache = OS.unet_forward(xv[..., :7], P, ch=ch, act_round=lambda a: bf16_round(a)[0])
    got = host(out).reshape(D, H, W, 8)[..., :6] + xv[..., :6]
    err = np.abs(got - pred_ref).max() / np.abs(pred_ref - xv[..., :6]).max()
    say(f"[gpu] unet forward rel err {err:.2e}")
    assert err < 3e-2
    gy = RNG.normal(size=(D, H, W, 6))
    g8 = np.zeros((D, H, W, 8), np.float32)
    g8[..., :6] = gy
    tg8 = dev(g8.reshape(-1))
    net.zero_grad()
    net.backward(tg8)
    G = OS.unet_backward(gy, P, cache, ch=ch)
    for name, (gw, gb) in G.items():
        ww, bb = net.get_layer_grad(name)
        ww = ww[:, : gw.shape[1], : gw.shape[2]]
        bb = bb[: gb.shape[0]]
        rel = np.linalg.norm(ww - gw) / np.linalg.norm(gw)
        cos = float((ww * gw).sum() / (np.linalg.norm(ww) * np.linalg.norm(gw)))
        say(f"[gpu] grad {name}: rel {rel:.2e} cos {cos:.6f}")
        assert rel < 2e-2 and cos > 0.9998, name
        assert np.linalg.norm(bb - gb) <= 2e-2 * np.linalg.norm(gb) + 1e-6, name


def test_training_beats_persistence_on_lbm_trajectories():
    """The network trained on LBM trajectories with the library's kernels
    predicts a held-out droplet's next snapshot better than persistence."""
    from paper_2607_06794_amd import inputs
    from paper_2607_06794_amd import surrogate as SU
    from paper_2607_06794_amd.sim import Batch, Lattice

    shape = (32, 32, 64)
    D, H, W = 16, 16, 32
    lats = []
    for seed in (5101, 5102, 5103, 5104):
        spec = inputs.CapSpec(shape=shape, footprint=(40.0, 14.0), height=10.0, stripe=(46, 20), seed=seed, noise=1e-2)
        rho, mat = inputs.sessile_cap(spec)
        c = dict(shape=shape, periodic=(True, True, False), G=3.6, tau=(1.0, 1.0), evaporation=True,
                 body_force=(0.0, 0.0, 0.0))
        lats.append(Lattice(cases.lattice_params(c, "f32"), rho, mat))
    batch = Batch(lats)
    xf, xb, healthy = SU.rollout_snapshots(batch, lats, 7, 40, D, H, W, warm=20, rods=False)
    assert healthy.all()
    batch.close()
    for lat in lats:
        lat.close()
    train = [(xf[i, s], xb[i, s], xf[i, s + 1]) for i in range(3) for s in range(6)]
    test = [(xf[3, s], xb[3, s], xf[3, s + 1]) for s in range(6)]
    net = SU.UNet(D, H, W, ch=(16, 16, 32, 32)).init(1)
    before = SU.evaluate(net, test)
    assert before["net"] == pytest.approx(before["persistence"], rel=1e-6)  # zero output layer
    hist = SU.fit(net, train, epochs=40, batch=2, lr=2e-3, lam=1.0, seed=3)
    after = SU.evaluate(net, test)
    say(f"[gpu] surrogate train loss {hist[0]:.3e} -> {hist[-1]:.3e}; test net {after['net']:.3e} "
        f"persistence {after['persistence']:.3e}")
    assert hist[-1] < 0.5 * hist[0]
    assert after["net"] < 0.9 * after["persistence"]


def _min_gap(orods):
    """Smallest axis-segment distance over all rod pairs (minimum image)."""
    from oracle import rods as R

    best = np.inf
    for a in range(orods.n):
        pa, qa = orods.ends(a)
        for b in range(a + 1, orods.n):
            pb, qb = orods.ends(b)
            sh = R.min_image(orods.X[b] - orods.X[a], orods.box, orods.periodic) - (orods.X[b] - orods.X[a])
            best = min(best, R.segment_segment(pa, qa, pb + sh, qb + sh)[0])
    return best


def test_rod_jump_relaxes_overlaps():
    """Three rods placed crossing each other and one touching the wall; a jump
    of zero steps leaves only the relaxation: every axis pair ends at least
    d0 apart, the axis ends d0_wall above the wall, the pair moves are
    symmetric (the mean centre of the crossing pair stays put in x, y), and
    the re-placed lattice steps on healthily."""
    from oracle import rods as R
    from paper_2607_06794_amd import inputs
    from paper_2607_06794_amd import surrogate as SU
    from paper_2607_06794_amd.sim import Lattice

    spec = inputs.CapSpec(shape=(32, 48, 96), footprint=(70.0, 28.0), height=14.0, stripe=(80, 34), seed=5301)
    rho, mat = inputs.sessile_cap(spec)
    s2 = np.sqrt(0.5)
    rods = np.zeros((3, 13))
    rods[0, :3], rods[0, 3:7] = (46.0, 24.0, 8.0), (s2, 0.0, s2, 0.0)  # along x
    rods[1, :3], rods[1, 3:7] = (48.0, 24.5, 9.5), (s2, -s2, 0.0, 0.0)  # along y, 1.5 above rod 0
    rods[2, :3], rods[2, 3:7] = (30.0, 20.0, 4.2), (s2, 0.0, s2, 0.0)  # flat, axis 3.7 above the wall
    c = dict(shape=spec.shape, periodic=(True, True, False), G=3.6, tau=(1.0, 1.0), evaporation=True,
             body_force=(0.0, 0.0, 0.0))
    lp = cases.lattice_params(c, "f32")
    lp.rod_length, lp.rod_radius, lp.wall_z = 12.0, 2.0, 0.5
    lp.rod_d0, lp.rod_d0_wall = 5.0, 4.0
    say("[gpu] rod relaxation: 3 rods, shape", spec.shape)
    lat = Lattice(lp, rho, mat, rods=rods)
    D, H, W = 16, 24, 48
    now_f, _ = SU.restrict(lat, D, H, W)
    before = lat.rods()
    SU.jump_rods(lat, now_f, now_f, D, H, W, 0)
    SU.lift(lat, now_f, D, H, W)
    after = lat.rods()
    assert np.abs(after[:, 3:7] - before[:, 3:7]).max() == 0.0
    rp = R.RodParams(length=12.0, radius=2.0)
    orods = R.Rods(after[:, :3], after[:, 3:7], after[:, 7:10], after[:, 10:13], rp, (96, 48, 32), (True, True, False))
    assert _min_gap(orods) >= 5.0 - 1e-5
    assert _min_gap(orods) <= 5.0 + 1e-3  # moved no further than needed
    low = min(orods.ends(2)[0][2], orods.ends(2)[1][2])
    assert low - 0.5 >= 4.0 - 1e-5
    assert np.allclose(after[0, :2] + after[1, :2], before[0, :2] + before[1, :2], atol=1e-9)
    assert after[0, 2] < before[0, 2] and after[1, 2] > before[1, 2]  # pushed apart along z
    want = (orods.mask(spec.shape) >= 0).sum(axis=0)
    assert np.array_equal(lat.rod_map(), want)
    lat.coupled_step(20)
    assert lat.observables(allow_unstable=True)["status"] == 0
    lat.close()


def test_rod_jump_moves_and_replaces_rods():
    """A jump moves every rod centre by steps x the mean coarse velocity and
    re-places the rods: the rod nodes afterwards are exactly the capsules at
    the new poses (oracle mask), and the lattice stays healthy."""
    import torch

    from oracle import rods as R
    from paper_2607_06794_amd import inputs
    from paper_2607_06794_amd import surrogate as SU
    from paper_2607_06794_amd.sim import Lattice

    spec = inputs.CapSpec(shape=(32, 48, 96), footprint=(70.0, 28.0), height=14.0, stripe=(80, 34), seed=5201)
    rho, mat = inputs.sessile_cap(spec)
    rods = inputs.place_rods(4, 12.0, 2.0, (96, 48, 32), inside=inputs.cap_inside(spec), seed=5202, margin=1.0,
                             max_trials=20000)
    assert len(rods) >= 2
    c = dict(shape=spec.shape, periodic=(True, True, False), G=3.6, tau=(1.0, 1.0), evaporation=True,
             body_force=(0.0, 0.0, 0.0))
    lp = cases.lattice_params(c, "f32")
    lp.rod_length, lp.rod_radius, lp.wall_z = 12.0, 2.0, 0.5
    lat = Lattice(lp, rho, mat, rods=rods)
    lat.coupled_step(10)
    D, H, W = 16, 24, 48
    now_f, _ = SU.restrict(lat, D, H, W)
    nxt = now_f.clone()
    v = torch.zeros(8, device="cuda:0")
    v[2], v[3], v[4] = 0.004, -0.002, 0.0005
    nxt.view(-1, 8).add_(v)  # a uniform velocity change of the predicted canvas
    before = lat.rods()
    SU.jump_rods(lat, now_f, nxt, D, H, W, 500)
    SU.lift(lat, nxt, D, H, W)
    after = lat.rods()
    # each centre moved by 500 x its new velocity (the mean of the two
    # canvases), up to the relaxation of overlaps the move made
    rp = R.RodParams(length=12.0, radius=2.0)
    for r in range(len(before)):
        d = after[r, :3] - before[r, :3]
        d[0] -= 96 * np.round(d[0] / 96)
        d[1] -= 48 * np.round(d[1] / 48)
        assert np.abs(d[:2] - 500 * after[r, 7:9]).max() < 0.5
    assert np.abs(after[:, 3:7] - before[:, 3:7]).max() == 0.0  # orientation kept
    orods = R.Rods(after[:, :3], after[:, 3:7], after[:, 7:10], after[:, 10:13], rp, (96, 48, 32), (True, True, False))
    assert _min_gap(orods) >= lp.rod_d0 - 1e-5
    want = (orods.mask(spec.shape) >= 0).sum(axis=0)
    assert np.array_equal(lat.rod_map(), want)
    lat.coupled_step(20)
    o = lat.observables(allow_unstable=True)
    assert o["status"] == 0
    lat.close()


def test_rod_drift_continues_the_previous_displacement():
    """lb_sur_drift_rods: with the centres of one interval earlier given as
    the present ones shifted by (1.2, -0.6, 0), each rod has moved by
    (-1.2, 0.6, 0) since then and moves by half of that again, (-0.6, 0.3,
    0) with the periodic wrap, orientation and velocity kept; the rod map is the oracle's mask of the new poses, and the
    lattice steps on healthily after the lift."""
    import torch

    from oracle import rods as R
    from paper_2607_06794_amd import inputs
    from paper_2607_06794_amd import surrogate as SU
    from paper_2607_06794_amd.sim import Lattice

    spec = inputs.CapSpec(shape=(32, 48, 96), footprint=(70.0, 28.0), height=14.0, stripe=(80, 34), seed=5201)
    rho, mat = inputs.sessile_cap(spec)
    rods = inputs.place_rods(4, 12.0, 2.0, (96, 48, 32), inside=inputs.cap_inside(spec), seed=5202, margin=1.0,
                             max_trials=20000)
    assert len(rods) >= 2
    c = dict(shape=spec.shape, periodic=(True, True, False), G=3.6, tau=(1.0, 1.0), evaporation=True,
             body_force=(0.0, 0.0, 0.0))
    lp = cases.lattice_params(c, "f32")
    lp.rod_length, lp.rod_radius, lp.wall_z = 12.0, 2.0, 0.5
    lat = Lattice(lp, rho, mat, rods=rods)
    lat.coupled_step(10)
    say(f"[gpu] rod drift: {len(rods)} rods on {spec.shape}")
    before = lat.rods()
    prev = before[:, :3] - np.array([-1.2, 0.6, 0.0])
    prev[:, 0] %= 96  # the earlier centres as the lattice stores them (wrapped)
    prev[:, 1] %= 48
    SU.drift_rods(lat, torch.from_numpy(np.ascontiguousarray(prev)).to("cuda:0"), 0.5)
    D, H, W = 16, 24, 48
    now_f, _ = SU.restrict(lat, D, H, W)
    SU.lift(lat, now_f, D, H, W)
    after = lat.rods()
    want_x = before[:, :3] + np.array([-0.6, 0.3, 0.0])
    want_x[:, 0] %= 96
    want_x[:, 1] %= 48
    # z stays, kept between the closed end planes as every jump keeps it
    for r in range(len(before)):
        ez = abs(R.axis(before[r, 3:7])[2]) * 6.0 + 2.0
        want_x[r, 2] = min(max(want_x[r, 2], 1.5 + ez), 32 - 2.5 - ez)
    assert np.abs(after[:, :3] - want_x).max() < 1e-12
    assert np.array_equal(after[:, 3:13], before[:, 3:13])  # orientation, velocity, angular momentum kept
    rp = R.RodParams(length=12.0, radius=2.0)
    orods = R.Rods(after[:, :3], after[:, 3:7], after[:, 7:10], after[:, 10:13], rp, (96, 48, 32), (True, True, False))
    assert np.array_equal(lat.rod_map(), (orods.mask(spec.shape) >= 0).sum(axis=0))
    with pytest.raises(Exception):
        SU.drift_rods(lat, torch.from_numpy(np.ascontiguousarray(prev)).to("cuda:0"), float("nan"))
    lat.coupled_step(20)
    assert lat.observables(allow_unstable=True)["status"] == 0
    lat.close()


def test_surrogate_advance_and_fallback():
    """A network that keeps the state (zero output) passes a loose mass check:
    the surrogate path runs (jump, lift, K steps).  A network whose output adds
    0.2 to rho_A everywhere fails the 0.5 % check: the lattice goes back to its
    state before the jump and runs the plain interval, bit-identical to a twin
    lattice that never tried the jump."""
    from paper_2607_06794_amd import inputs
    from paper_2607_06794_amd import surrogate as SU
    from paper_2607_06794_amd.sim import Lattice

    spec = inputs.CapSpec(shape=(32, 48, 96), footprint=(70.0, 28.0), height=14.0, stripe=(80, 34), seed=5401)
    rho, mat = inputs.sessile_cap(spec)
    rods = inputs.place_rods(4, 12.0, 2.0, (96, 48, 32), inside=inputs.cap_inside(spec), seed=5402, margin=1.0,
                             max_trials=20000)
    c = dict(shape=spec.shape, periodic=(True, True, False), G=3.6, tau=(1.0, 1.0), evaporation=True,
             body_force=(0.0, 0.0, 0.0))

    def make():
        lp = cases.lattice_params(c, "f32")
        lp.rod_length, lp.rod_radius, lp.wall_z = 12.0, 2.0, 0.5
        lat = Lattice(lp, rho, mat, rods=rods)
        lat.coupled_step(10)
        return lat

    D, H, W = 16, 24, 48
    say(f"[gpu] surrogate advance: shape {spec.shape}, {len(rods)} rods")
    keep = SU.UNet(D, H, W, ch=(8, 16, 16, 16)).init(0)
    lat = make()
    r = SU.advance(lat, keep, D, H, W, interval=40, K=10, rate=0.0, threshold=1.0)
    say(f"[gpu] persistence jump: mass error {r['mass_error']:.3e}")
    assert r["surrogate"] and r["mass_error"] < 0.05
    assert lat.observables(allow_unstable=True)["status"] == 0
    lat.close()
    bad = SU.UNet(D, H, W, ch=(8, 16, 16, 16)).init(0)
    bad.set_layer("out", np.zeros((27, 8, 6)), np.array([0.2, 0, 0, 0, 0, 0]))
    lat, twin = make(), make()
    r = SU.advance(lat, bad, D, H, W, interval=40, K=10, rate=0.0, threshold=0.005)
    assert not r["surrogate"] and r["mass_error"] > 0.005
    twin.coupled_step(40)
    _, fa = lat.export()
    _, fb = twin.export()
    assert np.array_equal(fa, fb) and np.array_equal(lat.rods(), twin.rods())
    oa, ob = lat.observables(), twin.observables()
    assert np.array_equal(oa["ledger"], ob["ledger"]) and np.array_equal(oa["solid"], ob["solid"])
    # a snapshot goes back only into its own lattice: the workspace it holds
    # carries the device addresses of that lattice's buffers
    with pytest.raises(ValueError):
        twin.restore(lat.snapshot())
    lat.close()
    twin.close()
