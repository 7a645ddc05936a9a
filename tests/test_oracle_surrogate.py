"""Pins of the surrogate oracle: brute force, library convolution and autograd
(PyTorch CPU, FP64), finite differences, adjoint identities, closed forms."""
import numpy as np
import pytest
import torch

from oracle import lbm
from oracle import surrogate as S

RNG = np.random.default_rng(7007)


def _torch_conv(x, w, b):
    """Independent library check: torch.nn.functional.conv3d in FP64 on the CPU."""
    xt = torch.from_numpy(np.ascontiguousarray(np.moveaxis(x, -1, 0)[None]))
    wt = torch.from_numpy(np.ascontiguousarray(w.reshape(3, 3, 3, w.shape[1], w.shape[2]).transpose(4, 3, 0, 1, 2)))
    y = torch.nn.functional.conv3d(xt, wt, torch.from_numpy(b), padding=1)
    return np.moveaxis(y[0].numpy(), 0, -1)


def test_conv_matches_direct_loops_and_torch():
    x = RNG.normal(size=(3, 4, 5, 2))
    w = RNG.normal(size=(27, 2, 3))
    b = RNG.normal(size=3)
    y = S.conv3d(x, w, b)
    assert np.allclose(y, S.conv3d_direct(x, w, b), rtol=0, atol=1e-12)
    x2 = RNG.normal(size=(6, 5, 7, 4))
    w2 = RNG.normal(size=(27, 4, 5))
    b2 = RNG.normal(size=5)
    assert np.allclose(S.conv3d(x2, w2, b2), _torch_conv(x2, w2, b2), rtol=0, atol=1e-12)


def test_centre_tap_is_a_matmul():
    x = RNG.normal(size=(4, 3, 5, 6))
    w = np.zeros((27, 6, 4))
    w[13] = RNG.normal(size=(6, 4))  # tap (0, 0, 0)
    assert np.allclose(S.conv3d(x, w), x @ w[13], rtol=0, atol=1e-13)


def test_conv_gradients_finite_differences():
    x = RNG.normal(size=(3, 3, 4, 2))
    w = RNG.normal(size=(27, 2, 3))
    r = RNG.normal(size=(3, 3, 4, 3))
    f = lambda xx, ww: float((S.conv3d(xx, ww) * r).sum())
    dx = S.conv3d_dgrad(r, w)
    dw, db = S.conv3d_wgrad(x, r)
    h = 1e-6
    for _ in range(12):
        i = tuple(RNG.integers(0, n) for n in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        assert (f(xp, w) - f(xm, w)) / (2 * h) == pytest.approx(dx[i], rel=1e-6, abs=1e-8)
        j = tuple(RNG.integers(0, n) for n in w.shape)
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        assert (f(x, wp) - f(x, wm)) / (2 * h) == pytest.approx(dw[j], rel=1e-6, abs=1e-8)
    assert np.allclose(db, r.reshape(-1, 3).sum(axis=0))


def test_pool_and_upsample_adjoints():
    x = RNG.normal(size=(4, 6, 8, 3))
    y = RNG.normal(size=(2, 3, 4, 3))
    assert (S.pool2(x) * y).sum() == pytest.approx((x * S.pool2_back(y)).sum(), rel=1e-13)
    assert (S.up2(y) * x).sum() == pytest.approx((y * S.up2_back(x)).sum(), rel=1e-13)
    assert np.allclose(S.pool2(S.up2(y)), y)


def _torch_unet(P, ch):
    """The same U-Net written with torch modules (FP64, CPU) for autograd."""
    import torch.nn.functional as F

    params = {k: (torch.tensor(w, requires_grad=True), torch.tensor(b, requires_grad=True)) for k, (w, b) in P.items()}

    def conv(h, name):
        w, b = params[name]
        wt = w.reshape(3, 3, 3, w.shape[1], w.shape[2]).permute(4, 3, 0, 1, 2)
        return F.conv3d(h, wt, b, padding=1)

    def run(x):
        h = x
        skips = []
        for lvl in range(len(ch)):
            h = F.relu(conv(h, f"enc{lvl}a"))
            h = F.relu(conv(h, f"enc{lvl}b"))
            if lvl < len(ch) - 1:
                skips.append(h)
                h = F.avg_pool3d(h, 2)
        for lvl in range(len(ch) - 2, -1, -1):
            h = torch.cat([F.interpolate(h, scale_factor=2, mode="nearest"), skips[lvl]], dim=1)
            h = F.relu(conv(h, f"dec{lvl}a"))
            h = F.relu(conv(h, f"dec{lvl}b"))
        return x[:, : S.OUT_CH] + conv(h, "out")

    return params, run


def test_unet_gradients_match_torch_autograd():
    ch = (4, 6, 8, 8)
    P = S.init_params(11, ch=ch)
    P["out"] = (RNG.normal(size=P["out"][0].shape) * 0.1, RNG.normal(size=6) * 0.1)
    x = RNG.normal(size=(8, 8, 16, S.IN_CH))
    pred, cache = S.unet_forward(x, P, ch=ch)
    gy = RNG.normal(size=pred.shape)
    G = S.unet_backward(gy, P, cache, ch=ch)
    params, run = _torch_unet(P, ch)
    xt = torch.from_numpy(np.ascontiguousarray(np.moveaxis(x, -1, 0)[None]))
    yt = run(xt)
    assert np.allclose(np.moveaxis(yt[0].detach().numpy(), 0, -1), pred, rtol=0, atol=1e-11)
    (yt * torch.from_numpy(np.ascontiguousarray(np.moveaxis(gy, -1, 0)[None]))).sum().backward()
    for name, (gw, gb) in G.items():
        assert np.allclose(gw, params[name][0].grad.numpy(), rtol=1e-9, atol=1e-11), name
        assert np.allclose(gb, params[name][1].grad.numpy(), rtol=1e-9, atol=1e-11), name


def test_untrained_network_is_persistence_and_param_count():
    P = S.init_params(3)
    x = RNG.normal(size=(8, 8, 8, S.IN_CH))
    small = S.init_params(3, ch=(4, 6, 8, 8))
    pred, _ = S.unet_forward(x, small, ch=(4, 6, 8, 8))
    assert np.array_equal(pred, x[..., :6])
    n = sum(w.size + b.size for w, b in P.values())
    assert 3.0e6 < n < 4.0e6  # the 32-64-128-128 network: about 3.5 M parameters


def test_loss_gradient_finite_differences():
    pred = RNG.normal(size=(2, 3, 4, 6)) + 1.0
    tgt = RNG.normal(size=(2, 3, 4, 6)) + 1.0
    mask = (RNG.uniform(size=(2, 3, 4)) > 0.3).astype(float)
    scale = np.array([0.5, 2.0, 0.01, 0.02, 0.03, 1.0])
    for sc in (None, scale):
        L, g = S.loss(pred, tgt, mask, 0.7, sc)
        h = 1e-4  # the loss is quadratic: central differences are exact up to rounding
        for _ in range(10):
            i = tuple(RNG.integers(0, n) for n in pred.shape)
            p1, p2 = pred.copy(), pred.copy()
            p1[i] += h
            p2[i] -= h
            fd = (S.loss(p1, tgt, mask, 0.7, sc)[0] - S.loss(p2, tgt, mask, 0.7, sc)[0]) / (2 * h)
            assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-7)
    # unit scale is the plain masked MSE
    diff = (pred - tgt) * mask[..., None]
    me = (mask * (pred[..., 0] - tgt[..., 0])).sum() / (mask * tgt[..., 0]).sum()
    assert S.loss(pred, tgt, mask, 0.7)[0] == pytest.approx((diff ** 2).sum() / (6 * mask.sum()) + 0.7 * me ** 2,
                                                            rel=1e-13)


def test_adam_first_step_is_signed_lr():
    p = RNG.normal(size=10)
    g = RNG.normal(size=10)
    p1, m, v = S.adam(p, g, np.zeros(10), np.zeros(10), 1, lr=0.01)
    # m_hat / sqrt(v_hat) = g / (|g| + eps): the sign up to eps / |g|
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1e-6)


def test_restrict_uniform_state_and_rod_fraction():
    shape = (6, 8, 10)
    rho = np.zeros((2,) + shape)
    rho[0], rho[1] = 0.7, 0.2
    f = lbm.initial_state(rho)
    mat = np.zeros(shape, np.uint8)
    mat[0:2, 0:2, 0:2] = lbm.ROD  # one whole block of rod nodes
    mat[2, 2, 2] = lbm.ROD  # one node of another block
    f[:, :, mat != 0] = 0.0
    c = S.restrict(f, mat, (4, 6, 8), lbm.Params(shape=shape, G=0.0))
    inside = c[:3, :4, :5]
    assert np.allclose(inside[..., 6], 1.0) and np.allclose(c[3:, ..., 6], 0.0) and np.allclose(c[:, 4:, :, 6], 0)
    assert np.allclose(c[3:, ..., 0], S.GAS[0]) and np.allclose(c[3:, ..., 1], S.GAS[1])
    assert c[0, 0, 0, 5] == 1.0 and c[1, 1, 1, 5] == 1.0 / 8.0
    assert c[0, 0, 0, 0] == 0.0 and c[0, 0, 0, 7] == 0.0  # no fluid node in the block
    assert c[1, 1, 1, 7] == 7.0 / 8.0 and np.allclose(c[3:, ..., 7], 0.0)
    assert np.allclose(inside[1:, 1:, 1:, 0], 0.7) and np.allclose(inside[..., 2:5], 0.0, atol=1e-15)


def test_prolong_reproduces_linear_fields_and_lift_moments():
    shape = (8, 10, 12)
    cz, cy, cx = 4, 5, 6
    zz, yy, xx = np.meshgrid(np.arange(cz), np.arange(cy), np.arange(cx), indexing="ij")
    coarse = np.zeros((cz, cy, cx, 8))
    coarse[..., 7] = 1.0  # every cell holds fluid
    for ch, (a, b, c, d) in enumerate([(0.5, 0.01, 0.02, 0.03), (0.3, -0.01, 0.0, 0.02), (0.0, 0.001, 0.0, 0.0),
                                       (0.01, 0.0, 0.002, 0.0), (0.0, 0.0, 0.0, 0.001)]):
        coarse[..., ch] = a + b * xx + c * yy + d * zz
    mat = np.zeros(shape, np.uint8)
    rho, u = S.prolong(coarse, mat)
    # interior fine nodes (not clamped): the coarse linear function at x/2 - 1/4
    z, y, x = 3, 4, 5
    X, Y, Z = x / 2 - 0.25, y / 2 - 0.25, z / 2 - 0.25
    assert rho[0, z, y, x] == pytest.approx(0.5 + 0.01 * X + 0.02 * Y + 0.03 * Z, rel=1e-13)
    assert u[1, z, y, x] == pytest.approx(0.01 + 0.002 * Y, rel=1e-13)
    # cells without fluid take no part: the rest of the stencil is renormalised,
    # and a node whose 8 corner cells hold none takes the mean of the
    # fluid-holding cells around them
    holed = coarse.copy()
    holed[1, 1, 1, 7] = 0.0
    holed[1, 1, 1, :5] = 99.0  # would show up if used
    rho_h, _ = S.prolong(holed, mat)
    assert np.all(rho_h[0] < 10)
    # fine node (3, 3, 3) -> coarse 1.25 per axis: corners 1 and 2, weights 3/4 and 1/4
    w = np.array([0.75, 0.25])
    wts = np.einsum("i,j,k->ijk", w, w, w)
    wts[0, 0, 0] = 0.0
    vals = coarse[1:3, 1:3, 1:3, 0]
    assert rho_h[0, 3, 3, 3] == pytest.approx((wts * vals).sum() / wts.sum(), rel=1e-13)
    dead = coarse.copy()
    dead[0:3, 0:3, 0:3, 7] = 0.0
    rho_d, _ = S.prolong(dead, mat)
    # node (1, 1, 1) -> coarse 0.25: corners 0, 1 and the block 0..2 hold no fluid: gas
    assert rho_d[0, 1, 1, 1] == S.GAS[0]
    # node (3, 3, 3) -> coarse 1.25: corners 1, 2 hold none; the block 0..3 has
    # fluid in the cells with an index 3: their plain mean
    cells = [coarse[iz, iy, ix, 0] for iz in range(4) for iy in range(4) for ix in range(4) if max(iz, iy, ix) == 3]
    assert rho_d[0, 3, 3, 3] == pytest.approx(np.mean(cells), rel=1e-13)
    # without forces the lifted state is the plain equilibrium of the fields
    f = S.lift(coarse, mat, lbm.Params(shape=shape, G=0.0))
    r0 = f[0].sum(axis=0)
    assert np.allclose(r0, rho[0], rtol=1e-13)
    j = np.einsum("izyx,id->dzyx", f[0], lbm.C.astype(float))
    assert np.allclose(j, rho[0][None] * u, rtol=1e-12, atol=1e-15)


def test_lift_maps_a_canvas_onto_admissible_states():
    # a uniform canvas with a negative rho_A and a speed of sqrt(0.1) on a
    # periodic fluid box: prolongation keeps it uniform and a uniform psi
    # exerts no force, so the lifted state is the plain equilibrium of
    # rho = (0, 1) moving at 0.15 in the canvas's direction (3, 1, 0)
    shape = (6, 8, 10)
    coarse = np.zeros((3, 4, 5, 8))
    coarse[..., 0], coarse[..., 1] = -0.1, 1.0
    coarse[..., 2], coarse[..., 3] = 0.3, 0.1
    coarse[..., 6], coarse[..., 7] = 1.0, 1.0
    mat = np.zeros(shape, np.uint8)
    f = S.lift(coarse, mat, lbm.Params(shape=shape, G=3.6))
    assert np.all(f[0] == 0.0)
    assert np.allclose(f[1].sum(axis=0), 1.0, rtol=0, atol=1e-15)
    j = np.einsum("izyx,id->dzyx", f[1], lbm.C.astype(float))
    want = 0.15 * np.array([3.0, 1.0, 0.0]) / np.sqrt(10.0)
    assert np.allclose(j, want[:, None, None, None], rtol=0, atol=1e-15)
    pxx = np.einsum("izyx,i->zyx", f[1], lbm.C[:, 0].astype(float) ** 2)
    assert np.allclose(pxx, 1.0 / 3.0 + want[0] ** 2, rtol=0, atol=1e-15)
    # below the limits the map leaves a canvas alone
    coarse[..., 0], coarse[..., 2] = 0.05, 0.1
    f = S.lift(coarse, mat, lbm.Params(shape=shape, G=3.6))
    assert np.allclose(f[0].sum(axis=0), 0.05, rtol=1e-14)
    j = np.einsum("izyx,id->dzyx", f[0] + f[1], lbm.C.astype(float))
    assert np.allclose(j[0], 1.05 * 0.1, rtol=1e-13) and np.allclose(j[1], 1.05 * 0.1, rtol=1e-13)


def _two_phase(shape, seed):
    """A sessile cap of A in B on a patterned wall under a reservoir, with a body force."""
    from tests import cases

    c = cases.cap_case(shape=shape, footprint=(9.0, 6.0), height=4.0, stripe=(8, 5), seed=seed)
    c["body_force"] = (2e-6, -1e-6, -3e-6)
    return c["rho"], c["mat"], cases.oracle_params(c)


def test_restrict_velocity_is_the_physical_velocity_of_the_collision():
    # the stored state after a step is the collision output of moments (rho,
    # j) under the Shan-Chen force F; the canvas velocity must be the block
    # mean of the physical velocity (j + F/2) / rho of that collision,
    # although restriction sees only f* (a dropped or flipped F/2 fails)
    shape = (10, 12, 14)
    rho, mat, p = _two_phase(shape, 71)
    run = lbm.Run(rho, mat, p).step(4)
    fn, _, d = lbm.fluid_step(run.f, mat, p)
    c = S.restrict(fn, mat, (5, 6, 7), p)
    fl = mat == lbm.FLUID
    mom = np.where(fl, d["j"][0] + d["j"][1] + 0.5 * (d["F"][0] + d["F"][1]), 0.0)
    tot = np.where(fl, d["rho"][0] + d["rho"][1], 0.0)
    blk = lambda a: a.reshape(a.shape[:-3] + (5, 2, 6, 2, 7, 2)).sum(axis=(-5, -3, -1))
    want = blk(mom) / np.where(blk(tot) > 0, blk(tot), 1.0)
    has = blk(fl.astype(float)) > 0
    got = c[..., 2:5].transpose(3, 0, 1, 2)
    assert np.allclose(np.where(has, got, 0), np.where(has, want, 0), rtol=1e-12, atol=1e-14)
    # the force term matters here: the post-collision momentum alone is off
    jpost = sum(np.einsum("izyx,id->dzyx", fn[k], lbm.C.astype(float)) for k in range(2))
    naive = blk(np.where(fl, jpost, 0.0)) / np.where(blk(tot) > 0, blk(tot), 1.0)
    assert np.abs(np.where(has, naive - want, 0)).max() > 100 * np.abs(np.where(has, want, 0)).max() * 1e-3


def test_lift_is_the_collision_output_of_the_prolonged_fields():
    # node by node the lifted state carries the prolonged densities, and its
    # physical velocity (j* - F/2) / rho under the force of those densities
    # is the prolonged velocity
    shape = (10, 12, 14)
    rho, mat, p = _two_phase(shape, 72)
    run = lbm.Run(rho, mat, p).step(3)
    coarse = S.restrict(run.f, mat, (5, 6, 7), p)
    coarse[..., 2] += 0.01  # a drift on top
    f = S.lift(coarse, mat, p)
    rp, up = S.prolong(coarse, mat)
    fl = mat == lbm.FLUID
    r = f.sum(axis=1)
    assert np.allclose(np.where(fl, r, 0), np.where(fl, rp, 0), rtol=1e-13, atol=0)
    F = lbm.sc_force(lbm.pseudopotential(r, mat, p), r, p)
    j = sum(np.einsum("izyx,id->dzyx", f[k], lbm.C.astype(float)) for k in range(2))
    u = (j - 0.5 * (F[0] + F[1])) / np.where(fl, r[0] + r[1], 1.0)
    assert np.allclose(np.where(fl, u, 0), np.where(fl, up, 0), rtol=1e-12, atol=1e-14)
    # and each component is the equilibrium of its shifted velocity: its
    # second moment is rho_k (c_s^2 + u_k u_k) along every axis
    for k in range(2):
        jk = np.einsum("izyx,id->dzyx", f[k], lbm.C.astype(float))
        uk = jk / np.where(fl, r[k], 1.0)
        pxx = np.einsum("izyx,i->zyx", f[k], lbm.C[:, 0].astype(float) ** 2)
        assert np.allclose(np.where(fl, pxx, 0), np.where(fl, r[k] * (1 / 3 + uk[0] ** 2), 0), rtol=1e-12, atol=1e-14)


def test_lift_keeps_each_components_canvas_mass():
    # a two-phase canvas pushed negative in a block of cells (the admissible
    # map raises those to 0, which adds mass): the lifted populations still
    # carry each component's canvas mass, the sum over the cells of rho_k x
    # 8 x the fluid fraction, while the map alone would not
    shape = (10, 12, 14)
    rho, mat, p = _two_phase(shape, 73)
    run = lbm.Run(rho, mat, p).step(3)
    coarse = S.restrict(run.f, mat, (5, 6, 7), p)
    coarse[1:3, 2:4, 1:4, 0] = -0.05
    f = S.lift(coarse, mat, p)
    fl = mat == lbm.FLUID
    for k in range(2):
        want = float((coarse[..., k] * 8.0 * coarse[..., 7]).sum())
        got = float(f[k].sum(axis=0)[fl].sum())
        assert got == pytest.approx(want, rel=1e-12)
    r_adm, _ = S.admissible(*S.prolong(coarse, mat))
    assert r_adm[0][fl].sum() > 1.001 * float((coarse[..., 0] * 8.0 * coarse[..., 7]).sum())
