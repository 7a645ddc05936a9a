"""Learned surrogate: a 3-D convolutional U-Net on the coarse canvas, trained
and run with the library's own kernels (BF16 matrix-core convolutions with
FP32 accumulation, pooling and gradient plumbing, the loss and Adam).

This module only allocates device buffers (PyTorch tensors), describes them
to the library (lb_unet) and sequences the C-ABI calls; every arithmetic step
runs in liblbm.so, the whole network's forward and backward passes in one call
each (lb_sur_forward, lb_sur_backward).

Network (four levels, 32-64-128-128 channels): per level two 3x3x3 ReLU
convolutions; 2x2x2 average pooling down; on the way up nearest-neighbour
upsampling concatenated with the skip (read in place by the convolution),
two ReLU convolutions; a final linear 3x3x3 convolution to the six predicted
channels, added to the input channels (residual).  Canvas tensors are
[D][H][W][8] channels-last; the input's 7 channels are rho_A, rho_B, u_x, u_y,
u_z, rod fraction, mask (+1 zero channel), the output's 6 the same minus the
mask (+2 zero channels).
"""
from __future__ import annotations

import ctypes as ct

import numpy as np

from . import _lib

CH = (32, 64, 128, 128)
CIN, COUT = 8, 8  # padded input / output channel counts (7 and 6 used)


def layer_shapes(ch=CH):
    """(name, c1, c2, cout, up1, level) of every convolution in forward order."""
    L = []
    c = CIN
    for lvl, co in enumerate(ch):
        L.append((f"enc{lvl}a", c, 0, co, 0, lvl))
        L.append((f"enc{lvl}b", co, 0, co, 0, lvl))
        c = co
    for lvl in range(len(ch) - 2, -1, -1):
        L.append((f"dec{lvl}a", c, ch[lvl], ch[lvl], 1, lvl))
        L.append((f"dec{lvl}b", ch[lvl], 0, ch[lvl], 0, lvl))
        c = ch[lvl]
    L.append(("out", c, 0, COUT, 0, 0))
    return L


def _p(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


class UNet:
    def __init__(self, D=32, H=64, W=128, ch=CH, device="cuda:0", stream=None):
        import torch

        self.torch = torch
        self.lib = _lib.load()
        self.D, self.H, self.W, self.ch = D, H, W, tuple(ch)
        nlev = len(self.ch)
        if any(n % (1 << (nlev - 1)) for n in (D, H, W)):
            raise ValueError(f"canvas {D}x{H}x{W} must be divisible by {1 << (nlev - 1)}")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.layers = layer_shapes(self.ch)
        # flat FP32 master parameters (w then b per layer), BF16 copy, grads, moments
        self.off = {}
        n = 0
        for name, c1, c2, co, _, _ in self.layers:
            nw = 27 * (c1 + c2) * co
            self.off[name] = (n, nw, n + nw, co)
            n += nw + co
            n = (n + 7) // 8 * 8  # keep every block 16-byte aligned
        self.nparam = n
        f32 = dict(dtype=torch.float32, device=self.device)
        self.p = torch.zeros(n, **f32)
        self.g = torch.zeros(n, **f32)
        self.m = torch.zeros(n, **f32)
        self.v = torch.zeros(n, **f32)
        self.pb = torch.zeros(n, dtype=torch.int16, device=self.device)
        self.pt = torch.zeros(n, dtype=torch.int16, device=self.device)  # weights packed for the forward
        self.step_count = 0
        # activations (BF16) and gradients (FP32) per level
        self.P = [(D >> l) * (H >> l) * (W >> l) for l in range(nlev)]
        bf = dict(dtype=torch.int16, device=self.device)
        self.act = {}
        for name, c1, c2, co, _, lvl in self.layers[:-1]:
            self.act[name] = torch.zeros(self.P[lvl] * co, **bf)
        self.pooled = [torch.zeros(self.P[l + 1] * self.ch[l], **bf) for l in range(nlev - 1)]
        self.out = torch.zeros(self.P[0] * COUT, **f32)
        cmax = [max(self.ch[l] + (self.ch[l + 1] if l + 1 < nlev else 0), self.ch[l]) for l in range(nlev)]
        self.gA = [torch.zeros(self.P[l] * max(cmax[l], CIN, self.ch[-1] * 2), **f32) for l in range(nlev)]
        self.gB = [torch.zeros(self.P[l] * max(self.ch), **f32) for l in range(nlev)]
        self.gcat = [torch.zeros(self.P[l] * (self.ch[l] + (self.ch[l + 1] if l + 1 < nlev - 1 else self.ch[-1])), **f32)
                     for l in range(nlev - 1)]
        self.loss_scratch = torch.zeros(self.lib.lb_sur_loss_scratch_bytes() // 4 + 64, **f32)
        # BF16 pre-activation gradient of the layer being differentiated
        self.gm = torch.zeros(max(self.P[lvl] * co for _, _, _, co, _, lvl in self.layers), **bf)
        # FP32 scratch for the split-K forward of the coarse levels
        self.acc = torch.zeros(max(self.P[lvl] * co for _, _, _, co, _, lvl in self.layers if lvl >= 1), **f32)
        # output scale per channel (the network predicts changes in these units)
        self.scale = np.ones(6, np.float32)
        # input normalisation: lattice velocities are O(1e-3 .. 1e-2) next to
        # O(1) densities and fractions, so they enter the network scaled by 100
        self.in_shift = np.zeros(8, np.float32)
        self.in_gain = np.array([1, 1, 100, 100, 100, 1, 1, 1], np.float32)
        self.xin = torch.zeros(self.P[0] * CIN, **bf)
        self.desc = self._descriptor()

    def _descriptor(self):
        """The library's description of this network's buffers (lb_unet)."""
        d = _lib.LbUnet()
        d.D, d.H, d.W, d.nlev, d.cin, d.cout = self.D, self.H, self.W, len(self.ch), CIN, COUT
        for l, c in enumerate(self.ch):
            d.ch[l] = c
        d.p, d.g, d.pb, d.pt = self.p.data_ptr(), self.g.data_ptr(), self.pb.data_ptr(), self.pt.data_ptr()
        for L, (name, *_rest) in enumerate(self.layers):
            o, _, ob, _ = self.off[name]
            d.off_w[L], d.off_b[L] = o, ob
            if name != "out":
                d.act[L] = self.act[name].data_ptr()
        for l in range(len(self.ch)):
            d.gA[l], d.gB[l] = self.gA[l].data_ptr(), self.gB[l].data_ptr()
            if l < len(self.ch) - 1:
                d.pooled[l], d.gcat[l] = self.pooled[l].data_ptr(), self.gcat[l].data_ptr()
        d.out, d.gm, d.acc = self.out.data_ptr(), self.gm.data_ptr(), self.acc.data_ptr()
        return d

    def set_scale(self, scale):
        self.scale = np.ascontiguousarray(scale, dtype=np.float32).reshape(6)

    def prepare(self, x_f32):
        """The normalised BF16 network input of an FP32 canvas (kept in self.xin)."""
        _lib.check(self.lib.lb_sur_normalize(_p(x_f32), self.P[0], self.in_shift.ctypes.data_as(ct.c_void_p),
                                             self.in_gain.ctypes.data_as(ct.c_void_p), _p(self.xin), self._s()))
        return self.xin

    # ------------------------------------------------------------------ params
    def _s(self):
        return ct.c_void_p(self.stream.cuda_stream)

    def init(self, seed=0):
        """He-normal weights (std sqrt(2 / (27 Cin))) from a seeded generator, zero
        biases, a zero output layer (the untrained network is persistence)."""
        rng = np.random.Generator(np.random.PCG64(seed))
        host = np.zeros(self.nparam, np.float32)
        for name, c1, c2, co, _, _ in self.layers:
            o, nw, ob, _ = self.off[name]
            if name != "out":
                host[o:o + nw] = rng.normal(0.0, np.sqrt(2.0 / (27 * (c1 + c2))), nw)
        self.set_flat(host)
        return self

    def set_flat(self, host):
        self.p.copy_(self.torch.from_numpy(np.asarray(host, np.float32)))
        self.m.zero_()
        self.v.zero_()
        self.step_count = 0
        _lib.check(self.lib.lb_to_bf16(_p(self.p), self.nparam, _p(self.pb), self._s()))
        self._pack()

    def _pack(self):
        """Forward copies of the BF16 weights, [cout][27][cin] per layer."""
        for name, c1, c2, co, _, _ in self.layers:
            o = self.off[name][0]
            _lib.check(self.lib.lb_conv_pack_weights(ct.c_void_p(self.pb.data_ptr() + 2 * o), c1 + c2, co,
                                                     ct.c_void_p(self.pt.data_ptr() + 2 * o), self._s()))

    def set_layer(self, name, w, b):
        """w [27][cin_used][cout_used] and b [cout_used] (host arrays), zero padded."""
        o, nw, ob, co = self.off[name]
        c = next(l for l in self.layers if l[0] == name)
        cin = c[1] + c[2]
        full = np.zeros((27, cin, co), np.float32)
        full[:, : w.shape[1], : w.shape[2]] = w
        host = self.p.cpu().numpy()
        host[o:o + nw] = full.ravel()
        host[ob:ob + co] = 0.0
        host[ob:ob + len(b)] = b
        self.set_flat(host)

    def get_layer_grad(self, name):
        o, nw, ob, co = self.off[name]
        c = next(l for l in self.layers if l[0] == name)
        g = self.g.cpu().numpy()
        return g[o:o + nw].reshape(27, c[1] + c[2], co), g[ob:ob + co]

    def _conv(self, name, x1, x2, y=None, yf=None, relu=1):
        o, nw, ob, co = self.off[name]
        c = next(l for l in self.layers if l[0] == name)
        lvl = c[5]
        cv = _lib.LbConv()
        cv.x1, cv.c1, cv.up1 = x1.data_ptr(), c[1], c[4]
        cv.x2, cv.c2 = (x2.data_ptr() if x2 is not None else None), c[2]
        cv.w = self.pb.data_ptr() + 2 * o
        cv.wt = self.pt.data_ptr() + 2 * o
        cv.b = self.p.data_ptr() + 4 * ob
        cv.y = y.data_ptr() if y is not None else None
        cv.yf = yf.data_ptr() if yf is not None else None
        cv.acc = self.acc.data_ptr() if lvl >= 1 else None
        cv.D, cv.H, cv.W = self.D >> lvl, self.H >> lvl, self.W >> lvl
        cv.cout, cv.relu = co, relu
        return cv, o, ob

    # ---------------------------------------------------------------- forward
    def forward(self, x_bf16):
        """x_bf16: int16 tensor [P0 * 8] (BF16 canvas).  Returns self.out, the FP32
        [P0][8] network output before the residual (lb_sur_forward: the whole
        network in one library call)."""
        self._x = x_bf16
        _lib.check(self.lib.lb_sur_forward(ct.byref(self.desc), _p(x_bf16), self._s()))
        return self.out

    # --------------------------------------------------------------- backward
    def zero_grad(self):
        _lib.check(self.lib.lb_fill_f32(_p(self.g), self.nparam, 0.0, self._s()))

    def backward(self, gout):
        """Accumulate the parameter gradients for dloss/dout = gout [P0][8] FP32
        (uses the activations of the last forward call; lb_sur_backward)."""
        _lib.check(self.lib.lb_sur_backward(ct.byref(self.desc), _p(self._x), _p(gout), self._s()))

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        _lib.check(self.lib.lb_adam(_p(self.p), _p(self.g), _p(self.m), _p(self.v), _p(self.pb), self.nparam,
                                    self.step_count, lr, b1, b2, eps, self._s()))
        self._pack()

    def loss(self, xin_f32, tgt_f32, lam=1.0, grad=None, sync=True):
        """(loss, relative mass error) of pred = xin + out against tgt; grad
        (FP32 [P0][8]) receives dloss/dout when given."""
        res = (ct.c_double * 4)()
        _lib.check(self.lib.lb_sur_loss(_p(self.out), _p(xin_f32), _p(tgt_f32), self.P[0],
                                        self.scale.ctypes.data_as(ct.c_void_p), float(lam), _p(grad),
                                        _p(self.loss_scratch), res if sync else None, self._s()))
        return (res[3], res[2]) if sync else None

    def train_step(self, x_bf16, xin_f32, tgt_f32, lam=1.0, lr=1e-3):
        """One Adam step on one pair; x_bf16 is the network input (None: the
        normalised input of xin_f32)."""
        if not hasattr(self, "_gout"):
            self._gout = self.torch.zeros(self.P[0] * COUT, dtype=self.torch.float32, device=self.device)
        self.zero_grad()
        self.forward(x_bf16 if x_bf16 is not None else self.prepare(xin_f32))
        out = self.loss(xin_f32, tgt_f32, lam, grad=self._gout)
        self.backward(self._gout)
        self.adam(lr)
        return out


# ---------------------------------------------------------------------------
# canvas I/O, rollouts, training and evaluation (sequencing only)
# ---------------------------------------------------------------------------
def restrict(lat, D, H, W, out_f32=None, out_bf16=None):
    """Coarse canvas of a lattice's current state (library kernel)."""
    import torch

    lib = _lib.load()
    P = D * H * W
    if out_f32 is None:
        out_f32 = torch.empty(P * 8, dtype=torch.float32, device=lat.device)
    if out_bf16 is None:
        out_bf16 = torch.empty(P * 8, dtype=torch.int16, device=lat.device)
    _lib.check(lib.lb_sur_restrict(lat._ctx, D, H, W, _p(out_f32), _p(out_bf16), _stream(lat)))
    return out_f32, out_bf16


def lift(lat, pred_f32, D, H, W):
    """Replace a lattice's state by the prolonged equilibrium of a predicted canvas."""
    lib = _lib.load()
    _lib.check(lib.lb_sur_lift(lat._ctx, _p(pred_f32), D, H, W, _stream(lat)))


def jump_rods(lat, now_f32, next_f32, D, H, W, steps):
    """Advect and re-place a lattice's rods over a jump (before lift)."""
    lib = _lib.load()
    _lib.check(lib.lb_sur_jump_rods(lat._ctx, _p(now_f32), _p(next_f32), D, H, W, float(steps), _stream(lat)))


def drift_rods(lat, x_prev, factor):
    """Each rod continues factor x its displacement since x_prev (a CUDA FP64
    tensor [n_rods, 3] of the centres one interval earlier); re-placed."""
    lib = _lib.load()
    x_prev = x_prev.contiguous()
    _lib.check(lib.lb_sur_drift_rods(lat._ctx, _p(x_prev), float(factor), _stream(lat)))


def _stream(lat):
    import torch

    s = lat.stream if lat.stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def predict(net, x_f32, x_bf16=None, pred_f32=None, pred_bf16=None):
    """pred = x + network(x) on the first six channels (library kernels); the
    network reads the normalised input of x_f32 (x_bf16 is not used)."""
    net.forward(net.prepare(x_f32))
    _lib.check(net.lib.lb_sur_residual(_p(net.out), _p(x_f32), net.P[0], net.scale.ctypes.data_as(ct.c_void_p),
                                       _p(pred_f32), _p(pred_bf16), net._s()))
    return pred_f32, pred_bf16


def advance(lat, net, D, H, W, interval=500, K=50, rate=0.0, threshold=0.005, rod_mobility=0.0, rods_prev=None,
            drift=0.5):
    """One interval of a lattice by the surrogate, with the fallback rule.

    The network's prediction is lifted onto the lattice (rods advected and
    re-placed first); if its rho_A mass differs from M_t - rate * interval
    by more than `threshold` of M_t, the lattice returns to its state before
    the jump and runs the `interval` steps of the method instead; otherwise
    K coupled re-equilibration steps follow.  `rate` is the caller's estimate
    of the rho_A mass the lattice loses per step over the interval, from
    every cause (the reservoir, mass taken into moving rods); the drying
    lattice's own loss rate is only steady enough for such an estimate once
    the start-up transient of a fresh cap has passed.  A jump books nothing
    in the reservoir ledger.  The rods' centres move by rod_mobility x
    interval x the mean coarse fluid velocity at the centre (before and
    after): over 500 steps of the drying caps the rods moved 1.5 nodes on
    average, and that advection put them 2.4 nodes from where the method
    took them against 1.5 for centres held in place, so the default holds
    them.  Given rods_prev (a CUDA FP64 tensor [n_rods, 3] of the centres
    one interval earlier), each rod instead continues `drift` times its
    displacement since then (1.2 nodes off the method's for drift = 0.5).
    Returns {"surrogate": bool, "mass_error": float, "mass": the lifted
    rho_A mass, "mass_t": M_t}.
    """
    import torch

    m_t = float(lat.observables(allow_unstable=True)["mass"][0])
    snap = lat.snapshot()
    xf, _ = restrict(lat, D, H, W)
    pf = torch.empty_like(xf)
    predict(net, xf, pred_f32=pf)
    if lat.n_rods and rods_prev is not None:
        drift_rods(lat, rods_prev, drift)
    elif lat.n_rods:
        jump_rods(lat, xf, pf, D, H, W, interval * float(rod_mobility))
    lift(lat, pf, D, H, W)
    m_pred = float(lat.observables(allow_unstable=True)["mass"][0])
    err = float(abs(m_pred - (m_t - float(rate) * interval)) / m_t)
    if err > threshold:
        lat.restore(snap)
        lat.coupled_step(interval)
        return {"surrogate": False, "mass_error": err, "mass": m_pred, "mass_t": m_t}
    lat.coupled_step(K)
    return {"surrogate": True, "mass_error": err, "mass": m_pred, "mass_t": m_t}


def channel_scales(net, pairs, floor=1e-6):
    """RMS change of each of the six channels over the training pairs (masked),
    from the library's moments kernel."""
    acc = np.zeros(7)
    res = (ct.c_double * 7)()
    for xf, _, yf in pairs:
        _lib.check(net.lib.lb_sur_moments(_p(xf), _p(yf), net.P[0], _p(net.loss_scratch), res, net._s()))
        acc += np.array(res[:])
    return np.maximum(np.sqrt(acc[:6] / max(acc[6], 1.0)), floor).astype(np.float32)


def rollout_snapshots(batch, lats, n_snap, interval, D, H, W, warm=0, rods=True, log=None):
    """Canvases of every lattice every `interval` steps (after `warm` steps):
    tensors [n_lat, n_snap, P * 8] in FP32 and BF16, and a host array
    healthy[n_lat, n_snap]: so far no NaN, no non-positive density, no rod
    limit (status bits 1, 2, 8, 16, 32; the velocity bit 4 alone also trips
    on the start-up transient of a fresh cap) and no canvas speed above
    0.15.  log(str), if given, hears of every snapshot taken."""
    import torch

    P = D * H * W
    dev = lats[0].device
    xf = torch.empty((len(lats), n_snap, P * 8), dtype=torch.float32, device=dev)
    xb = torch.empty((len(lats), n_snap, P * 8), dtype=torch.int16, device=dev)
    healthy = np.zeros((len(lats), n_snap), bool)
    if warm:
        batch.step(warm, rods=rods)
    for s in range(n_snap):
        if s:
            batch.step(interval, rods=rods)
        for i, lat in enumerate(lats):
            restrict(lat, D, H, W, xf[i, s], xb[i, s])
            st = int(lat.observables(allow_unstable=True)["status"])
            u = xf[i, s].view(P, 8)[:, 2:5]
            healthy[i, s] = (st & ~(4 | 64)) == 0 and bool(torch.isfinite(u).all()) and float(u.abs().max()) <= 0.15
        if log:
            log(f"[surrogate] snapshot {s + 1}/{n_snap}: {int(healthy[:, s].sum())} of {len(lats)} lattices healthy")
    torch.cuda.synchronize()
    return xf, xb, healthy


def fit(net, pairs, epochs=1, batch=4, lr=1e-3, lam=1.0, seed=0, log=None, warmup=100, lr_end=0.1):
    """Adam on (x_f32, x_bf16, y_f32) pairs, `batch` samples per update
    (gradients summed), in channel-normalised units (scales from the pairs);
    the learning rate ramps up linearly over the first `warmup` updates and
    then follows a half cosine down to lr_end x lr at the last update (at a
    constant rate, runs of several hundred updates per epoch blew up into a
    network that predicts no change).  Returns the mean training loss of
    every epoch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    import torch

    net.set_scale(channel_scales(net, pairs))
    gout = torch.zeros(net.P[0] * COUT, dtype=torch.float32, device=net.device)
    hist = []
    total = epochs * ((len(pairs) + batch - 1) // batch)
    done = 0
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        tot = 0.0
        for k in range(0, len(order), batch):
            net.zero_grad()
            for j in order[k:k + batch]:
                xf, xb, yf = pairs[j]
                net.forward(net.prepare(xf))
                loss, _ = net.loss(xf, yf, lam, grad=gout)
                net.backward(gout)
                tot += loss
            done += 1
            decay = lr_end + (1.0 - lr_end) * 0.5 * (1.0 + np.cos(np.pi * min(1.0, done / max(1, total))))
            net.adam(lr * min(1.0, done / max(1, warmup)) * decay)
        hist.append(tot / max(1, len(pairs)))
        if log:
            log(f"[surrogate] epoch {ep}: loss {hist[-1]:.4e}")
    return hist


def evaluate(net, pairs, lam=1.0, prev=None):
    """Mean loss of the network, of persistence (y = x) and, when the previous
    snapshots are given, of linear extrapolation (y = 2 x - x_prev), using the
    library's loss kernel for all three."""
    import torch

    zeros = torch.zeros(net.P[0] * COUT, dtype=torch.float32, device=net.device)
    res = {"net": 0.0, "persistence": 0.0, "mass_err_net": 0.0, "mass_err_persistence": 0.0}
    if prev is not None:
        res["linear"] = 0.0
    for k, (xf, xb, yf) in enumerate(pairs):
        net.forward(net.prepare(xf))
        l, me = net.loss(xf, yf, lam)
        res["net"] += l
        res["mass_err_net"] += abs(me)
        saved = net.out.clone()
        net.out.copy_(zeros)
        l0, me0 = net.loss(xf, yf, lam)
        res["persistence"] += l0
        res["mass_err_persistence"] += abs(me0)
        if prev is not None:
            # x + (x - x_prev): the network output that gives it, in scaled units
            sc = torch.ones(8, dtype=torch.float32, device=net.device)
            sc[:6] = torch.from_numpy(net.scale)
            net.out.copy_(((xf - prev[k]).view(-1, 8) / sc).view(-1))
            l1, _ = net.loss(xf, yf, lam)
            res["linear"] += l1
        net.out.copy_(saved)
    for key in res:
        res[key] /= max(1, len(pairs))
    return res
