"""FP64 oracle of the learned surrogate: restriction, prolongation, 3-D
convolutions with their gradients, the U-Net and Adam.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

What it follows (a learned surrogate: a small 3-D convolutional encoder-decoder
advancing coarse-grained fields of the lattice Boltzmann state; the paper
itself has no surrogate):
* restriction: 2 x 2 x 2 block means onto a coarse canvas of the channels
  rho_A, rho_B, u_x, u_y, u_z (densities are means over the block's fluid
  nodes; u is the block's physical velocity, sum of (j* - F/2) over its fluid
  nodes divided by their summed density, where j* = sum_k sum_i f*_i c_i is
  the momentum of the stored post-collision state and F = F_A + F_B the
  Shan-Chen plus body force of its densities (the fluid step's force), so that with equal tau
  the momentum before collision is j* - F and the velocity u = (j + F/2) / rho
  the one the method reports), the rod volume
  fraction (rod nodes / 8), a domain mask (1 inside the lattice) and the
  fluid fraction (fluid nodes / 8); canvas cells outside a smaller lattice
  hold gas (rho_A 0.03, rho_B 1), zero velocity, mask 0 and fluid fraction 0;
* prolongation: trilinear interpolation of rho_A, rho_B, u at fine node x from
  coarse coordinate x / 2 - 1/4 (clamped to the lattice's own coarse extent)
  over the corner cells that hold fluid (fluid fraction > 0), the weights
  renormalised; when none of the 8 corners holds fluid, the plain mean of the
  fluid-holding cells of the 4 x 4 x 4 block around them, and gas at rest
  when there is none either; then the post-collision state of those fields:
  with F_k the Shan-Chen force of the prolonged densities, u' = u - F / (2 rho)
  and u_k^eq = u' + tau_k F_k / rho_k (the velocity shift of the collision),
  (u' alone where rho_k < 1e-12), f_i^k = f_i^eq(rho_k, u_k^eq) (Eq. 2) at
  fluid nodes, so that restricting
  the lifted state node by node gives back rho_k and u;
* convolution: y[p, o] = b[o] + sum_{t, c} x[p + o_t, c] w[t, c, o] over the
  27 taps o_t in {-1, 0, 1}^3 with zero padding, channels-last tensors;
  input gradient dx[q, c] = sum_{t, o} g[q - o_t, o] w[t, c, o]; weight
  gradient dw[t, c, o] = sum_p x[p + o_t, c] g[p, o]; bias gradient sum_p g;
* U-Net with four levels (32, 64, 128, 128 channels), two ReLU convolutions
  per level, 2 x 2 x 2 average pooling down, nearest-neighbour upsampling and
  channel concatenation of the skip on the way up, a final linear
  convolution to the six predicted channels added to the input (residual);
* loss: masked mean squared error over the six channels, each channel in
  units of its own scale (the RMS change of that channel over the training
  interval), plus lambda times the squared relative mass error of rho_A;
* Adam (Kingma and Ba) with bias correction.
"""
from __future__ import annotations

import numpy as np

from . import lbm

GAS = (0.03, 1.0)
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


# ---------------------------------------------------------------------------
# restriction / prolongation
# ---------------------------------------------------------------------------
def restrict(f, material, canvas, p):
    """Coarse canvas [D, H, W, 8] (FP64) of a stored post-collision state
    f[2, 19, nz, ny, nx] with the lattice parameters p (lbm.Params)."""
    D, H, W = canvas
    nz, ny, nx = material.shape
    fluid = material == lbm.FLUID
    rho_all = f.sum(axis=1)
    F = lbm.sc_force(lbm.pseudopotential(rho_all, material, p), rho_all, p)
    rho = np.where(fluid, rho_all, 0.0)  # [2, nz, ny, nx]
    C = lbm.C.astype(np.float64)
    mom = np.einsum("kizyx,id->dzyx", f, C) - 0.5 * (F[0] + F[1])
    mom = np.where(fluid[None], mom, 0.0)
    out = np.zeros((D, H, W, 8))
    out[..., 0], out[..., 1] = GAS
    for cz in range(D):
        for cy in range(H):
            for cx in range(W):
                z0, y0, x0 = 2 * cz, 2 * cy, 2 * cx
                if z0 + 1 >= nz or y0 + 1 >= ny or x0 + 1 >= nx:
                    continue  # outside the lattice: gas, mask 0
                blk = (slice(z0, z0 + 2), slice(y0, y0 + 2), slice(x0, x0 + 2))
                nf = int(fluid[blk].sum())
                cell = np.zeros(8)
                if nf:
                    r = rho[(slice(None),) + blk].reshape(2, -1).sum(axis=1)
                    m = mom[(slice(None),) + blk].reshape(3, -1).sum(axis=1)
                    cell[0:2] = r / nf
                    tot = r.sum()
                    cell[2:5] = m / tot if tot > 0 else 0.0
                cell[5] = float((material[blk] == lbm.ROD).sum()) / 8.0
                cell[6] = 1.0
                cell[7] = nf / 8.0
                out[cz, cy, cx] = cell
    return out


def _lerp_axis(n_fine, n_coarse):
    """Per fine index x: (lower coarse index, upper, weight of upper) for x/2 - 1/4."""
    lo, hi, wt = [], [], []
    for x in range(n_fine):
        c = x / 2.0 - 0.25
        c = min(max(c, 0.0), n_coarse - 1.0)
        i0 = int(np.floor(c))
        i1 = min(i0 + 1, n_coarse - 1)
        lo.append(i0)
        hi.append(i1)
        wt.append(c - i0)
    return np.array(lo), np.array(hi), np.array(wt)


def prolong(coarse, material):
    """Fine (rho[2], u[3]) on the lattice from coarse [D, H, W, 8] fields; the
    lattice occupies coarse cells [0, n/2) per axis."""
    nz, ny, nx = material.shape
    cz, cy, cx = nz // 2, ny // 2, nx // 2
    a = coarse[:cz, :cy, :cx, :5]
    ok = coarse[:cz, :cy, :cx, 7] > 0
    lz, hz, wz = _lerp_axis(nz, cz)
    ly, hy, wy = _lerp_axis(ny, cy)
    lx, hx, wx = _lerp_axis(nx, cx)
    gas = np.array([GAS[0], GAS[1], 0.0, 0.0, 0.0])
    out = np.zeros((nz, ny, nx, 5))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                acc = np.zeros(5)
                wsum = 0.0
                for iz, fz in ((lz[z], 1 - wz[z]), (hz[z], wz[z])):
                    for iy, fy in ((ly[y], 1 - wy[y]), (hy[y], wy[y])):
                        for ix, fx in ((lx[x], 1 - wx[x]), (hx[x], wx[x])):
                            if ok[iz, iy, ix]:
                                wt = fz * fy * fx
                                acc += wt * a[iz, iy, ix]
                                wsum += wt
                if wsum > 0:
                    out[z, y, x] = acc / wsum
                    continue
                acc[:] = 0.0
                cnt = 0
                for iz in range(lz[z] - 1, lz[z] + 3):
                    for iy in range(ly[y] - 1, ly[y] + 3):
                        for ix in range(lx[x] - 1, lx[x] + 3):
                            if 0 <= iz < cz and 0 <= iy < cy and 0 <= ix < cx and ok[iz, iy, ix]:
                                acc += a[iz, iy, ix]
                                cnt += 1
                out[z, y, x] = acc / cnt if cnt else gas
    rho = np.moveaxis(out[..., 0:2], -1, 0)
    u = np.moveaxis(out[..., 2:5], -1, 0)
    return rho, u


# largest lifted speed: half the lattice's stability flag |u| > 0.3, the
# speed above which a canvas is no longer taken as training data
LIFT_SPEED_MAX = 0.15


def admissible(rho, u):
    """The prolonged fields mapped onto states the lattice can take: each
    rho_k clamped at 0, and a speed above LIFT_SPEED_MAX scaled down to it
    (direction kept).  A predicted canvas can leave both sets; the method's
    own states never do."""
    rho = np.maximum(rho, 0.0)
    speed = np.sqrt((u * u).sum(axis=0))
    scale = np.where(speed > LIFT_SPEED_MAX, LIFT_SPEED_MAX / np.where(speed > 0, speed, 1.0), 1.0)
    return rho, u * scale


def conserve(rho, coarse, material):
    """Each component's prolonged density scaled so that its total over the
    fluid nodes is the canvas's: the sum over the cells inside the lattice of
    rho_k times the cell's fluid nodes (8 x channel 7); no scaling unless
    both totals are positive."""
    nz, ny, nx = material.shape
    cells = coarse[: nz // 2, : ny // 2, : nx // 2]
    fluid = material == lbm.FLUID
    out = rho.copy()
    for k in range(2):
        want = float((cells[..., k] * 8.0 * cells[..., 7]).sum())
        have = float(rho[k][fluid].sum())
        if want > 0.0 and have > 0.0:
            out[k] = rho[k] * (want / have)
    return out


def lift(coarse, material, p):
    """Post-collision state f^k = f^eq(rho_k, u_k^eq) (Eq. 2) of the prolonged
    fields, made admissible and mass-conserving (conserve), at fluid nodes, 0
    elsewhere; u_k^eq = u - F / (2 rho) + tau_k F_k / rho_k with F_k the
    Shan-Chen force of the lifted densities (no half-force shift where rho
    vanishes)."""
    rho, u = admissible(*prolong(coarse, material))
    rho = conserve(rho, coarse, material)
    fluid = material == lbm.FLUID
    F = lbm.sc_force(lbm.pseudopotential(rho, material, p), rho, p)
    tot = rho[0] + rho[1]
    has = fluid & (tot > 1e-12)
    up = u - np.where(has, 0.5 * (F[0] + F[1]) / np.where(has, tot, 1.0), 0.0)
    f = []
    for k in range(2):
        ok = fluid & (rho[k] >= 1e-12)  # the shift is skipped for a vanishing component
        ueq = np.where(ok, up + p.tau[k] * F[k] / np.where(ok, rho[k], 1.0), up)
        f.append(lbm.equilibrium(rho[k], ueq))
    return np.where(fluid[None, None], np.stack(f), 0.0)


# ---------------------------------------------------------------------------
# convolution and its gradients (channels last: x[D, H, W, C])
# ---------------------------------------------------------------------------
def _shifted(x, off):
    """x[p + off] with zero padding."""
    D, H, W = x.shape[:3]
    out = np.zeros_like(x)
    dz, dy, dx = off
    zs = slice(max(0, -dz), min(D, D - dz))
    ys = slice(max(0, -dy), min(H, H - dy))
    xs = slice(max(0, -dx), min(W, W - dx))
    zt = slice(max(0, dz), min(D, D + dz))
    yt = slice(max(0, dy), min(H, H + dy))
    xt = slice(max(0, dx), min(W, W + dx))
    out[zs, ys, xs] = x[zt, yt, xt]
    return out


def conv3d(x, w, b=None):
    """x [D, H, W, Cin], w [27, Cin, Cout] (tap index (dz+1)*9 + (dy+1)*3 + dx+1)."""
    y = np.zeros(x.shape[:3] + (w.shape[2],))
    for t, off in enumerate(TAPS):
        y += _shifted(x, off) @ w[t]
    if b is not None:
        y += b
    return y


def conv3d_dgrad(g, w):
    dx = np.zeros(g.shape[:3] + (w.shape[1],))
    for t, off in enumerate(TAPS):
        dx += _shifted(g, tuple(-o for o in off)) @ w[t].T
    return dx


def conv3d_wgrad(x, g):
    cin, cout = x.shape[3], g.shape[3]
    dw = np.zeros((27, cin, cout))
    gm = g.reshape(-1, cout)
    for t, off in enumerate(TAPS):
        dw[t] = _shifted(x, off).reshape(-1, cin).T @ gm
    return dw, gm.sum(axis=0)


def conv3d_direct(x, w, b):
    """Seven nested loops, for tiny shapes (pins the tap convention)."""
    D, H, W, cin = x.shape
    cout = w.shape[2]
    y = np.zeros((D, H, W, cout))
    for z in range(D):
        for yy in range(H):
            for xx in range(W):
                for o in range(cout):
                    s = b[o]
                    for t, (dz, dy, dx) in enumerate(TAPS):
                        qz, qy, qx = z + dz, yy + dy, xx + dx
                        if 0 <= qz < D and 0 <= qy < H and 0 <= qx < W:
                            for c in range(cin):
                                s += x[qz, qy, qx, c] * w[t, c, o]
                    y[z, yy, xx, o] = s
    return y


def pool2(x):
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def pool2_back(g):
    return np.repeat(np.repeat(np.repeat(g, 2, 0), 2, 1), 2, 2) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up2_back(g):
    D, H, W, C = g.shape
    return g.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


# ---------------------------------------------------------------------------
# U-Net
# ---------------------------------------------------------------------------
CH = (32, 64, 128, 128)
IN_CH, OUT_CH = 7, 6


def layer_shapes(cin=IN_CH, ch=CH, cout=OUT_CH):
    """(name, Cin, Cout) of every convolution, in forward order."""
    L = []
    c = cin
    for lvl, co in enumerate(ch):
        L.append((f"enc{lvl}a", c, co))
        L.append((f"enc{lvl}b", co, co))
        c = co
    for lvl in range(len(ch) - 2, -1, -1):
        L.append((f"dec{lvl}a", c + ch[lvl], ch[lvl]))
        L.append((f"dec{lvl}b", ch[lvl], ch[lvl]))
        c = ch[lvl]
    L.append(("out", c, cout))
    return L


def init_params(seed, cin=IN_CH, ch=CH, cout=OUT_CH):
    """He-normal weights (std sqrt(2 / (27 Cin))), zero biases; the output layer
    starts at zero so the untrained network is the persistence baseline."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = {}
    for name, ci, co in layer_shapes(cin, ch, cout):
        std = 0.0 if name == "out" else np.sqrt(2.0 / (27 * ci))
        P[name] = (rng.normal(0.0, 1.0, (27, ci, co)) * std, np.zeros(co))
    return P


def unet_forward(x, P, ch=CH, act_round=None):
    """x [D, H, W, 7] -> (prediction [D, H, W, 6], cache).  act_round
    (optional) models the storage precision of the activations: it is applied
    to every hidden layer's output after the ReLU and to every pooled map."""
    rnd = act_round if act_round is not None else (lambda a: a)
    cache = {"x": x}
    h = x
    skips = []
    nlev = len(ch)
    for lvl in range(nlev):
        for s in "ab":
            name = f"enc{lvl}{s}"
            cache[name + ":in"] = h
            h = rnd(np.maximum(conv3d(h, *P[name]), 0.0))
            cache[name + ":out"] = h
        if lvl < nlev - 1:
            skips.append(h)
            h = rnd(pool2(h))
    for lvl in range(nlev - 2, -1, -1):
        h = np.concatenate([up2(h), skips[lvl]], axis=-1)
        for s in "ab":
            name = f"dec{lvl}{s}"
            cache[name + ":in"] = h
            h = rnd(np.maximum(conv3d(h, *P[name]), 0.0))
            cache[name + ":out"] = h
    cache["out:in"] = h
    y = conv3d(h, *P["out"])
    return x[..., :OUT_CH] + y, cache


def unet_backward(gy, P, cache, ch=CH):
    """Gradients of every parameter for dL/dprediction = gy."""
    G = {}
    dw, db = conv3d_wgrad(cache["out:in"], gy)
    G["out"] = (dw, db)
    gh = conv3d_dgrad(gy, P["out"][0])
    nlev = len(ch)
    gskip = [None] * (nlev - 1)
    for lvl in range(0, nlev - 1):
        for s in "ba":
            name = f"dec{lvl}{s}"
            g = gh * (cache[name + ":out"] > 0)
            G[name] = conv3d_wgrad(cache[name + ":in"], g)
            gh = conv3d_dgrad(g, P[name][0])
        cu = gh.shape[-1] - ch[lvl]
        gskip[lvl] = gh[..., cu:]
        gh = up2_back(gh[..., :cu])
    for lvl in range(nlev - 1, -1, -1):
        if lvl < nlev - 1:
            gh = pool2_back(gh) + gskip[lvl]
        for s in "ba":
            name = f"enc{lvl}{s}"
            g = gh * (cache[name + ":out"] > 0)
            G[name] = conv3d_wgrad(cache[name + ":in"], g)
            gh = conv3d_dgrad(g, P[name][0])
    return G


def loss(pred, target, mask, lam, scale=None):
    """Masked MSE over the six channels in channel-normalised units
    e_c = (pred_c - target_c) / scale_c, plus lam * (relative rho_A mass
    error)^2, and its gradient with respect to pred."""
    s = np.ones(OUT_CH) if scale is None else np.asarray(scale, dtype=np.float64)
    m = mask[..., None]
    n = mask.sum()
    diff = (pred - target) / s * m
    mse = float((diff * diff).sum() / (OUT_CH * n))
    mt = float((mask * target[..., 0]).sum())
    me = float((mask * (pred[..., 0] - target[..., 0])).sum()) / mt
    g = 2.0 * diff / s / (OUT_CH * n)
    g[..., 0] += 2.0 * lam * me * mask / mt
    return mse + lam * me * me, g


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
