"""FP64 oracle: two-component colour-gradient D3Q19 step (the paper's fluid model).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

What it follows (Methods, "Fluid-filament simulation method")
-------------------------------------------------------------
* Per component k the lattice Boltzmann equation with BGK relaxation tau_k
  (Eq. 1) towards the second-order equilibrium (Eq. 2) taken with the common
  fluid velocity u; moments rho_k = sum_i f_i^k, rho u = sum_k sum_i f_i^k c_i
  (Eq. 3, rho_0 = 1).
* Phase segregation: a colour-blind collision followed by recolouring.
* Interfacial tension by a continuum-surface force: the curvature comes from
  gradients of the colour field C = (rho_1 - rho_2) / (rho_1 + rho_2), the
  capillary force acts as a body force before the collision, weighted by the
  local density fractions.
* Wetting: wall normals reconstructed from the voxel geometry, a prescribed
  contact angle imposed through the colour indicator of the solid ghost
  layer.

Readings where the paper is silent (listed in the design notes)
---------------------------------------------------------------
* Gradients: the isotropic D3Q19 stencil grad phi(x) = (1/c_s^2) sum_i w_i
  phi(x + c_i) c_i; n = grad C / |grad C| where |grad C| > 10^-2, else 0 (in
  the bulk the direction of a vanishing gradient is noise, and between two
  interfaces it flips, which the curvature would turn into a force);
  curvature kappa = -div n by the same stencil.
* CSF force (Brackbill's form for an indicator that jumps by 2):
  F = (sigma / 2) kappa |grad C| n, so that a drop of radius R carries the
  Laplace jump sigma kappa = 2 sigma / R; component k feels
  F_k = (rho_k / rho) F.
* Force in the collision: Guo's scheme, u = (sum_k j_k + F / 2) / rho and
  f*_i^k = f_i^k - (f_i^k - f_i^{k,eq}(rho_k, u)) / tau_k
           + (1 - 1 / (2 tau_k)) w_i [(c_i - u) / c_s^2 + (c_i.u) c_i / c_s^4] . F_k.
* Recolouring (the Latva-Kokko--Rothman form used by Leclaire et al.):
  with f*_i = sum_k f*_i^k and cos phi_i = c_i . n / |c_i|,
  f_i^1 = (rho_1 / rho) f*_i + beta (rho_1 rho_2 / rho) w_i cos phi_i,
  f_i^2 = (rho_2 / rho) f*_i - beta (rho_1 rho_2 / rho) w_i cos phi_i
  (rest population split by the fractions alone); beta = 0.7 by default.
* Ghost layer and contact angle: a solid node next to the fluid carries the
  weighted mean C_g = sum w_i C(y + c_i) / sum w_i over its fluid
  neighbours; a fluid node next to a wall has the wall normal
  n_w = -normalise(sum_i w_i [x + c_i solid] c_i) (into the fluid) and the
  contact angle of its solid neighbours (cos theta averaged with weights
  w_i), and its interface normal is replaced by
  n* = -cos(theta) n_w + sin(theta) t, t the unit tangential part of n
  (unchanged when n has no tangential part).  n points into the liquid
  (component 1), so theta is measured through the liquid.  The corrected
  normal drives the recolouring and the force there.  In the curvature
  stencil a neighbour without a normal of its own (a solid node, or one
  below the gradient threshold) enters with the node's own normal.

Conventions as in oracle.lbm: f[k, i, z, y, x], post-collision state stored,
material 0 fluid, 2..7 static walls (halfway bounce-back).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import lbm

C = lbm.C
W = lbm.W
Q = lbm.Q
CS2 = lbm.CS2
GRAD_EPS = 1e-2


@dataclass
class CGParams:
    shape: tuple  # (nz, ny, nx)
    periodic: tuple = (True, True, True)  # (x, y, z)
    tau: tuple = (1.0, 1.0)
    sigma: float = 0.01
    beta: float = 0.7
    body_force: tuple = (0.0, 0.0, 0.0)  # acceleration g (x, y, z)
    # contact angle per wall material (radians), theta[m] for m = 2..7
    theta: np.ndarray = field(default_factory=lambda: np.full(9, np.pi / 2))


def _ahead(a, c):
    return lbm._ahead(a, c)


def grad(phi):
    """(1/c_s^2) sum_i w_i phi(x + c_i) c_i over the periodic array phi."""
    g = np.zeros((3,) + phi.shape)
    for i in range(1, Q):
        nb = _ahead(phi, C[i])
        for a in range(3):
            if C[i, a] != 0:
                g[a] = g[a] + (W[i] * nb) * C[i, a]
    return g / CS2


def ghost_colour(Cf, fluid):
    """Colour of every node: C on fluid nodes; on solid nodes the w-weighted
    mean over their fluid neighbours (0 where there is none)."""
    num = np.zeros(Cf.shape)
    den = np.zeros(Cf.shape)
    for i in range(1, Q):
        nbf = _ahead(fluid, C[i])
        num = num + W[i] * np.where(nbf, _ahead(Cf, C[i]), 0.0)
        den = den + W[i] * nbf
    ghost = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
    return np.where(fluid, Cf, ghost)


def wall_geometry(material, p: CGParams):
    """Per fluid node next to a wall: unit wall normal (into the fluid) and the
    w-weighted mean cos(theta) of its solid neighbours.  Returns (near, n_w,
    cos_theta) with near the mask of such nodes."""
    solid = lbm.is_static_solid(material)
    fluid = material == lbm.FLUID
    s = np.zeros((3,) + material.shape)
    wsum = np.zeros(material.shape)
    ctsum = np.zeros(material.shape)
    th = np.asarray(p.theta, dtype=np.float64)
    for i in range(1, Q):
        nbs = _ahead(solid, C[i])
        nbm = _ahead(material, C[i])
        for a in range(3):
            if C[i, a] != 0:
                s[a] = s[a] + W[i] * nbs * C[i, a]
        wsum = wsum + W[i] * nbs
        ctsum = ctsum + W[i] * nbs * np.cos(th[np.clip(nbm, 0, len(th) - 1)])
    near = fluid & (wsum > 0)
    norm = np.sqrt((s * s).sum(axis=0))
    nw = np.where(norm > 0, -s / np.where(norm > 0, norm, 1.0), 0.0)
    ct = np.where(wsum > 0, ctsum / np.where(wsum > 0, wsum, 1.0), 0.0)
    return near, nw, ct


def normals(gC, near, nw, ct):
    """Unit interface normal n = grad C / |grad C| (0 where |grad C| <= 10^-2),
    with the contact-angle correction at fluid nodes next to walls."""
    mag = np.sqrt((gC * gC).sum(axis=0))
    has = mag > GRAD_EPS
    n = np.where(has, gC / np.where(has, mag, 1.0), 0.0)
    dot = (n * nw).sum(axis=0)
    t = n - dot * nw
    tm = np.sqrt((t * t).sum(axis=0))
    tang = tm > 1e-12
    that = np.where(tang, t / np.where(tang, tm, 1.0), 0.0)
    st = np.sqrt(np.maximum(1.0 - ct * ct, 0.0))
    corr = -ct * nw + st * that
    use = near & has & tang
    return np.where(use, corr, n), mag


def curvature(n, defined):
    """kappa = -div n with the D3Q19 stencil; a neighbour without a normal of
    its own (a solid node, or |grad C| at or below the threshold) enters with
    the node's own normal, so a flat interface has zero curvature up to where
    its normals end."""
    div = np.zeros(defined.shape)
    for i in range(1, Q):
        nbf = _ahead(defined, C[i])
        nbn = np.stack([_ahead(n[a], C[i]) for a in range(3)])
        v = np.where(nbf[None], nbn, n)
        div = div + W[i] * (v[0] * C[i, 0] + v[1] * C[i, 1] + v[2] * C[i, 2])
    return -div / CS2


def csf_force(kappa, mag, n, p: CGParams):
    """F = (sigma / 2) kappa |grad C| n."""
    return 0.5 * p.sigma * kappa * mag * n


def guo_source(u, Fk, tau):
    """(1 - 1/(2 tau)) w_i [(c_i - u)/c_s^2 + (c_i.u) c_i / c_s^4] . F_k -> (19, ...)."""
    out = np.empty((Q,) + u.shape[1:])
    uF = u[0] * Fk[0] + u[1] * Fk[1] + u[2] * Fk[2]
    for i in range(Q):
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        cF = C[i, 0] * Fk[0] + C[i, 1] * Fk[1] + C[i, 2] * Fk[2]
        out[i] = W[i] * ((cF - uF) / CS2 + cu * cF / (CS2 * CS2))
    return (1.0 - 0.5 / tau) * out


def recolour(fstar, rho, n, beta):
    """Split the colour-blind post-collision populations f*_i = sum_k f*_i^k
    between the colours: proportional share plus the segregation term
    +- beta (rho_1 rho_2 / rho) w_i cos phi_i with cos phi_i = c_i . n / |c_i|."""
    tot = fstar[0] + fstar[1]
    rt = rho[0] + rho[1]
    rts = np.where(rt > 0, rt, 1.0)
    out = np.empty_like(fstar)
    seg = beta * rho[0] * rho[1] / rts
    for i in range(Q):
        if i == 0:
            cphi = np.zeros(rt.shape)
        else:
            cphi = (C[i, 0] * n[0] + C[i, 1] * n[1] + C[i, 2] * n[2]) / np.sqrt(float((C[i] ** 2).sum()))
        out[0, i] = rho[0] / rts * tot[i] + seg * W[i] * cphi
        out[1, i] = rho[1] / rts * tot[i] - seg * W[i] * cphi
    return out


def check_boundaries(material, p: CGParams):
    lp = lbm.Params(shape=p.shape, periodic=p.periodic)
    lbm.check_boundaries(material, lp)
    if np.any(material == lbm.GHOST) or np.any(material == lbm.ROD):
        raise ValueError("the colour-gradient step takes fluid and static walls only")


def cg_step(fpost, material, p: CGParams, geo=None):
    """One colour-gradient step t -> t+1 on the post-collision state.

    Returns (f*(t+1), diagnostics dict with rho, j, C, n, kappa, F, u)."""
    fluid = material == lbm.FLUID
    if geo is None:
        geo = wall_geometry(material, p)
    near, nw, ct = geo
    lp = lbm.Params(shape=p.shape, periodic=p.periodic)
    f, _ = lbm.pull_stream(fpost, material, lp)
    rho = np.empty((2,) + material.shape)
    j = np.empty((2, 3) + material.shape)
    for k in range(2):
        rho[k], j[k] = lbm.moments(f[k])
    rho = np.where(fluid, rho, 0.0)
    j = np.where(fluid, j, 0.0)
    rt = rho[0] + rho[1]
    rts = np.where(rt > 0, rt, 1.0)
    Cf = np.where(fluid, (rho[0] - rho[1]) / rts, 0.0)
    Cg = ghost_colour(Cf, fluid)
    gC = np.where(fluid, grad(Cg), 0.0)
    n, mag = normals(gC, near, nw, ct)
    n = np.where(fluid, n, 0.0)
    kappa = np.where(fluid, curvature(n, fluid & (mag > GRAD_EPS)), 0.0)
    F = np.where(fluid, csf_force(kappa, mag, n, p), 0.0)
    F = F + rt * np.asarray(p.body_force, dtype=np.float64)[:, None, None, None]
    u = (j[0] + j[1] + 0.5 * F) / rts
    out = np.empty_like(f)
    for k in range(2):
        Fk = rho[k] / rts * F
        feq = lbm.equilibrium(rho[k], u)
        out[k] = f[k] - (f[k] - feq) / p.tau[k] + guo_source(u, Fk, p.tau[k])
    out = recolour(out, rho, n, p.beta)
    out = np.where(fluid, out, 0.0)
    return out, {"rho": rho, "j": j, "C": Cf, "n": n, "kappa": kappa, "F": F, "u": np.where(fluid, u, 0.0)}


class CGRun:
    """Holds the state of one colour-gradient oracle run."""

    def __init__(self, rho0, material, p: CGParams):
        self.p = p
        self.material = np.ascontiguousarray(material, dtype=np.uint8)
        check_boundaries(self.material, p)
        self.geo = wall_geometry(self.material, p)
        self.f = lbm.initial_state(np.where(self.material == lbm.FLUID, rho0, 0.0))
        self.t = 0
        self.last = None

    def step(self, n=1):
        for _ in range(n):
            self.f, self.last = cg_step(self.f, self.material, self.p, self.geo)
            self.t += 1
        return self

    def masses(self):
        fl = self.material == lbm.FLUID
        return np.array([float(np.where(fl, self.f[k].sum(axis=0), 0.0).sum()) for k in range(2)])
