"""FP64 oracle: two-component Shan-Chen D3Q19 BGK lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

What it follows
---------------
* Lattice Boltzmann equation per component k, BGK relaxation with tau_k
  (Methods, "Fluid-filament simulation method", Eq. 1).
* Second-order equilibrium with c_s^2 = 1/3 (Eq. 2).
* Moments rho_k = sum_i f_i^k and rho u = sum_k sum_i f_i^k c_i (Eq. 3); the
  reference density rho_0 of Eq. 3 is taken as 1.
* The paper applies its interfacial force as a body force before collision
  (Methods, paragraph on the continuum-surface-force formulation).  Here the
  interfacial force is the Shan-Chen cross-component pseudopotential force,
  incorporated through the Shan-Chen velocity shift of the equilibrium
  velocity.  The paper names no velocity set; D3Q19 is used.
* Substrate wetting (paper: a ghost layer inside the solid carries the wetting
  information, Methods, Akai formulation) is realised the Shan-Chen way: solid
  nodes carry fixed ghost pseudo-densities psi^s(material) that enter the same
  force sum as fluid neighbours.
* Evaporation: the top plane is a fixed reservoir (Dirichlet ghost layer) with
  prescribed densities rho_top; populations streaming into it are lost and the
  reservoir's equilibrium populations stream out of it.  The mass lost is kept
  in an FP64 ledger.  (The paper's own interfacial sink, Eq. 8, is a different
  evaporation model.)

Conventions
-----------
* Populations are arrays f[k, i, z, y, x] (k = 0 liquid-forming component A,
  k = 1 component B).
* The stored state at time t is the POST-COLLISION population f*(t).  At t = 0
  it is f* = w_i rho_k (the initial densities at rest).  One step pulls
  f_i(x, t+1) = f*_i(x - c_i, t), takes moments, force and collision, and
  returns f*(t+1).
* Material codes (uint8): 0 fluid, 1 top ghost reservoir, 2..7 static solid
  wall materials, 8 rod solid.  Solid nodes hold no populations.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# D3Q19 lattice (Eq. 1's discrete velocities c_i with weights w_i of Eq. 2)
# --------------------------------------------------------------------------
C = np.array(
    [
        [0, 0, 0],
        [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
        [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
        [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
        [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1],
    ],
    dtype=np.int64,
)
W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)
Q = 19
CS2 = 1.0 / 3.0
OPP = np.array([int(np.where((C == -C[i]).all(axis=1))[0][0]) for i in range(Q)])

FLUID, GHOST, ROD = 0, 1, 8


def is_static_solid(material):
    return (material >= 2) & (material <= 7)


@dataclass
class Params:
    """Physical and lattice parameters of one run (all plain numbers)."""

    shape: tuple  # (nz, ny, nx)
    periodic: tuple = (True, True, True)  # (x, y, z)
    tau: tuple = (1.0, 1.0)
    G: float = 3.6
    body_force: tuple = (0.0, 0.0, 0.0)  # acceleration g (x, y, z)
    psi_solid: np.ndarray = field(default_factory=lambda: np.zeros((9, 2)))
    rho_top: tuple = (0.0, 1.0)
    evaporation: bool = False
    # the paper's evaporation law (Eq. 8): an interfacial sink with flux
    # J = J0 / (K + h / h0) per interface node and step
    sink: bool = False
    sink_J0: float = 0.0
    sink_K: float = 0.01
    sink_h0: float = 1.0


def _shift(a, c):
    """Value at x - c for every x (periodic wrap on the last three axes)."""
    return np.roll(a, shift=(int(c[2]), int(c[1]), int(c[0])), axis=(-3, -2, -1))


def _ahead(a, c):
    """Value at x + c for every x (periodic wrap on the last three axes)."""
    return np.roll(a, shift=(-int(c[2]), -int(c[1]), -int(c[0])), axis=(-3, -2, -1))


def equilibrium(rho, u):
    """Eq. 2: f_i^eq = w_i rho [1 + c.u/cs2 + (c.u)^2/(2 cs4) - u^2/(2 cs2)].

    rho: (...), u: (3, ...) -> (19, ...)
    """
    usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    out = np.empty((Q,) + rho.shape)
    for i in range(Q):
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        out[i] = W[i] * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - usq / (2.0 * CS2))
    return out


def moments(f):
    """Eq. 3 with rho_0 = 1: rho = sum_i f_i, j = sum_i f_i c_i.

    f: (19, ...) -> rho (...), j (3, ...)
    """
    rho = np.zeros(f.shape[1:])
    j = np.zeros((3,) + f.shape[1:])
    for i in range(Q):
        rho = rho + f[i]
        for a in range(3):
            if C[i, a] != 0:
                j[a] = j[a] + C[i, a] * f[i]
    return rho, j


def initial_state(rho0):
    """Post-collision state at t = 0: f*_i = w_i rho_k (fluid at rest).

    rho0: (2, nz, ny, nx) FP64 densities (zero on non-fluid nodes is fine).
    """
    return W[None, :, None, None, None] * rho0[:, None]


def pseudopotential(rho, material, p: Params):
    """psi_k: rho_k on fluid, rho_top on the ghost plane, psi^s(m) on solids."""
    psi = np.empty_like(rho)
    for k in range(2):
        ps = np.asarray(p.psi_solid, dtype=np.float64)[:, k]
        solid_val = ps[np.clip(material, 0, len(ps) - 1)]
        psi[k] = np.where(material == FLUID, rho[k], np.where(material == GHOST, p.rho_top[k], solid_val))
    return psi


def sc_force(psi, rho, p: Params):
    """Shan-Chen cross-component force plus body force.

    F_k(x) = -G psi_k(x) sum_{i=1..18} w_i psi_kbar(x + c_i) c_i + rho_k g.
    Summed over i in index order.
    """
    F = np.zeros((2, 3) + rho.shape[1:])
    for k in range(2):
        kb = 1 - k
        s = np.zeros((3,) + rho.shape[1:])
        for i in range(1, Q):
            nb = _ahead(psi[kb], C[i])
            for a in range(3):
                if C[i, a] != 0:
                    s[a] = s[a] + (W[i] * nb) * C[i, a]
        for a in range(3):
            F[k, a] = -p.G * psi[k] * s[a] + rho[k] * p.body_force[a]
    return F


def eq_velocities(rho, j, F, p: Params):
    """Shan-Chen velocity shift.

    u' = sum_k (j_k / tau_k) / sum_k (rho_k / tau_k);
    u_k^eq = u' + tau_k F_k / rho_k  (u' where rho_k < 1e-12).
    """
    num = j[0] / p.tau[0] + j[1] / p.tau[1]
    den = rho[0] / p.tau[0] + rho[1] / p.tau[1]
    den_safe = np.where(den > 0, den, 1.0)
    up = num / den_safe
    ueq = np.empty((2, 3) + rho.shape[1:])
    for k in range(2):
        ok = rho[k] >= 1e-12
        r = np.where(ok, rho[k], 1.0)
        for a in range(3):
            ueq[k, a] = np.where(ok, up[a] + p.tau[k] * F[k, a] / r, up[a])
    return up, ueq


def physical_velocity(rho, j, F):
    """Observable barycentric velocity u = (sum_k j_k + F/2) / sum_k rho_k."""
    tot = rho[0] + rho[1]
    tot = np.where(tot > 0, tot, 1.0)
    return (j[0] + j[1] + 0.5 * (F[0] + F[1])) / tot


def pull_stream(fpost, material, p: Params, rod_link=None):
    """Pull streaming f_i(x, t+1) = f*_i(x - c_i, t) with boundary rules.

    Source s = x - c_i of a fluid node x:
      fluid          -> f*_i(s)
      static solid   -> f*_ibar(x)                       (halfway bounce-back)
      rod            -> f*_ibar(x) + rod_link(...)        (moving bounce-back)
      ghost          -> w_i rho_top_k                      (reservoir)
    Returns (f_new, ledger_delta[2]) where ledger_delta is the mass that left
    the fluid into the reservoir minus the mass that came in from it.
    """
    fluid = material == FLUID
    fnew = np.zeros_like(fpost)
    ledger = np.zeros(2)
    for i in range(Q):
        src_mat = _shift(material, C[i])
        from_fluid = src_mat == FLUID
        from_wall = is_static_solid(src_mat)
        from_ghost = src_mat == GHOST
        from_rod = src_mat == ROD
        for k in range(2):
            v = np.where(from_fluid, _shift(fpost[k, i], C[i]), 0.0)
            v = np.where(from_wall | from_rod, fpost[k, OPP[i]], v)
            v = np.where(from_ghost, W[i] * p.rho_top[k], v)
            fnew[k, i] = np.where(fluid, v, 0.0)
            # mass coming in from the reservoir
            ledger[k] -= float(np.sum(np.where(fluid & from_ghost, W[i] * p.rho_top[k], 0.0)))
            # mass leaving a fluid node towards the reservoir
            dst_mat = _ahead(material, C[i])
            ledger[k] += float(np.sum(np.where(fluid & (dst_mat == GHOST), fpost[k, i], 0.0)))
    if rod_link is not None:
        rod_link(fnew, fpost)
    return fnew, ledger


def collide(f, rho, ueq, p: Params):
    """Eq. 1 right-hand side: f* = f - (f - f^eq(rho_k, u_k^eq)) / tau_k."""
    out = np.empty_like(f)
    for k in range(2):
        feq = equilibrium(rho[k], ueq[k])
        out[k] = f[k] - (f[k] - feq) / p.tau[k]
    return out


# --------------------------------------------------------------------------
# Evaporation as an interfacial sink (Methods, evaporation paragraph; Eq. 8)
#
# Readings where the paper is silent: a node is liquid where rho_A > rho_B and
# gas where rho_A < rho_B; the interface node of a column is a liquid fluid
# node whose upper neighbour (z + 1) is a gas fluid node; the local height h
# of a column (x, y) is its number of liquid fluid nodes in the stored state
# the step starts from, h0 the initial apex height; the sink moves
# delta = min(J0 / (K + h / h0), f*_0^A) of the liquid's post-collision rest
# population into the rest population of the gas (component B), so the total
# mass is kept and both ledgers book the transfer.
# --------------------------------------------------------------------------
def column_heights(rho, material):
    """h[y, x]: liquid fluid nodes (rho_A > rho_B) in each column."""
    liquid = (material == FLUID) & (rho[0] > rho[1])
    return liquid.sum(axis=0)


def interface_nodes(rho, material, p: Params):
    """Liquid fluid nodes whose upper neighbour is a gas fluid node."""
    fluid = material == FLUID
    liquid = fluid & (rho[0] > rho[1])
    gas = fluid & (rho[0] < rho[1])
    above = np.roll(gas, -1, axis=0)  # gas at z + 1
    if not p.periodic[2]:
        above[-1] = False
    return liquid & above


def evaporation_sink(fpost, rho, material, h, p: Params):
    """Eq. 8 applied to the post-collision state: at each interface node,
    delta = min(J0 / (K + h / h0), f*_0^A), at least 0, leaves the rest
    population of A for that of B.  Returns (f*, total delta)."""
    iface = interface_nodes(rho, material, p)
    J = p.sink_J0 / (p.sink_K + h / p.sink_h0)
    delta = np.where(iface, np.maximum(np.minimum(J[None], fpost[0, 0]), 0.0), 0.0)
    out = fpost.copy()
    out[0, 0] = fpost[0, 0] - delta
    out[1, 0] = fpost[1, 0] + delta
    return out, float(delta.sum())


def fluid_step(fpost, material, p: Params, rod_link=None):
    """One full step t -> t+1 on the post-collision state.

    Returns (f*(t+1), ledger_delta[2], diagnostics dict).
    """
    fluid = material == FLUID
    if p.sink:
        h = column_heights(fields(fpost, material)[0], material)
    f, dledger = pull_stream(fpost, material, p, rod_link)
    rho = np.empty((2,) + material.shape)
    j = np.empty((2, 3) + material.shape)
    for k in range(2):
        rho[k], j[k] = moments(f[k])
    rho = np.where(fluid, rho, 0.0)
    j = np.where(fluid, j, 0.0)
    psi = pseudopotential(rho, material, p)
    F = sc_force(psi, rho, p)
    F = np.where(fluid, F, 0.0)
    up, ueq = eq_velocities(rho, j, F, p)
    out = collide(f, rho, ueq, p)
    out = np.where(fluid, out, 0.0)
    if p.sink:
        out, moved = evaporation_sink(out, rho, material, h, p)
        dledger = dledger + np.array([moved, -moved])
    return out, dledger, {"rho": rho, "j": j, "F": F, "psi": psi}


def fields(fpost, material):
    """Densities and post-collision barycentric velocity at the stored level.

    rho_k is a collision invariant, so it is read off f*.  The velocity
    returned is (sum_k j*_k) / (sum_k rho_k) of the post-collision momenta.
    """
    fluid = material == FLUID
    rho = np.empty((2,) + material.shape)
    j = np.empty((2, 3) + material.shape)
    for k in range(2):
        rho[k], j[k] = moments(fpost[k])
    rho = np.where(fluid, rho, 0.0)
    j = np.where(fluid, j, 0.0)
    tot = rho[0] + rho[1]
    u = (j[0] + j[1]) / np.where(tot > 0, tot, 1.0)
    return rho, u


def pressure(rho, G):
    """Shan-Chen equation of state p = c_s^2 (rho_1 + rho_2) + G c_s^2 rho_1 rho_2."""
    return CS2 * (rho[0] + rho[1]) + G * CS2 * rho[0] * rho[1]


def check_boundaries(material, p: Params):
    """A non-periodic direction must be closed by non-fluid end planes."""
    px, py, pz = p.periodic
    planes = []
    if not px:
        planes += [material[:, :, 0], material[:, :, -1]]
    if not py:
        planes += [material[:, 0, :], material[:, -1, :]]
    if not pz:
        planes += [material[0], material[-1]]
    for pl in planes:
        if np.any(pl == FLUID):
            raise ValueError("fluid node on the end plane of a non-periodic direction")
    if p.evaporation and not np.all(material[-1] == GHOST):
        raise ValueError("evaporation needs the whole top plane z = nz-1 to be the ghost reservoir")


class Run:
    """Convenience driver: holds the state and ledger of one oracle run."""

    def __init__(self, rho0, material, p: Params):
        self.p = p
        self.material = np.ascontiguousarray(material, dtype=np.uint8)
        check_boundaries(self.material, p)
        self.f = initial_state(np.where(self.material == FLUID, rho0, 0.0))
        self.ledger = np.zeros(2)
        self.t = 0
        self.last = None

    def step(self, n=1):
        for _ in range(n):
            self.f, dl, self.last = fluid_step(self.f, self.material, self.p)
            self.ledger += dl
            self.t += 1
        return self

    def masses(self):
        fluid = self.material == FLUID
        return np.array([float(np.sum(np.where(fluid, self.f[k].sum(axis=0), 0.0))) for k in range(2)])
