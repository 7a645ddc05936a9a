"""FP64 oracle: bead-spring filaments coupled to the Shan-Chen fluid.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

The paper models each nanowire as a chain of beads (Methods, filament
paragraphs):

* bonds between neighbouring beads of a chain: FENE (Eq. 9),
  U = -1/2 k_s R_m^2 ln(1 - d^2 / R_m^2), k_s = 0.3, R_m = 2.4;
* excluded volume between every pair of beads: the WCA form (Eq. 10),
  U = eps [(d0/d)^12 - 2 (d0/d)^6] + eps for d <= d0, d0 = 2, eps = 0.03;
* stiffness: a harmonic spring between second neighbours of a chain (Eq. 11),
  U = 1/2 k_b (d - 2 d0)^2, k_b = 8;
* cohesion between beads of different filaments: the Lennard-Jones form of
  Eq. 12 with well depth eps_coh (zero: purely repulsive);
* the substrate: Lennard-Jones adhesion of well depth eps_s = 0.006 between a
  bead and the wall, and friction proportional to the normal load;
* two-way coupling to the fluid by a drag on each bead relative to the local
  fluid velocity, whose momentum goes back to the fluid (Ahlrichs-Duenweg),
  and a solvation force from the local density gradient that keeps beads in
  the liquid;
* five substeps of the beads per lattice Boltzmann step.

The paper leaves the following open; these are the readings taken here (the
design notes list them as well):

* chain: N = L / d0 beads, initially straight at spacing d0; bead mass
  m = pi d0^3 / 6 (a neutrally buoyant sphere of the bead's diameter in the
  liquid of density 1);
* cohesion: U = eps_coh [phi(d) - phi(r_c)] for d0 <= d < r_c and
  eps_coh [phi(d0) - phi(r_c)] below d0 (held at its minimum, so that the
  excluded volume alone acts at short range), phi(d) = (d0/d)^12 - 2 (d0/d)^6,
  r_c = 1.5 d0; not between beads of one chain at most two apart;
* substrate: h = z - z_wall is the height of the bead centre above the wall
  plane; U_s = eps_s [phi_s(h) - phi_s(r_cs)] for h < r_cs with
  phi_s(h) = (sigma/h)^12 - 2 (sigma/h)^6, sigma = d0 / 2 (the bead's surface
  touches the wall at the minimum), r_cs = 2.5 sigma;
* normal load N = max(0, -(z-force on the bead from everything except the
  substrate's repulsive branch)) for a bead with h < r_cs; friction
  F_f = -v_t min(mu N / |v_t|, m / dt) on the tangential velocity v_t (it
  never reverses v_t within a substep), mu = 0.5;
* fluid velocity at a bead: trilinear interpolation over the eight nodes
  around it of the physical velocity u = (sum_k j*_k - F/2) / rho of the
  stored post-collision state (F the Shan-Chen force of its densities, as the
  fused step computed it), taken once per lattice step at the step-start
  position and held over the substeps; non-fluid nodes drop out and the
  remaining weights are renormalised (no fluid node: no coupling);
* drag F_d = -gamma (V - u), gamma = 1;
* solvation F_s = kappa_s grad C interpolated the same way, C = (rho_A -
  rho_B) / (rho_A + rho_B) the colour, grad C = 3 sum_i w_i C(x + c_i) c_i
  with C(x) in place of non-fluid neighbours, kappa_s = 0.05;
* the fluid receives the reactions: the impulse sum over substeps of
  (gamma (V_s - u) - F_s) dt per bead, spread with the same weights onto the
  stored state by the exact-difference rule
  f*_k <- f*_k + f^eq(rho_k, u_k + dp / rho) - f^eq(rho_k, u_k) with
  u_k = j*_k / rho_k (mass kept, momentum dp added exactly);
* substeps: forces at the substep start, V then X (symplectic Euler, as for
  the rods); periodic positions wrapped after each substep;
* step order: fluid step, then the filament update on its output.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lbm


@dataclass
class FilParams:
    n_per: int = 6            # beads per filament (L / d0)
    k_s: float = 0.3          # FENE spring constant (Eq. 9)
    R_m: float = 2.4          # FENE maximum extension (Eq. 9)
    eps: float = 0.03         # excluded volume (Eq. 10)
    d0: float = 2.0           # bead diameter (Eqs. 10-12)
    k_b: float = 8.0          # bending (Eq. 11)
    eps_coh: float = 0.0      # cohesion between filaments (Eq. 12)
    r_cut: float = 3.0        # cohesion cut-off, 1.5 d0
    eps_s: float = 0.006      # substrate adhesion
    sigma_s: float = 1.0      # substrate LJ minimum, d0 / 2
    r_cut_s: float = 2.5      # substrate cut-off, 2.5 sigma_s
    mu: float = 0.5           # friction coefficient
    gamma: float = 1.0        # drag coefficient
    kappa_s: float = 0.05     # solvation strength
    wall_z: float | None = 0.5
    n_sub: int = 5

    @property
    def mass(self):
        return np.pi * self.d0**3 / 6.0


def phi(d, d0):
    """(d0/d)^12 - 2 (d0/d)^6."""
    x6 = (d0 / d) ** 6
    return x6 * x6 - 2.0 * x6


def dphi(d, d0):
    """d phi / d d."""
    x6 = (d0 / d) ** 6
    return 12.0 * (x6 - x6 * x6) / d


def fene_force(d, p):
    """-dU/dd of Eq. 9 (negative: attractive)."""
    return -p.k_s * d / (1.0 - (d / p.R_m) ** 2)


def wca_force(d, p):
    """-dU/dd of Eq. 10 for d <= d0 (positive: repulsive)."""
    return -p.eps * dphi(d, p.d0) if d <= p.d0 else 0.0


def bend_force(d, p):
    """-dU/dd of Eq. 11."""
    return -p.k_b * (d - 2.0 * p.d0)


def cohesion_force(d, p):
    """-dU/dd of the cohesion (zero below d0 and beyond r_c)."""
    if p.eps_coh > 0.0 and p.d0 < d < p.r_cut:
        return -p.eps_coh * dphi(d, p.d0)
    return 0.0


def substrate_force(h, p):
    """-dU_s/dh at height h above the wall plane (z-component)."""
    if 0.0 < h < p.r_cut_s:
        return -p.eps_s * dphi(h, p.sigma_s)
    return 0.0


def min_image(d, box, periodic):
    d = np.array(d, dtype=np.float64)
    for a in range(3):
        if periodic[a]:
            d[a] -= box[a] * np.round(d[a] / box[a])
    return d


class Filaments:
    """n filaments of n_per beads: positions X and velocities V, (n*n_per, 3),
    bead b of filament f at row f * n_per + b; (x, y, z) order."""

    def __init__(self, X, V, p: FilParams, box, periodic):
        self.X = np.array(X, dtype=np.float64).reshape(-1, 3)
        self.V = np.array(V, dtype=np.float64).reshape(-1, 3)
        self.p = p
        self.box = np.array(box, dtype=np.float64)
        self.periodic = tuple(bool(v) for v in periodic)
        assert self.X.shape[0] % p.n_per == 0

    @property
    def n_beads(self):
        return self.X.shape[0]

    def chain_of(self, b):
        return b // self.p.n_per, b % self.p.n_per

    def internal_forces(self):
        """Bonds, bending, excluded volume, cohesion and the substrate's
        force at the current positions; (n, 3) each for the inter-bead part
        and the substrate part (z only)."""
        p = self.p
        n = self.n_beads
        F = np.zeros((n, 3))
        Fs = np.zeros((n, 3))
        for a in range(n):
            fa, ia = self.chain_of(a)
            for b in range(a + 1, n):
                fb, ib = self.chain_of(b)
                r = min_image(self.X[a] - self.X[b], self.box, self.periodic)
                d = float(np.sqrt(r @ r))
                same = fa == fb
                sep = abs(ia - ib) if same else None
                fm = 0.0
                if d <= p.d0:
                    fm += wca_force(d, p)
                if same and sep == 1:
                    fm += fene_force(d, p)
                if same and sep == 2:
                    fm += bend_force(d, p)
                if not same:
                    fm += cohesion_force(d, p)
                if fm != 0.0:
                    f = fm * r / d
                    F[a] += f
                    F[b] -= f
        if p.wall_z is not None:
            for a in range(n):
                Fs[a, 2] = substrate_force(self.X[a, 2] - p.wall_z, p)
        return F, Fs

    def friction(self, Fother, Fs, V):
        """Coulomb friction on beads within the substrate's range."""
        p = self.p
        dt = 1.0 / p.n_sub
        Ff = np.zeros_like(V)
        if p.wall_z is None:
            return Ff
        for a in range(self.n_beads):
            h = self.X[a, 2] - p.wall_z
            if not (0.0 < h < p.r_cut_s):
                continue
            fz = Fother[a, 2] + min(Fs[a, 2], 0.0)  # the substrate's attractive branch counts
            N = max(0.0, -fz)
            vt = np.array([V[a, 0], V[a, 1], 0.0])
            s = float(np.sqrt(vt @ vt))
            if N > 0.0 and s > 0.0:
                Ff[a] = -vt * min(p.mu * N / s, p.mass / dt)
        return Ff


# --------------------------------------------------------------------------
# fluid side: velocity, colour gradient, stencil weights
# --------------------------------------------------------------------------


def stencil(x, shape, periodic):
    """The eight nodes around x (x, y, z order) with trilinear weights:
    [(z, y, x, w)], None for a node outside a closed direction."""
    nz, ny, nx = shape
    base = np.floor(x).astype(int)
    fr = x - base
    out = []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = (fr[0] if dx else 1 - fr[0]) * (fr[1] if dy else 1 - fr[1]) * (fr[2] if dz else 1 - fr[2])
                idx = [base[0] + dx, base[1] + dy, base[2] + dz]
                ok = True
                for a, n in enumerate((nx, ny, nz)):
                    if periodic[a]:
                        idx[a] %= n
                    elif not (0 <= idx[a] < n):
                        ok = False
                out.append((idx[2], idx[1], idx[0], w) if ok else None)
    return out


def fluid_fields(fpost, material, fp: lbm.Params):
    """Physical velocity u (3, ...) and colour C of the stored state, plus
    the densities and post-collision momenta per component."""
    fluid = material == lbm.FLUID
    rho = np.empty((2,) + material.shape)
    js = np.empty((2, 3) + material.shape)
    for k in range(2):
        rho[k], js[k] = lbm.moments(fpost[k])
    rho = np.where(fluid, rho, 0.0)
    js = np.where(fluid, js, 0.0)
    psi = lbm.pseudopotential(rho, material, fp)
    F = np.where(fluid, lbm.sc_force(psi, rho, fp), 0.0)
    tot = rho[0] + rho[1]
    tsafe = np.where(tot > 0, tot, 1.0)
    u = np.where(fluid, (js[0] + js[1] - 0.5 * (F[0] + F[1])) / tsafe, 0.0)
    C = np.where(fluid, (rho[0] - rho[1]) / tsafe, 0.0)
    return u, C, rho, js


def colour_gradient(C, material, periodic):
    """grad C = 3 sum_i w_i C(x + c_i) c_i, C(x) in place of non-fluid
    neighbours (the isotropic lattice gradient); zero on non-fluid nodes."""
    fluid = material == lbm.FLUID
    g = np.zeros((3,) + C.shape)
    for i in range(1, lbm.Q):
        c = lbm.C[i]
        nb = lbm._ahead(C, c)
        nbf = lbm._ahead(fluid, c)
        if not periodic[0] or not periodic[1] or not periodic[2]:
            # a neighbour across a closed face does not exist: use C(x)
            nz, ny, nx = C.shape
            z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
            inside = np.ones(C.shape, bool)
            for a, (n, coord) in enumerate(((nx, x), (ny, y), (nz, z))):
                if not periodic[a]:
                    inside &= (coord + c[a] >= 0) & (coord + c[a] < n)
            nbf = nbf & inside
        v = np.where(nbf, nb, C)
        for a in range(3):
            if c[a] != 0:
                g[a] = g[a] + 3.0 * lbm.W[i] * v * c[a]
    return np.where(fluid[None], g, 0.0)


# --------------------------------------------------------------------------
# coupled fluid + filament step
# --------------------------------------------------------------------------


class FilamentRun:
    """Fluid (oracle.lbm) plus filaments; one step = fluid step, then the
    filament update with its momentum handed back to the fluid."""

    def __init__(self, rho0, material, fp: lbm.Params, fil: Filaments):
        self.fp = fp
        self.material = np.ascontiguousarray(material, dtype=np.uint8)
        self.fil = fil
        self.f = lbm.initial_state(np.where(self.material == lbm.FLUID, rho0, 0.0))
        self.ledger = np.zeros(2)
        self.t = 0
        self.last = None

    def step(self, n=1):
        for _ in range(n):
            self._step()
        return self

    def gather(self):
        """Per bead: the eight stencil entries with renormalised fluid
        weights, the interpolated fluid velocity and colour gradient."""
        fp, fil = self.fp, self.fil
        shape = self.material.shape
        u, C, _, _ = fluid_fields(self.f, self.material, fp)
        gC = colour_gradient(C, self.material, fp.periodic)
        sts, us, gs = [], [], []
        for b in range(fil.n_beads):
            st = [e for e in stencil(fil.X[b], shape, fp.periodic)
                  if e is not None and self.material[e[0], e[1], e[2]] == lbm.FLUID]
            wsum = sum(e[3] for e in st)
            if wsum > 0.0:
                st = [(z, y, x, w / wsum) for z, y, x, w in st]
            else:
                st = []
            ub = np.zeros(3)
            gb = np.zeros(3)
            for z, y, x, w in st:
                ub += w * u[:, z, y, x]
                gb += w * gC[:, z, y, x]
            sts.append(st)
            us.append(ub)
            gs.append(gb)
        return sts, np.array(us).reshape(-1, 3), np.array(gs).reshape(-1, 3)

    def apply_impulse(self, dp):
        """Exact-difference update of the stored state at each node of dp
        ({(z, y, x): momentum})."""
        for (z, y, x), d in dp.items():
            rho = np.array([self.f[k, :, z, y, x].sum() for k in range(2)])
            tot = rho.sum()
            if tot <= 0.0:
                continue
            du = d / tot
            for k in range(2):
                if rho[k] <= 0.0:
                    continue
                _, jk = lbm.moments(self.f[k, :, z, y, x][:, None])
                uk = jk[:, 0] / rho[k]
                new = lbm.equilibrium(np.array([rho[k]]), (uk + du)[:, None])[:, 0]
                old = lbm.equilibrium(np.array([rho[k]]), uk[:, None])[:, 0]
                self.f[k, :, z, y, x] = self.f[k, :, z, y, x] + (new - old)

    @staticmethod
    def reaction(Fd, Fs):
        """Force the fluid receives from a bead that feels drag Fd and
        solvation Fs (their reactions)."""
        return -(Fd + Fs)

    def _step(self):
        fp, fil = self.fp, self.fil
        p = fil.p
        self.f, dled, _ = lbm.fluid_step(self.f, self.material, fp)
        self.ledger += dled
        sts, ub, gb = self.gather()
        dt = 1.0 / p.n_sub
        m = p.mass
        Fsolv = p.kappa_s * gb
        coupled = np.array([len(s) > 0 for s in sts])
        imp = np.zeros((fil.n_beads, 3))
        for _ in range(p.n_sub):
            Fi, Fs = fil.internal_forces()
            Fd = np.where(coupled[:, None], -p.gamma * (fil.V - ub), 0.0)
            Fsv = np.where(coupled[:, None], Fsolv, 0.0)
            Fother = Fi + Fd + Fsv
            Ff = fil.friction(Fother, Fs, fil.V)
            imp += self.reaction(Fd, Fsv) * dt
            fil.V = fil.V + (Fother + Fs + Ff) / m * dt
            fil.X = fil.X + fil.V * dt
            for a in range(3):
                if fp.periodic[a]:
                    fil.X[:, a] = np.mod(fil.X[:, a], fil.box[a])
        dp = {}
        for b in range(fil.n_beads):
            for z, y, x, w in sts[b]:
                dp[(z, y, x)] = dp.get((z, y, x), np.zeros(3)) + w * imp[b]
        self.apply_impulse(dp)
        self.t += 1
        self.last = {"impulse": imp, "u": ub, "gradC": gb, "coupled": coupled}

    # ------------------------------------------------------------ totals --
    def fluid_mass(self):
        fl = self.material == lbm.FLUID
        return np.array([float(np.where(fl, self.f[k].sum(axis=0), 0.0).sum()) for k in range(2)])

    def fluid_momentum(self):
        fl = self.material == lbm.FLUID
        tot = np.zeros(3)
        for k in range(2):
            _, j = lbm.moments(self.f[k])
            tot += np.where(fl[None], j, 0.0).reshape(3, -1).sum(axis=1)
        return tot


def straight_chains(centres, axes, p: FilParams):
    """Bead positions of straight chains at spacing d0 centred at each
    centre along each unit axis: (n * n_per, 3)."""
    out = []
    for c, e in zip(np.asarray(centres, float), np.asarray(axes, float)):
        e = e / np.linalg.norm(e)
        for b in range(p.n_per):
            out.append(c + (b - 0.5 * (p.n_per - 1)) * p.d0 * e)
    return np.array(out)
