"""FP64 oracle: rigid capsule rods coupled to the Shan-Chen fluid.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

The paper's nanowires are bead-spring filaments (Methods: FENE bonds, Eq. 9;
excluded volume, Eq. 10; bending, Eq. 11; Lennard-Jones cohesion, Eq. 12;
five particle substeps per lattice Boltzmann step).  Here they are rigid
capsules, the stiff limit of the filament, coupled to the fluid by moving
bounce-back on every boundary link:

* Shape: tip-to-tip length L, radius R; a node belongs to the rod iff the
  distance from its centre to the axis segment (half-length (L - 2R)/2 about
  the centre X along the unit axis e) is <= R.
* Moving bounce-back: for a fluid node x whose pull source s = x - c_i is a
  rod node, f_i(x, t+1) = f*_ibar(x, t) + 2 w_i rho_k(x) (c_i . u_b) / c_s^2
  with u_b = V + Omega x (x_b - X) at the link midpoint x_b = x - c_i / 2
  (minimum image).  The rod receives dP = -c_i (f*_ibar(x) + f_i(x, t+1)).
* Wetting: rod nodes carry the ghost pseudo-densities psi^s(rod); the rod
  receives the reaction to the adhesion force its nodes exert on the fluid.
* Pair forces (segment-segment closest points, distance d): excluded volume
  U_WCA(d) = e_rep [(d0/d)^12 - 2 (d0/d)^6] + e_rep for d <= d0 (Eq. 10)
  plus cohesion eps [(d0/d)^12 - 2 (d0/d)^6] (Eq. 12) truncated and shifted
  to zero at r_c and held at its minimum value for d < d0.
* Rod-wall: the same WCA form between the lowest axis point and the wall
  plane z = 1/2 with its own d0.
* Time integration: five substeps per lattice step (Methods), dt = 1/5,
  hydrodynamic force and torque held fixed; symplectic Euler for V, X and the
  angular momentum L; omega = I^-1 L for a solid cylinder; orientation by the
  quaternion exponential map.
* Re-mask after the move: a node the rod now covers gives its fluid mass to
  the solid-exchange ledger and its momentum to the rod; a node it uncovers
  gets f^eq(rho_bar, u_b) with rho_bar the mean density of its fluid
  neighbours (fluid before and after the move), paid for by the rod and the
  ledger.  A node with no such neighbour -- a pocket enclosed by touching
  capsules -- takes the mean over the nearest ring x + s c_i (s = 2, 3, ...,
  up to one more than a capsule's diameter plus one) that has fluid nodes.  All transfers of one
  re-mask use the rod state right after the substeps and are applied to the
  rod together.

Readings of the paper and the task that these choices take are listed in the
design notes (rod shape, d0 = 2R + 1, r_c = 1.5 d0, shifted cohesion, wall
WCA, cover/uncover rule).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lbm

# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------


def quat_mul(a, b):
    """Hamilton product of quaternions (w, x, y, z)."""
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([
        w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
        w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
        w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
        w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2,
    ])


def quat_rotate(q, v):
    """Rotate vector v by unit quaternion q."""
    qv = np.array([0.0, v[0], v[1], v[2]])
    qc = np.array([q[0], -q[1], -q[2], -q[3]])
    return quat_mul(quat_mul(q, qv), qc)[1:]


def axis(q):
    """Rod axis e = R(q) e_z."""
    return quat_rotate(q, np.array([0.0, 0.0, 1.0]))


def min_image(d, box, periodic):
    """Minimum-image displacement (x, y, z order) in the periodic directions."""
    d = np.array(d, dtype=np.float64)
    for a in range(3):
        if periodic[a]:
            d[a] -= box[a] * np.round(d[a] / box[a])
    return d


def point_segment_distance(p, a, b):
    """Distance from point p to segment [a, b] and the closest point."""
    ab = b - a
    L2 = ab @ ab
    t = 0.0 if L2 == 0 else float(np.clip((p - a) @ ab / L2, 0.0, 1.0))
    c = a + t * ab
    return float(np.linalg.norm(p - c)), c


def segment_segment(p1, q1, p2, q2):
    """Closest points of segments [p1, q1] and [p2, q2].

    Minimises |(p1 + s d1) - (p2 + t d2)|^2 over s, t in [0, 1]: the
    unconstrained stationary point, then clamping one parameter and solving
    for the other (the minimum of a convex quadratic over a square lies on the
    stationary point or on an edge).  Returns (distance, c1, c2, s, t).
    """
    d1, d2, r = q1 - p1, q2 - p2, p1 - p2
    a, e, f = d1 @ d1, d2 @ d2, d2 @ r
    c, b = d1 @ r, d1 @ d2
    cands = []
    den = a * e - b * b
    if den > 1e-14 * max(a * e, 1e-300):
        s = (b * f - c * e) / den
        t = (a * f - b * c) / den
        if 0.0 <= s <= 1.0 and 0.0 <= t <= 1.0:
            cands.append((s, t))
    # edges: s in {0, 1} with t optimal, t in {0, 1} with s optimal
    for s in (0.0, 1.0):
        t = 0.0 if e == 0 else float(np.clip((b * s + f) / e, 0.0, 1.0))
        cands.append((s, t))
    for t in (0.0, 1.0):
        s = 0.0 if a == 0 else float(np.clip((b * t - c) / a, 0.0, 1.0))
        cands.append((s, t))
    best = None
    for s, t in cands:
        c1 = p1 + s * d1
        c2 = p2 + t * d2
        dd = float(np.linalg.norm(c1 - c2))
        if best is None or dd < best[0]:
            best = (dd, c1, c2, s, t)
    return best


# --------------------------------------------------------------------------
# potentials
# --------------------------------------------------------------------------


def lj_form(d, d0):
    """phi(d) = (d0/d)^12 - 2 (d0/d)^6 (Eqs. 10 and 12 without prefactor)."""
    x6 = (d0 / d) ** 6
    return x6 * x6 - 2.0 * x6


def lj_form_deriv(d, d0):
    """d phi / d d."""
    x6 = (d0 / d) ** 6
    return (-12.0 * x6 * x6 + 12.0 * x6) / d


def pair_energy(d, p):
    """Rod-rod energy U(d) = U_WCA + U_cohesion (see module docstring)."""
    u = 0.0
    if d <= p.d0:
        u += p.eps_rep * lj_form(d, p.d0) + p.eps_rep
    if p.eps_att > 0.0 and d < p.r_cut:
        dd = max(d, p.d0)
        u += p.eps_att * (lj_form(dd, p.d0) - lj_form(p.r_cut, p.d0))
    return u


def pair_force_mag(d, p):
    """-dU/dd (positive = repulsive)."""
    f = 0.0
    if d <= p.d0:
        f -= p.eps_rep * lj_form_deriv(d, p.d0)
    if p.eps_att > 0.0 and p.d0 < d < p.r_cut:
        f -= p.eps_att * lj_form_deriv(d, p.d0)
    return f


def wall_force_mag(h, p):
    """-dU/dh of the wall WCA at height h above the wall plane."""
    if h <= p.d0_wall:
        return -p.eps_wall * lj_form_deriv(h, p.d0_wall)
    return 0.0


# --------------------------------------------------------------------------
# rod set
# --------------------------------------------------------------------------


@dataclass
class RodParams:
    length: float = 24.0
    radius: float = 2.0
    rho_rod: float = 1.0
    eps_att: float = 1e-4
    eps_rep: float = 0.03
    d0: float = 5.0
    r_cut: float = 7.5
    eps_wall: float = 0.03
    d0_wall: float = 3.0
    wall_z: float | None = 0.5  # wall plane, None without a wall
    n_sub: int = 5

    @property
    def half(self):
        return 0.5 * (self.length - 2.0 * self.radius)

    @property
    def mass(self):
        return self.rho_rod * np.pi * self.radius**2 * self.length

    @property
    def inertia(self):
        """(I_parallel, I_perpendicular) of a solid cylinder."""
        m, r, L = self.mass, self.radius, self.length
        return 0.5 * m * r * r, m * (3.0 * r * r + L * L) / 12.0


class Rods:
    """State of n rods: X, q (w, x, y, z), V, L (angular momentum)."""

    def __init__(self, X, q, V, Lang, p: RodParams, box, periodic):
        self.X = np.array(X, dtype=np.float64).reshape(-1, 3)
        self.q = np.array(q, dtype=np.float64).reshape(-1, 4)
        self.V = np.array(V, dtype=np.float64).reshape(-1, 3)
        self.L = np.array(Lang, dtype=np.float64).reshape(-1, 3)
        self.p = p
        self.box = np.array(box, dtype=np.float64)  # (nx, ny, nz)
        self.periodic = tuple(bool(v) for v in periodic)

    @property
    def n(self):
        return self.X.shape[0]

    def omega(self, r):
        Ipar, Iperp = self.p.inertia
        e = axis(self.q[r])
        L = self.L[r]
        return L / Iperp + (1.0 / Ipar - 1.0 / Iperp) * (L @ e) * e

    def ends(self, r):
        e = axis(self.q[r])
        return self.X[r] - self.p.half * e, self.X[r] + self.p.half * e

    def velocity_at(self, r, x):
        """Rigid-body velocity V + Omega x (x - X) at lattice position x (min image)."""
        d = min_image(np.asarray(x, dtype=np.float64) - self.X[r], self.box, self.periodic)
        return self.V[r] + np.cross(self.omega(r), d)

    # ---------------------------------------------------------------- mask --
    def mask(self, shape):
        """Rod id per node (-1 none) for lattice shape (nz, ny, nx)."""
        nz, ny, nx = shape
        rid = np.full(shape, -1, dtype=np.int32)
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        pts = np.stack([x, y, z], axis=-1).astype(np.float64)
        for r in range(self.n):
            a, b = self.ends(r)
            # displacement to the centre by minimum image, then distance to the
            # axis segment expressed relative to the centre
            d = pts - self.X[r]
            for ax in range(3):
                if self.periodic[ax]:
                    d[..., ax] -= self.box[ax] * np.round(d[..., ax] / self.box[ax])
            e = axis(self.q[r])
            t = np.clip(d @ e, -self.p.half, self.p.half)
            c = d - t[..., None] * e
            inside = (c * c).sum(-1) <= self.p.radius**2
            rid[inside] = r
        return rid

    # ------------------------------------------------------- pair + wall --
    def contact_forces(self):
        """Pair and wall forces/torques (n, 3) each at the current positions."""
        F = np.zeros((self.n, 3))
        T = np.zeros((self.n, 3))
        p = self.p
        ends = [self.ends(r) for r in range(self.n)]
        for a in range(self.n):
            for b in range(a + 1, self.n):
                shift = min_image(self.X[b] - self.X[a], self.box, self.periodic) - (self.X[b] - self.X[a])
                pa, qa = ends[a]
                pb, qb = ends[b][0] + shift, ends[b][1] + shift
                d, ca, cb, _, _ = segment_segment(pa, qa, pb, qb)
                if d >= max(p.d0, p.r_cut if p.eps_att > 0 else p.d0) or d <= 0.0:
                    continue
                fm = pair_force_mag(d, p)
                if fm == 0.0:
                    continue
                n = (ca - cb) / d
                fa = fm * n
                F[a] += fa
                F[b] -= fa
                T[a] += np.cross(ca - self.X[a], fa)
                T[b] += np.cross(cb - (self.X[b] + shift), -fa)
        if p.wall_z is not None:
            for r in range(self.n):
                a0, b0 = ends[r]
                low = a0 if a0[2] <= b0[2] else b0
                h = low[2] - p.wall_z
                if h <= p.d0_wall and h > 0.0:
                    f = np.array([0.0, 0.0, wall_force_mag(h, p)])
                    F[r] += f
                    T[r] += np.cross(low - self.X[r], f)
        return F, T

    # ------------------------------------------------------------ substeps --
    def integrate(self, F_hyd, T_hyd):
        """n_sub substeps of dt = 1/n_sub with fixed hydrodynamic load."""
        p = self.p
        dt = 1.0 / p.n_sub
        M = p.mass
        for _ in range(p.n_sub):
            Fc, Tc = self.contact_forces()
            F = F_hyd + Fc
            T = T_hyd + Tc
            self.V = self.V + F / M * dt
            self.X = self.X + self.V * dt
            self.L = self.L + T * dt
            for r in range(self.n):
                w = self.omega(r)
                wn = float(np.linalg.norm(w))
                if wn > 0.0:
                    h = 0.5 * wn * dt
                    dq = np.concatenate([[np.cos(h)], np.sin(h) * w / wn])
                    qn = quat_mul(dq, self.q[r])
                    self.q[r] = qn / np.linalg.norm(qn)
            for ax in range(3):
                if self.periodic[ax]:
                    self.X[:, ax] = np.mod(self.X[:, ax], self.box[ax])


# --------------------------------------------------------------------------
# coupled fluid + rod step
# --------------------------------------------------------------------------


def refill_reach(radius):
    """Farthest ring searched for the fluid neighbours of an uncovered node:
    one more than a capsule's diameter plus one, so that a pocket between
    touching capsules always reaches the fluid around them."""
    return int(np.ceil(2.0 * radius)) + 2



class CoupledRun:
    """Fluid (oracle.lbm) plus rods: the coupled step of the drying problem.

    material: static material map (0 fluid, 1 reservoir, 2..7 walls); rod
    nodes are overlaid with code 8 from the rod mask.
    """

    def __init__(self, rho0, material, fp: lbm.Params, rods: Rods):
        self.fp = fp
        self.static = np.ascontiguousarray(material, dtype=np.uint8)
        self.rods = rods
        self.rid = rods.mask(self.static.shape)
        if np.any((self.rid >= 0) & (self.static != lbm.FLUID)):
            raise ValueError("rod overlaps a wall or the reservoir")
        self.material = np.where(self.rid >= 0, lbm.ROD, self.static).astype(np.uint8)
        lbm.check_boundaries(self.static, fp)
        self.f = lbm.initial_state(np.where(self.material == lbm.FLUID, rho0, 0.0))
        self.ledger = np.zeros(2)  # reservoir
        self.solid = np.zeros(2)  # mass exchanged with the rods (fluid -> rods positive)
        self.t = 0
        self.last = None

    def _cvec(self, i):
        return lbm.C[i].astype(np.float64)

    @staticmethod
    def link_term(i, rho_k, ub):
        """Ladd's moving bounce-back addition 2 w_i rho_k (c_i . u_b) / c_s^2."""
        return 2.0 * lbm.W[i] * rho_k * (lbm.C[i].astype(np.float64) @ ub) / lbm.CS2

    def moving_bounce_back(self, fpost, f, rho_t):
        """Rod links of the pull: a fluid node x whose source s = x - c_i is a
        rod node takes f_i(x, t+1) = f*_ibar(x, t) + link_term (u_b the rigid
        velocity at the link midpoint x_b = x - c_i / 2, minimum image).

        Overwrites those entries of the pulled populations f in place and
        returns the rod load (dP, dT: momentum -c_i (f*_ibar + f_i) per link,
        torque about the centre taken at x_b) and the mass the added terms
        carry out of the rods (dsolid[k], negative when the rods push mass
        into the fluid)."""
        rods = self.rods
        nz, ny, nx = self.material.shape
        fluid = self.material == lbm.FLUID
        dP = np.zeros((rods.n, 3))
        dT = np.zeros((rods.n, 3))
        dsolid = np.zeros(2)
        zz, yy, xx = np.nonzero(fluid)
        for i in range(1, lbm.Q):
            c = lbm.C[i]
            sx, sy, sz = (xx - c[0]) % nx, (yy - c[1]) % ny, (zz - c[2]) % nz
            rs = self.rid[sz, sy, sx]
            sel = np.nonzero(rs >= 0)[0]
            ci = self._cvec(i)
            for m in sel:
                x, y, z, r = xx[m], yy[m], zz[m], rs[m]
                xb = np.array([x, y, z], dtype=np.float64) - 0.5 * ci
                ub = rods.velocity_at(r, xb)
                for k in range(2):
                    add = self.link_term(i, rho_t[k, z, y, x], ub)
                    f[k, i, z, y, x] = fpost[k, lbm.OPP[i], z, y, x] + add
                    dsolid[k] -= add
                    dp = -ci * (fpost[k, lbm.OPP[i], z, y, x] + f[k, i, z, y, x])
                    dP[r] += dp
                    dT[r] += np.cross(min_image(xb - rods.X[r], rods.box, rods.periodic), dp)
        return dP, dT, dsolid

    def refill_density(self, node, stay_fluid, rho_now, reach):
        """rho_bar of an uncovered node (x, y, z): the mean density over the
        nodes x + c_i (i = 1..18) that are fluid before and after the move; a
        node with none of them (a pocket enclosed by touching capsules) takes
        the mean over the first ring x + s c_i, s = 2 .. reach, that holds any
        (positions beyond a closed end of a non-periodic direction are
        skipped).  Returns (rho_bar[2], s) with s = 0 and rho_bar = 0 when
        no ring up to `reach` holds a fluid node."""
        nz, ny, nx = stay_fluid.shape
        x, y, z = node
        per = self.fp.periodic
        for s in range(1, reach + 1):
            acc = np.zeros(2)
            cnt = 0
            for i in range(1, lbm.Q):
                q = []
                for v, ci, n, pp in ((z, lbm.C[i][2], nz, per[2]), (y, lbm.C[i][1], ny, per[1]),
                                     (x, lbm.C[i][0], nx, per[0])):
                    w = v + s * int(ci)
                    if pp:
                        w %= n
                    elif not 0 <= w < n:
                        break
                    q.append(w)
                if len(q) == 3 and stay_fluid[q[0], q[1], q[2]]:
                    acc += rho_now[:, q[0], q[1], q[2]]
                    cnt += 1
            if cnt:
                return acc / cnt, s
        return np.zeros(2), 0

    def step(self, n=1):
        for _ in range(n):
            self._step()
        return self

    def _step(self):
        fp, rods = self.fp, self.rods
        shape = self.material.shape
        nz, ny, nx = shape
        n = rods.n
        fpost = self.f
        fluid = self.material == lbm.FLUID
        rho_t = np.array([fpost[k].sum(axis=0) for k in range(2)])  # collision invariant

        # ---- stream with boundaries; moving bounce-back at rod links
        f, dled = lbm.pull_stream(fpost, self.material, fp)
        dP, dT, dsolid = self.moving_bounce_back(fpost, f, rho_t)
        self.solid += dsolid

        # ---- moments, force (rod nodes carry psi^s(rod)), collision
        rho = np.empty((2,) + shape)
        j = np.empty((2, 3) + shape)
        for k in range(2):
            rho[k], j[k] = lbm.moments(f[k])
        rho = np.where(fluid, rho, 0.0)
        j = np.where(fluid, j, 0.0)
        psi = lbm.pseudopotential(rho, self.material, fp)
        F = lbm.sc_force(psi, rho, fp)
        F = np.where(fluid, F, 0.0)
        _, ueq = lbm.eq_velocities(rho, j, F, fp)
        fnew = np.where(fluid, lbm.collide(f, rho, ueq, fp), 0.0)
        # reaction to the adhesion force exerted by rod nodes y = x + c_i
        ps = np.asarray(fp.psi_solid, dtype=np.float64)[lbm.ROD]
        zz, yy, xx = np.nonzero(fluid)
        for i in range(1, lbm.Q):
            c = lbm.C[i]
            ci = self._cvec(i)
            ty, tx, tz = (yy + c[1]) % ny, (xx + c[0]) % nx, (zz + c[2]) % nz
            rn = self.rid[tz, ty, tx]
            for m in np.nonzero(rn >= 0)[0]:
                x, y, z, r = xx[m], yy[m], zz[m], rn[m]
                fr = np.zeros(3)
                for k in range(2):
                    fr += fp.G * psi[k, z, y, x] * lbm.W[i] * ps[1 - k] * ci
                dP[r] += fr
                yb = np.array([tx[m], ty[m], tz[m]], dtype=np.float64)
                dT[r] += np.cross(min_image(yb - rods.X[r], rods.box, rods.periodic), fr)
        self.ledger += dled
        self.f = fnew

        # ---- rods move
        rods.integrate(dP, dT)

        # ---- re-mask: cover and uncover
        new_rid = rods.mask(shape)
        if np.any((new_rid >= 0) & (self.static != lbm.FLUID)):
            raise ValueError("rod moved into a wall or the reservoir")
        old_rid = self.rid
        covered = (old_rid < 0) & (new_rid >= 0)
        uncovered = (old_rid >= 0) & (new_rid < 0)
        stay_fluid = (old_rid < 0) & (new_rid < 0) & (self.static == lbm.FLUID)
        f = self.f
        # all transfers of one re-mask act on the rod state right after the
        # substeps: they are summed per rod and applied together at the end
        dV = np.zeros((n, 3))
        dL = np.zeros((n, 3))
        for z, y, x in zip(*np.nonzero(covered)):
            r = new_rid[z, y, x]
            pos = np.array([x, y, z], dtype=np.float64)
            mom = np.zeros(3)
            for k in range(2):
                rk, jk = lbm.moments(f[k, :, z, y, x][:, None])
                self.solid[k] += rk[0]
                mom += jk[:, 0]
            dV[r] += mom
            dL[r] += np.cross(min_image(pos - rods.X[r], rods.box, rods.periodic), mom)
            f[:, :, z, y, x] = 0.0
        rho_now = np.array([f[k].sum(axis=0) for k in range(2)])
        far = 0
        reach = refill_reach(rods.p.radius)
        for z, y, x in zip(*np.nonzero(uncovered)):
            r = old_rid[z, y, x]
            pos = np.array([x, y, z], dtype=np.float64)
            rbar, s_used = self.refill_density((x, y, z), stay_fluid, rho_now, reach)
            far += s_used > 1
            ub = rods.velocity_at(r, pos)
            mom = np.zeros(3)
            for k in range(2):
                f[k, :, z, y, x] = lbm.equilibrium(np.array([rbar[k]]), ub[:, None])[:, 0]
                self.solid[k] -= rbar[k]
                mom += rbar[k] * ub
            dV[r] -= mom
            dL[r] -= np.cross(min_image(pos - rods.X[r], rods.box, rods.periodic), mom)
        rods.V = rods.V + dV / rods.p.mass
        rods.L = rods.L + dL
        self.rid = new_rid
        self.material = np.where(new_rid >= 0, lbm.ROD, self.static).astype(np.uint8)
        self.f = f
        self.t += 1
        self.last = {"dP": dP, "dT": dT, "covered": int(covered.sum()), "uncovered": int(uncovered.sum()),
                     "far_refills": int(far)}

    # ------------------------------------------------------------ totals --
    def fluid_mass(self):
        fl = self.material == lbm.FLUID
        return np.array([float(np.where(fl, self.f[k].sum(axis=0), 0.0).sum()) for k in range(2)])

    def total_momentum(self):
        fl = self.material == lbm.FLUID
        P = np.zeros(3)
        for k in range(2):
            _, jk = lbm.moments(self.f[k])
            P += np.where(fl, jk, 0.0).sum(axis=(1, 2, 3))
        return P + self.rods.p.mass * self.rods.V.sum(axis=0)
