"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module builds initial density fields, material maps and rod lists.  It
holds geometry and random numbers only -- none of the lattice Boltzmann
arithmetic -- so that the HIP path and the oracle can both start from the
same data without sharing any of the method's code.

Random numbers come from ``numpy.random.Generator(PCG64(seed))``; the order
of every draw is fixed and documented per function.

Material codes: 0 fluid, 1 top reservoir plane, 2 hydrophilic stripe,
3 hydrophobic surround, 8 rod.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

FLUID, GHOST, STRIPE, SURROUND, ROD = 0, 1, 2, 3, 8


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def add_noise(rho, amplitude, seed):
    """Independent U[-a, a] on every rho_k at every node, drawn in [k][z][y][x] order."""
    if amplitude == 0:
        return rho
    return rho + _rng(seed).uniform(-amplitude, amplitude, size=rho.shape)


def sphere_droplet(shape, radius, rho_in=1.0, rho_out=0.03, noise=1e-4, seed=1000):
    """Static spherical droplet in a periodic box.

    Node (x, y, z) is inside iff |x - c| <= R with c = (n/2 - 1/2) per axis.
    Component A: rho_in inside, rho_out outside; component B mirrored.
    Returns (rho[2, nz, ny, nx] float64, material[nz, ny, nx] uint8).
    """
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d2 = (x - (nx / 2 - 0.5)) ** 2 + (y - (ny / 2 - 0.5)) ** 2 + (z - (nz / 2 - 0.5)) ** 2
    ins = d2 <= radius * radius
    rho = np.empty((2,) + tuple(shape))
    rho[0] = np.where(ins, rho_in, rho_out)
    rho[1] = np.where(ins, rho_out, rho_in)
    rho = add_noise(rho, noise, seed)
    return rho, np.zeros(shape, np.uint8)


@dataclass
class CapSpec:
    """Ellipsoidal sessile cap on a wall with a wettable stripe and a reservoir top."""

    shape: tuple = (64, 128, 256)  # (nz, ny, nx)
    footprint: tuple = (150.0, 36.0)  # full lengths along x, y
    height: float = 24.0
    stripe: tuple = (160, 40)  # full lengths along x, y
    rho_in: float = 1.0
    rho_out: float = 0.03
    noise: float = 1e-4
    seed: int = 2000
    reservoir: bool = True


def sessile_cap(spec: CapSpec):
    """Elongated droplet on a patterned wall.

    Wall plane z = 0 (surround material, stripe of full size stripe[0] x
    stripe[1] centred at ((nx-1)/2, (ny-1)/2)); reservoir plane z = nz-1 when
    ``spec.reservoir``; x and y periodic.  Cap: ((x-cx)/a)^2 + ((y-cy)/b)^2 +
    ((z-1/2)/h)^2 <= 1 for z >= 1 with a, b the footprint half-lengths and h
    the height (the wall surface sits at z = 1/2).
    """
    nz, ny, nx = spec.shape
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a, b = spec.footprint[0] / 2.0, spec.footprint[1] / 2.0
    ins = ((x - cx) / a) ** 2 + ((y - cy) / b) ** 2 + ((z - 0.5) / spec.height) ** 2 <= 1.0
    ins &= z >= 1
    mat = np.zeros(spec.shape, np.uint8)
    mat[0] = SURROUND
    sx, sy = spec.stripe
    in_stripe = (np.abs(x[0] - cx) <= sx / 2.0) & (np.abs(y[0] - cy) <= sy / 2.0)
    mat[0][in_stripe] = STRIPE
    if spec.reservoir:
        mat[-1] = GHOST
    rho = np.empty((2,) + tuple(spec.shape))
    rho[0] = np.where(ins, spec.rho_in, spec.rho_out)
    rho[1] = np.where(ins, spec.rho_out, spec.rho_in)
    rho = add_noise(rho, spec.noise, spec.seed)
    solid = mat != FLUID
    rho[:, solid] = 0.0
    return rho, mat


def channel(shape, rho=1.0):
    """Single-component channel between walls at z = 0 and z = nz-1 (Poiseuille)."""
    nz, ny, nx = shape
    mat = np.zeros(shape, np.uint8)
    mat[0] = SURROUND
    mat[-1] = SURROUND
    r = np.zeros((2,) + tuple(shape))
    r[0] = rho
    r[:, mat != FLUID] = 0.0
    return r, mat


# ---------------------------------------------------------------------------
# rods: random sequential placement of capsules
# ---------------------------------------------------------------------------


def _quat_from_axis(e):
    """Unit quaternion (w, x, y, z) of the shortest rotation taking e_z to e."""
    e = np.asarray(e, dtype=np.float64)
    e = e / np.linalg.norm(e)
    if e[2] < -1.0 + 1e-12:
        return np.array([0.0, 1.0, 0.0, 0.0])
    q = np.array([1.0 + e[2], -e[1], e[0], 0.0])
    return q / np.linalg.norm(q)


def _seg_dists(p1, q1, P2, Q2, samples=41):
    """Distances from segment [p1, q1] to segments [P2[m], Q2[m]]: dense
    sampling of the first, exact projection onto each of the others."""
    s = np.linspace(0.0, 1.0, samples)[:, None, None]
    pts = p1[None, None, :] + s * (q1 - p1)[None, None, :]  # (S, 1, 3)
    d2 = (Q2 - P2)[None]  # (1, M, 3)
    L2 = np.maximum((d2 * d2).sum(-1), 1e-300)
    t = np.clip(((pts - P2[None]) * d2).sum(-1) / L2, 0.0, 1.0)
    c = P2[None] + t[..., None] * d2
    return np.sqrt(((pts - c) ** 2).sum(-1)).min(axis=0)


def place_rods(n_req, length, radius, box, inside=None, seed=3000, gap=1.0, margin=3.0, zmin=None,
               max_trials=200000):
    """Random sequential placement of capsule rods.

    box: (nx, ny, nz).  Each trial draws a centre uniform in the box (3
    uniforms) and an axis from a normalised Gaussian triplet (3 normals), in
    that order, from PCG64(seed).  A trial is accepted when
      * ``inside`` is None (stress placement), or every point within
        ``radius + margin`` of the axis (sampled) satisfies ``inside(x, y, z)``
        (physical placement: fully immersed);
      * the lowest axis point is at least ``zmin`` (default radius + 2.5 above
        the wall plane z = 1/2);
      * the axis segment is at least 2 radius + gap from every placed rod.
    Stops after n_req rods or max_trials trials.  Returns an [n][13] array:
    centre, quaternion (w, x, y, z), zero velocity, zero angular momentum.
    """
    rng = _rng(seed)
    nx, ny, nz = box
    half = 0.5 * (length - 2.0 * radius)
    zmin = 0.5 + radius + 2.5 if zmin is None else zmin
    placed = []
    ends = []
    ring = [np.array([np.cos(a), np.sin(a)]) for a in np.linspace(0, 2 * np.pi, 8, endpoint=False)]
    for _ in range(max_trials):
        if len(placed) >= n_req:
            break
        c = rng.uniform(0.0, 1.0, 3) * np.array([nx, ny, nz], dtype=np.float64)
        e = rng.normal(size=3)
        e /= np.linalg.norm(e)
        a, b = c - half * e, c + half * e
        if min(a[2], b[2]) < zmin or max(a[2], b[2]) > nz - 1.5 - radius - 2.5:
            continue
        if inside is not None:
            u = np.cross(e, [1.0, 0, 0] if abs(e[0]) < 0.9 else [0, 1.0, 0])
            u /= np.linalg.norm(u)
            v = np.cross(e, u)
            ok = True
            for s in np.linspace(-half - radius - margin, half + radius + margin, 13):
                base = c + np.clip(s, -half, half) * e
                reach = radius + margin
                pts = [base + s_e * e for s_e in (0.0,)] + [base + reach * (r[0] * u + r[1] * v) for r in ring]
                if abs(s) > half:
                    pts.append(c + np.sign(s) * (half + reach) * e)
                if not all(inside(*p) for p in pts):
                    ok = False
                    break
            if not ok:
                continue
        if ends:
            PA = np.array([pa for pa, _ in ends])
            PB = np.array([pb for _, pb in ends])
            # minimum image in x and y (periodic); rods stay clear of the z ends
            mid = 0.5 * (PA + PB)
            shift = np.zeros_like(mid)
            shift[:, 0] = nx * np.round((c[0] - mid[:, 0]) / nx)
            shift[:, 1] = ny * np.round((c[1] - mid[:, 1]) / ny)
            if np.any(_seg_dists(a, b, PA + shift, PB + shift) < 2.0 * radius + gap):
                continue
        placed.append(np.concatenate([c, _quat_from_axis(e), np.zeros(6)]))
        ends.append((a, b))
    return np.array(placed).reshape(-1, 13)


def deposit_rods(n, x_range, y_range, z, seed=5000):
    """A dried deposit's rods: n rods lying on the substrate, axes in the xy
    plane at height z, centres uniform in x_range x y_range and directions at
    a uniform angle.  Draws per rod from PCG64(seed): centre x, centre y
    (2 uniforms), angle (1 uniform), in that order.  Rods may cross (a
    deposit's rods lie on each other).  Returns an [n][13] array: centre,
    quaternion (w, x, y, z), zero velocity, zero angular momentum."""
    rng = _rng(seed)
    out = np.zeros((n, 13))
    for r in range(n):
        cx = x_range[0] + (x_range[1] - x_range[0]) * rng.random()
        cy = y_range[0] + (y_range[1] - y_range[0]) * rng.random()
        phi = 2.0 * np.pi * rng.random()
        out[r, :3] = (cx, cy, z)
        out[r, 3:7] = _quat_from_axis((np.cos(phi), np.sin(phi), 0.0))
    return out


def place_filaments(n_req, n_per, spacing, box, inside=None, seed=3500, clearance=2.5, margin=1.0, zmin=2.0,
                    max_trials=100000):
    """Random sequential placement of straight bead chains.

    box: (nx, ny, nz).  Each trial draws a centre uniform in the box (3
    uniforms) and an axis from a normalised Gaussian triplet (3 normals), in
    that order, from PCG64(seed); the chain's n_per beads sit at
    centre + (b - (n_per - 1) / 2) spacing axis.  A trial is accepted when
    every bead is at least ``zmin`` above z = 0 and below nz - 1 - zmin,
    ``inside`` (if given) holds at each bead and at the six points ``margin``
    away from it along the axes, and every bead is at least ``clearance``
    from every bead already placed (minimum image in x and y).  Stops after
    n_req chains or max_trials trials.  Returns [n * n_per][6]: positions
    (x, y, z) and zero velocities.
    """
    rng = _rng(seed)
    nx, ny, nz = box
    offs = (np.arange(n_per) - 0.5 * (n_per - 1)) * spacing
    placed = []
    for _ in range(max_trials):
        if len(placed) >= n_req:
            break
        c = rng.uniform(0.0, 1.0, 3) * np.array([nx, ny, nz], dtype=np.float64)
        e = rng.normal(size=3)
        e /= np.linalg.norm(e)
        beads = c[None, :] + offs[:, None] * e[None, :]
        if beads[:, 2].min() < zmin or beads[:, 2].max() > nz - 1 - zmin:
            continue
        if inside is not None:
            ok = True
            for q in beads:
                for d in ([0, 0, 0], [margin, 0, 0], [-margin, 0, 0], [0, margin, 0], [0, -margin, 0],
                          [0, 0, margin], [0, 0, -margin]):
                    if not inside(*(q + np.array(d, dtype=np.float64))):
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                continue
        if placed:
            other = np.concatenate(placed)
            d = beads[:, None, :] - other[None, :, :]
            d[..., 0] -= nx * np.round(d[..., 0] / nx)
            d[..., 1] -= ny * np.round(d[..., 1] / ny)
            if np.sqrt((d * d).sum(-1)).min() < clearance:
                continue
        beads[:, 0] %= nx
        beads[:, 1] %= ny
        placed.append(beads)
    if not placed:
        return np.zeros((0, 6))
    X = np.concatenate(placed)
    return np.concatenate([X, np.zeros_like(X)], axis=1)


def cap_inside(spec: CapSpec):
    """Membership test of the sessile cap of ``sessile_cap`` (continuous coordinates)."""
    nz, ny, nx = spec.shape
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    a, b = spec.footprint[0] / 2.0, spec.footprint[1] / 2.0

    def inside(x, y, z):
        return z >= 1.0 and ((x - cx) / a) ** 2 + ((y - cy) / b) ** 2 + ((z - 0.5) / spec.height) ** 2 <= 1.0

    return inside


def sweep_droplets(n=64, seed0=4000, rods=True, placement="stress", first=0, run=0):
    """Parameter sweep of sessile caps of uneven size (many-droplet batches).

    Droplet i (seed seed0 + i): NX from (128, 160, 192, 224, 256) in turn,
    NY = NX / 2, NZ = 48 + 16 (NX - 128) / 128; from PCG64(seed0 + i), in
    this order: footprint aspect ratio U[1, 4], rod length from (12, 24, 48),
    cohesion depth from (0, 5e-5, 1e-4, 2e-4), rod count U{50..400}.  The cap
    footprint is 0.6 NX long (x) and 0.6 NX / aspect wide (y), its height
    min(0.4 NZ, 0.66 width); the stripe is the footprint plus 10 nodes on
    every side (clipped to the lattice).  Rods: the drawn count placed
    anywhere in the fluid (stress placement, place_rods with inside=None,
    seed seed0 + 500 + i, 3 trials per requested rod), or with
    placement="physical" as many of them as fit fully inside the cap with a
    one-node margin (seed seed0 + 500 + i, 20 trials per requested rod).
    Yields dicts with shape, rho, mat, rods, rod_length, eps_att, aspect for
    droplets first .. n - 1.  run > 0 gives an independent run of the same
    droplets: the same shape and parameters, the cap's noise drawn with seed
    seed0 + i + 1000 run and the rods placed with seed seed0 + 500 + i +
    1000 run.
    """
    for i in range(first, n):
        nx = (128, 160, 192, 224, 256)[i % 5]
        ny, nz = nx // 2, 48 + 16 * (nx - 128) // 128
        rng = _rng(seed0 + i)
        ar = rng.uniform(1.0, 4.0)
        length = (12.0, 24.0, 48.0)[int(rng.integers(3))]
        eps = (0.0, 5e-5, 1e-4, 2e-4)[int(rng.integers(4))]
        n_rods = int(rng.integers(50, 401))
        fx = 0.6 * nx
        fy = fx / ar
        spec = CapSpec(shape=(nz, ny, nx), footprint=(fx, fy), height=min(0.4 * nz, 0.66 * fy),
                       stripe=(min(fx + 20.0, nx), min(fy + 20.0, ny)), seed=seed0 + i + 1000 * run)
        rho, mat = sessile_cap(spec)
        r = None
        if rods and placement == "physical":
            r = place_rods(n_rods, length, 2.0, (nx, ny, nz), inside=cap_inside(spec),
                           seed=seed0 + 500 + i + 1000 * run, margin=1.0, max_trials=20 * n_rods)
        elif rods:
            r = place_rods(n_rods, length, 2.0, (nx, ny, nz), inside=None, seed=seed0 + 500 + i + 1000 * run,
                           max_trials=3 * n_rods)
        yield dict(shape=(nz, ny, nx), rho=rho, mat=mat, rods=r, rod_length=length, eps_att=eps, aspect=ar)
