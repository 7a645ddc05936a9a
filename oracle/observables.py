"""FP64 oracle of the droplet and deposit observables.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

What it follows
---------------
* Droplet shape (Results, drying dynamics: droplet height, footprint radii
  and contact angles along the axial x and transverse y directions).  The
  paper does not say how these are extracted; the reading used here:
    - colour field C = (rho_A - rho_B) / (rho_A + rho_B) on fluid nodes, the
      liquid is C > 0;
    - column height H(x, y): the topmost fluid node z* with C > 0, plus the
      linear-interpolated C = 0 crossing towards z* + 1, measured from the
      wall surface at z = 1/2 (H = 0 for a dry column); the droplet height h
      is the largest H;
    - footprint half-lengths r_x, r_y on the first fluid plane z = 1, along
      the row / column through the given centre: the run of C > 0 nodes that
      contains the centre node, ends interpolated at C = 0;
    - contact angles from the spherical-cap relation h / r = tan(theta / 2),
      i.e. theta_d = 2 atan(h / r_d) per direction.
* Deposit statistics of the rods (Methods, structural characterisation):
    - each rod is represented by beads evenly spaced along its axis segment
      (spacing about the paper's bead diameter) and by the segments joining
      consecutive beads;
    - g^b (Eq. 14): bead count in bin b over the mean bead count per bin
      (equal bins), inside a central strip of half the patch width;
    - S_x^b (Eq. 13): mean of 2 cos^2(zeta) - 1 over the segments whose
      midpoints fall in bin b, zeta the angle to the axial x direction;
    - axial profiles bin x inside |y - y_c| <= strip_y / 2; transverse
      profiles bin y inside |x - x_c| <= strip_x / 2;
    - the angle brackets of Eqs. 13 and 14 average over independent runs and
      over the mirror images of each run at the droplet centre (Results,
      nematic order and density profile): g^b is the mean of the images'
      normalised profiles, S_x^b the mean over the images with segments in
      the bin.
* Rod contact graph (Methods, electrical network model: filaments connect
  when closer than a cutoff): rods are connected when the distance between
  their axis segments is below r_c; reported are the edge count, the size of
  the largest connected cluster and whether one cluster joins the source
  side x < x_src to the sink side x > x_snk.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lbm
from .rods import axis, min_image, segment_segment


# ---------------------------------------------------------------------------
# droplet shape
# ---------------------------------------------------------------------------
def colour(rho, material):
    """C = (rho_A - rho_B) / (rho_A + rho_B) on fluid nodes, NaN elsewhere."""
    fluid = material == lbm.FLUID
    tot = rho[0] + rho[1]
    with np.errstate(invalid="ignore", divide="ignore"):
        c = (rho[0] - rho[1]) / tot
    return np.where(fluid & (tot > 0), c, np.nan)


def column_heights(rho, material):
    """H[y, x]: interface height above the wall surface z = 1/2 (0 if dry)."""
    C = colour(rho, material)
    nz, ny, nx = C.shape
    H = np.zeros((ny, nx))
    for y in range(ny):
        for x in range(nx):
            col = C[:, y, x]
            wet = [z for z in range(1, nz) if col[z] > 0]
            if not wet:
                continue
            zs = max(wet)
            frac = 0.5
            if zs + 1 < nz and not np.isnan(col[zs + 1]):
                frac = col[zs] / (col[zs] - col[zs + 1])
            H[y, x] = zs + frac - 0.5
    return H


def _run_half_length(line, centre):
    """Half-length of the run of line > 0 containing index `centre`, with the
    ends at the linear C = 0 crossings (0 if line[centre] <= 0)."""
    n = len(line)
    if not line[centre] > 0:
        return 0.0
    lo = centre
    while lo - 1 >= 0 and line[lo - 1] > 0:
        lo -= 1
    hi = centre
    while hi + 1 < n and line[hi + 1] > 0:
        hi += 1
    left = lo - 0.5
    if lo - 1 >= 0 and not np.isnan(line[lo - 1]):
        left = lo - line[lo] / (line[lo] - line[lo - 1])
    right = hi + 0.5
    if hi + 1 < n and not np.isnan(line[hi + 1]):
        right = hi + line[hi] / (line[hi] - line[hi + 1])
    return 0.5 * (right - left)


@dataclass
class Droplet:
    height: float
    r_x: float
    r_y: float
    theta_x: float
    theta_y: float
    wet_nodes: int


def droplet_shape(rho, material, xc, yc):
    """Height, footprint half-lengths and contact angles of a sessile droplet."""
    C = colour(rho, material)
    H = column_heights(rho, material)
    h = float(H.max())
    ix, iy = int(round(xc)), int(round(yc))
    rx = _run_half_length(C[1, iy, :], ix)
    ry = _run_half_length(C[1, :, ix], iy)
    tx = 2.0 * np.arctan2(h, rx) if rx > 0 else 0.0
    ty = 2.0 * np.arctan2(h, ry) if ry > 0 else 0.0
    return Droplet(h, rx, ry, tx, ty, int(np.sum(C > 0)))


# ---------------------------------------------------------------------------
# deposit statistics
# ---------------------------------------------------------------------------
@dataclass
class DepositSpec:
    n_bins_x: int
    n_bins_y: int
    xc: float
    yc: float
    strip_x: float  # transverse profiles average over |x - xc| <= strip_x / 2
    strip_y: float  # axial profiles average over |y - yc| <= strip_y / 2
    bead_spacing: float = 2.0
    r_contact: float = 5.25
    x_src: float = 0.0
    x_snk: float = 0.0


def beads(X, q, half, spacing):
    """Bead centres of one rod: nb = max(2, round(2 half / spacing) + 1)
    points evenly spaced from X - half e to X + half e."""
    e = axis(q)
    nb = max(2, int(np.floor(2.0 * half / spacing + 0.5)) + 1)
    t = -half + 2.0 * half * np.arange(nb) / (nb - 1)
    return X[None, :] + t[:, None] * e[None, :], e


def _wrap(v, n):
    return v - n * np.floor(v / n)


def deposit_profiles(X, Q, half, box, spec: DepositSpec, periodic=(True, True, False)):
    """(g_x, S_x(axial), N_x, g_y, S_x(transverse), N_y): Eqs. 14 and 13 on
    equal bins; bins with no segment report S = 0 and N = 0."""
    nx, ny = box[0], box[1]
    gx_cnt = np.zeros(spec.n_bins_x)
    gy_cnt = np.zeros(spec.n_bins_y)
    sx_sum = np.zeros(spec.n_bins_x)
    sy_sum = np.zeros(spec.n_bins_y)
    nsx = np.zeros(spec.n_bins_x, dtype=np.int64)
    nsy = np.zeros(spec.n_bins_y, dtype=np.int64)

    def in_axial_strip(p):
        dy = min_image(np.array([0.0, p[1] - spec.yc, 0.0]), box, periodic)[1]
        return abs(dy) <= 0.5 * spec.strip_y

    def in_transverse_strip(p):
        dx = min_image(np.array([p[0] - spec.xc, 0.0, 0.0]), box, periodic)[0]
        return abs(dx) <= 0.5 * spec.strip_x

    def bin_of(v, n, nb):
        return min(int(np.floor(_wrap(v, n) * nb / n)), nb - 1)

    for r in range(len(X)):
        B, e = beads(np.asarray(X[r], float), np.asarray(Q[r], float), half, spec.bead_spacing)
        s_val = 2.0 * e[0] * e[0] - 1.0
        for p in B:
            if in_axial_strip(p):
                gx_cnt[bin_of(p[0], nx, spec.n_bins_x)] += 1
            if in_transverse_strip(p):
                gy_cnt[bin_of(p[1], ny, spec.n_bins_y)] += 1
        for m in range(len(B) - 1):
            mid = 0.5 * (B[m] + B[m + 1])
            if in_axial_strip(mid):
                b = bin_of(mid[0], nx, spec.n_bins_x)
                sx_sum[b] += s_val
                nsx[b] += 1
            if in_transverse_strip(mid):
                b = bin_of(mid[1], ny, spec.n_bins_y)
                sy_sum[b] += s_val
                nsy[b] += 1

    def norm(cnt):
        mean = cnt.mean()
        return cnt / mean if mean > 0 else np.zeros_like(cnt)

    Sx = np.where(nsx > 0, sx_sum / np.maximum(nsx, 1), 0.0)
    Sy = np.where(nsy > 0, sy_sum / np.maximum(nsy, 1), 0.0)
    return norm(gx_cnt), Sx, nsx, norm(gy_cnt), Sy, nsy


def mirror_rods(X, Q, xc, yc, mx, my):
    """Mirror image of a rod configuration at the droplet centre: x -> 2 xc - x
    when mx, y -> 2 yc - y when my (centres and axes; a rod is symmetric end
    to end, so the reflected axis direction serves as its axis)."""
    Xm = np.array(X, dtype=np.float64).copy()
    Em = np.array([axis(np.asarray(q, float)) for q in Q])
    if mx:
        Xm[:, 0] = 2.0 * xc - Xm[:, 0]
        Em[:, 0] = -Em[:, 0]
    if my:
        Xm[:, 1] = 2.0 * yc - Xm[:, 1]
        Em[:, 1] = -Em[:, 1]
    return Xm, Em


def _quat_of_axis(e):
    """Unit quaternion turning e_z into e (the rod's axis is all the profiles use)."""
    e = np.asarray(e, float) / np.linalg.norm(e)
    if e[2] < -1.0 + 1e-12:
        return np.array([0.0, 1.0, 0.0, 0.0])
    q = np.array([1.0 + e[2], -e[1], e[0], 0.0])
    return q / np.linalg.norm(q)


def ensemble_profiles(runs, half, box, spec: DepositSpec, mirror=True, periodic=(True, True, False)):
    """Profiles averaged over independent runs and, with mirror, over each
    run's mirror images at the droplet centre (x, y and both reflected): the
    angle brackets of Eqs. 13 and 14.  runs: list of (X, Q) rod sets.
    g^b is the mean over all images of each image's normalised bead profile;
    S_x^b the mean over the images that have segments in bin b of their bin
    means (0 where none has); N^b the segments of bin b summed over images.
    Returns (g_x, S_x, N_x, g_y, S_y, N_y)."""
    images = [(0, 0), (1, 0), (0, 1), (1, 1)] if mirror else [(0, 0)]
    acc = None
    for X, Q in runs:
        for mx, my in images:
            Xm, Em = mirror_rods(X, Q, spec.xc, spec.yc, mx, my)
            Qm = [_quat_of_axis(e) for e in Em]
            prof = deposit_profiles(Xm, Qm, half, box, spec, periodic)
            if acc is None:
                acc = {"g": [np.zeros_like(prof[0]), np.zeros_like(prof[3])],
                       "s": [np.zeros_like(prof[1]), np.zeros_like(prof[4])],
                       "ns": [np.zeros_like(prof[2]), np.zeros_like(prof[5])],
                       "cnt": [np.zeros_like(prof[1]), np.zeros_like(prof[4])], "m": 0}
            for d, (g, S, N) in enumerate(((prof[0], prof[1], prof[2]), (prof[3], prof[4], prof[5]))):
                acc["g"][d] += g
                acc["s"][d] += np.where(N > 0, S, 0.0)
                acc["cnt"][d] += N > 0
                acc["ns"][d] += N
            acc["m"] += 1
    out = []
    for d in range(2):
        c = acc["cnt"][d]
        out += [acc["g"][d] / acc["m"], np.where(c > 0, acc["s"][d] / np.maximum(c, 1), 0.0), acc["ns"][d]]
    return tuple(out)


def rod_column_map(material):
    """z-projected rod occupancy: number of rod nodes in each (y, x) column."""
    return (material == lbm.ROD).sum(axis=0).astype(np.int32)


@dataclass
class Graph:
    edges: int
    largest: int
    spanning: bool
    labels: np.ndarray
    pairs: list


def contact_graph(X, Q, half, box, periodic, r_contact, x_src, x_snk):
    """Rods connected when their axis segments are closer than r_contact
    (minimum image); clusters by breadth-first search."""
    n = len(X)
    adj = [[] for _ in range(n)]
    pairs = []
    for a in range(n):
        ea = axis(Q[a])
        pa, qa = X[a] - half * ea, X[a] + half * ea
        for b in range(a + 1, n):
            eb = axis(Q[b])
            d = min_image(X[b] - X[a], box, periodic)
            Xb = X[a] + d
            dist = segment_segment(pa, qa, Xb - half * eb, Xb + half * eb)[0]
            if dist < r_contact:
                adj[a].append(b)
                adj[b].append(a)
                pairs.append((a, b))
    labels = -np.ones(n, dtype=np.int64)
    for s in range(n):
        if labels[s] >= 0:
            continue
        labels[s] = s
        todo = [s]
        while todo:
            u = todo.pop()
            for v in adj[u]:
                if labels[v] < 0:
                    labels[v] = s
                    todo.append(v)
    sizes = np.bincount(labels, minlength=n) if n else np.zeros(0, int)
    largest = int(sizes.max()) if n else 0
    spanning = False
    for lab in set(labels.tolist()):
        members = np.nonzero(labels == lab)[0]
        xs_lo = [min(X[m][0] - half * abs(axis(Q[m])[0]), X[m][0] + half * abs(axis(Q[m])[0])) for m in members]
        xs_hi = [max(X[m][0] - half * abs(axis(Q[m])[0]), X[m][0] + half * abs(axis(Q[m])[0])) for m in members]
        if min(xs_lo) < x_src and max(xs_hi) > x_snk:
            spanning = True
    return Graph(len(pairs), largest, spanning, labels, pairs)
