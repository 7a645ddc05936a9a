"""FP64 oracle of the deposit's resistor network (Methods, electrical
characterisation, Eqs. 15-18).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

What it follows
---------------
* Nodes are beads.  Two beads i, j are joined when their distance r_ij is
  below the cutoff r_c; the edge conductance is G_ij = 1 / r_ij.  Readings:
  the edge decision is taken on squared distances, 0 < r_ij^2 < r_c^2 with
  r_ij^2 = (dx^2 + dy^2) + dz^2 in FP64 (coincident beads are not joined);
  distances are plain Euclidean (the electrodes along x break any periodic
  wrap, so the network has no periodic images).
* Electrodes: beads with x < x_src are held at the potential dV (source),
  beads with x > x_snk at 0 (sink).  The other potentials follow from
  Kirchhoff's current law, sum_j G_ij (V_i - V_j) = 0 at every free bead.
  Free beads with no path to an electrode have no defined potential; the
  reading takes V = 0 there (they carry no current).
* Eq. 15: I_i = 1/2 sum_j |I_ij| with I_ij = G_ij (V_i - V_j).
* I_tot: the current leaving the source electrode, summed over the edges
  from source beads to beads outside it.
* Eq. 16 with kappa_0 A = 1: I_ref = dV / L, L = x_snk - x_src -- the current
  an ideal straight chain of beads across the gap carries (its resistances
  r_ij add up to L).  Eq. 18 for one deposit: kappa* = I_tot / I_ref (the
  average over deposits is the caller's).

Rods are turned into beads as for the deposit profiles: nb = max(2,
floor(2 h / spacing + 1/2) + 1) beads evenly along the axis segment of
half-length h = L_rod/2 - R, centred on the rod's stored centre.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse import csgraph
from scipy.sparse.linalg import spsolve


def rod_beads(X, axes, half, spacing):
    """Bead positions [n_rods * nb, 3], rod by rod, beads from -h to +h."""
    X = np.asarray(X, float).reshape(-1, 3)
    axes = np.asarray(axes, float).reshape(-1, 3)
    nb = max(2, int(np.floor(2.0 * half / spacing + 0.5)) + 1)
    out = []
    for r in range(len(X)):
        for j in range(nb):
            t = -half + 2.0 * half * j / (nb - 1)
            out.append(X[r] + t * axes[r])
    return np.array(out).reshape(-1, 3), nb


def edges(pos, r_c):
    """All joined pairs i < j and their conductances (brute force)."""
    pos = np.asarray(pos, float)
    n = len(pos)
    rc2 = r_c * r_c
    ii, jj, gg = [], [], []
    for i in range(n):
        d = pos[i + 1:] - pos[i]
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        sel = np.nonzero((r2 > 0.0) & (r2 < rc2))[0]
        ii.extend([i] * len(sel))
        jj.extend((i + 1 + sel).tolist())
        gg.extend((1.0 / np.sqrt(r2[sel])).tolist())
    return np.array(ii, int), np.array(jj, int), np.array(gg, float)


def kirchhoff(pos, r_c, x_src, x_snk, dV=1.0):
    """Potentials V, node currents I (Eq. 15), I_tot, I_ref, kappa* and the
    edge count for the beads `pos` [n, 3]."""
    pos = np.asarray(pos, float).reshape(-1, 3)
    n = len(pos)
    if not x_src < x_snk:
        raise ValueError("x_src must lie below x_snk")
    i, j, g = edges(pos, r_c)
    G = sp.coo_matrix((np.concatenate([g, g]), (np.concatenate([i, j]), np.concatenate([j, i]))), shape=(n, n)).tocsr()
    Lap = (sp.diags(np.asarray(G.sum(axis=1)).ravel()) - G).tocsr()
    src = pos[:, 0] < x_src
    snk = pos[:, 0] > x_snk
    free = ~(src | snk)
    V = np.zeros(n)
    V[src] = dV
    # free beads joined to an electrode through free beads: the solvable part
    ncomp, lab = csgraph.connected_components(G, directed=False)
    touches = np.zeros(ncomp, bool)
    touches[np.unique(lab[~free])] = True
    solve = free & touches[lab]
    idx = np.nonzero(solve)[0]
    if len(idx):
        A = Lap[idx][:, idx]
        b = -(Lap[idx][:, np.nonzero(~free)[0]] @ V[~free])
        V[idx] = spsolve(A.tocsc(), b) if len(idx) > 1 else b / A.toarray()[0, 0]
    dVe = V[i] - V[j]
    I = np.zeros(n)
    np.add.at(I, i, 0.5 * g * np.abs(dVe))
    np.add.at(I, j, 0.5 * g * np.abs(dVe))
    # current leaving the source: edges with exactly one end in it
    out_ij = src[i] & ~src[j]
    out_ji = src[j] & ~src[i]
    I_tot = float(np.sum(g[out_ij] * dVe[out_ij]) - np.sum(g[out_ji] * dVe[out_ji]))
    I_ref = dV / (x_snk - x_src)
    return dict(V=V, I=I, I_tot=I_tot, I_ref=I_ref, kappa=I_tot / I_ref, edges=len(g), n_source=int(src.sum()),
                n_sink=int(snk.sum()))
