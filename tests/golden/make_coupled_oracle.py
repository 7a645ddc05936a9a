"""Expected values of the coupled fluid + rod step over 1000 steps on a
reduced form of the benchmark's droplet: a 96 x 48 x 32 striped cap
(footprint 84 x 36, height 18, stripe 90 x 42, reservoir plane on top,
seeded noise 1e-4 with seed 2300) holding five rods of length 24 and radius
2 placed fully inside the liquid with their centres at most 12 above the
wall (physical placement, seed 2355, gap 4), cohesion eps = 1e-4.  Calls
the oracle only; about 40 minutes.

Written to coupled_cap96_oracle.npz:
  rods_<t>     [5][13] X, q, V, L at t = 100, 250, 500, 750, 1000
  scal_<t>     fluid mass (2), reservoir ledger (2), rod exchange ledger (2)
  nodes        1500 sampled fluid nodes at t = 1000 (flat z-y-x index): 750
               within 3 of a rod surface, 750 uniform (PCG64 seed 2399)
  f_nodes      their populations f[2][19][1500] at t = 1000 (FP64)

Usage: python tests/golden/make_coupled_oracle.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lbm  # noqa: E402
from oracle import rods as R  # noqa: E402
from tests import cases  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "coupled_cap96_oracle.npz")
CHECK = (100, 250, 500, 750, 1000)


def main():
    c = cases.coupled_cap_case()
    nz, ny, nx = c["shape"]
    fp = cases.oracle_params(c)
    rp = R.RodParams(**cases.COUPLED_RODS, wall_z=0.5)
    r0 = c["rods"]
    rods = R.Rods(r0[:, :3], r0[:, 3:7], r0[:, 7:10], r0[:, 10:13], rp, (nx, ny, nz), c["periodic"])
    run = R.CoupledRun(c["rho"], c["mat"], fp, rods)
    out = {}
    for t in range(1, CHECK[-1] + 1):
        run.step()
        if t in CHECK:
            out[f"rods_{t}"] = np.concatenate([run.rods.X, run.rods.q, run.rods.V, run.rods.L], axis=1)
            out[f"scal_{t}"] = np.concatenate([run.fluid_mass(), run.ledger, run.solid])
            print(t, out[f"scal_{t}"], flush=True)
    fl = run.material == lbm.FLUID
    dist = np.full(fl.shape, np.inf)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pts = np.stack([x, y, z], -1).astype(float)
    for r in range(run.rods.n):
        d = pts - run.rods.X[r]
        for a, n in ((0, nx), (1, ny)):
            d[..., a] -= n * np.round(d[..., a] / n)
        e = R.axis(run.rods.q[r])
        t = np.clip(d @ e, -rp.half, rp.half)
        dist = np.minimum(dist, np.sqrt(((d - t[..., None] * e) ** 2).sum(-1)) - rp.radius)
    rng = np.random.Generator(np.random.PCG64(2399))
    near = np.flatnonzero((fl & (dist <= 3.0)).ravel())
    anywhere = np.flatnonzero(fl.ravel())
    nodes = np.union1d(rng.choice(near, 750, replace=False), rng.choice(anywhere, 750, replace=False))
    out["nodes"] = nodes
    out["f_nodes"] = run.f.reshape(2, lbm.Q, -1)[:, :, nodes]
    np.savez_compressed(OUT, **out)
    print(OUT)


if __name__ == "__main__":
    main()
