"""How sensitive the coupled fluid + rod trajectory is to rounding: the FP64
oracle's reduced benchmark droplet (a 96 x 48 x 32 striped cap, reservoir on
top, six rods of length 24 placed fully inside the liquid, seed 2301; one
of them rises until its end pierces the liquid-vapour interface near step
350) run twice, the second time with one initial density changed by 1e-13.
Prints the largest difference of the rod centres every 50 steps.  Calls the
oracle only; about 40 minutes (two processes).

The output is in coupled_sensitivity.txt; no test reads it.  It shows why
the 1000-step parity test keeps its rods clear of the interface: here the
oracle's own two runs part by 1e-2 within 500 steps.

Usage: python tests/golden/oracle_sensitivity.py > tests/golden/coupled_sensitivity.txt
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import rods as R  # noqa: E402
from paper_2607_06794_amd import inputs  # noqa: E402
from tests import cases  # noqa: E402

STEPS = 600


def droplet():
    spec = inputs.CapSpec(shape=(32, 48, 96), footprint=(84.0, 36.0), height=18.0, stripe=(90, 42), seed=2300)
    rho, mat = inputs.sessile_cap(spec)
    rods = inputs.place_rods(6, 24.0, 2.0, (96, 48, 32), inside=inputs.cap_inside(spec), seed=2301, margin=1.0,
                             max_trials=200000)
    return dict(shape=spec.shape, periodic=(True, True, False), G=3.6, tau=(1.0, 1.0), rho=rho, mat=mat,
                evaporation=True, body_force=(0.0, 0.0, 0.0), rods=rods)


def run(delta):
    c = droplet()
    rho = c["rho"].copy()
    rho[0, 16, 24, 48] += delta  # a liquid node above the rods
    nz, ny, nx = c["shape"]
    rp = R.RodParams(**cases.COUPLED_RODS, wall_z=0.5)
    r0 = c["rods"]
    rods = R.Rods(r0[:, :3], r0[:, 3:7], r0[:, 7:10], r0[:, 10:13], rp, (nx, ny, nz), c["periodic"])
    run = R.CoupledRun(rho, c["mat"], cases.oracle_params(c), rods)
    out = []
    for t in range(1, STEPS + 1):
        run.step()
        if t % 50 == 0:
            out.append(run.rods.X.copy())
    return np.array(out)


def main():
    with Pool(2) as pool:
        a, b = pool.map(run, [0.0, 1e-13])
    print("step  max |X_perturbed - X| (lattice units)")
    for i in range(len(a)):
        print(f"{50 * (i + 1):4d}  {np.abs(a[i] - b[i]).max():.2e}")


if __name__ == "__main__":
    main()
