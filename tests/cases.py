"""Workload definitions shared by the parity tests and the benchmark.

Each case is plain numbers; ``oracle_params`` and ``lattice_params`` turn the
same numbers into the oracle's and the library's parameter objects.
"""
from __future__ import annotations

import numpy as np

from paper_2607_06794_amd import inputs

# Ghost pseudo-densities (psi_A, psi_B) of the wall materials: stripe wets A,
# the surround repels it; rods wet like the stripe.
PSI_SOLID = np.zeros((9, 2))
PSI_SOLID[inputs.STRIPE] = (0.60, 0.25)
PSI_SOLID[inputs.SURROUND] = (0.25, 0.60)
PSI_SOLID[inputs.ROD] = (0.60, 0.25)


def rel_err(a, b):
    """max |a - b| / max |b| (the per-field relative error used throughout)."""
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def sphere_case(n=32, radius=8, seed=1000, noise=1e-4, G=3.6, tau=(1.0, 1.0)):
    rho, mat = inputs.sphere_droplet((n, n, n), radius, noise=noise, seed=seed)
    return dict(shape=(n, n, n), periodic=(True, True, True), G=G, tau=tau, rho=rho, mat=mat,
                evaporation=False, body_force=(0.0, 0.0, 0.0))


def cap_case(shape=(64, 128, 256), footprint=(150.0, 36.0), height=24.0, stripe=(160, 40), seed=2000, noise=1e-4):
    spec = inputs.CapSpec(shape=shape, footprint=footprint, height=height, stripe=stripe, seed=seed, noise=noise)
    rho, mat = inputs.sessile_cap(spec)
    return dict(shape=shape, periodic=(True, True, False), G=3.6, tau=(1.0, 1.0), rho=rho, mat=mat,
                evaporation=True, body_force=(0.0, 0.0, 0.0))


def sink_case(shape=(16, 24, 40), footprint=(26.0, 10.0), height=8.0, stripe=(30, 14), seed=2100, J0=2e-4, K=0.01):
    """The sessile cap under a closed lid (top plane a wall) evaporating by the
    interfacial sink of Eq. 8 instead of the reservoir plane; h0 = the cap
    height."""
    c = cap_case(shape=shape, footprint=footprint, height=height, stripe=stripe, seed=seed)
    mat = c["mat"].copy()
    mat[-1] = inputs.SURROUND
    rho = c["rho"].copy()
    rho[:, -1] = 0.0
    c.update(mat=mat, rho=rho, evaporation=False, sink=(J0, K, height))
    return c


def oracle_params(c):
    from oracle import lbm

    sink = c.get("sink")
    return lbm.Params(shape=c["shape"], periodic=c["periodic"], tau=c["tau"], G=c["G"],
                      body_force=c["body_force"], psi_solid=PSI_SOLID.copy(), rho_top=(0.0, 1.0),
                      evaporation=c["evaporation"], sink=sink is not None,
                      sink_J0=sink[0] if sink else 0.0, sink_K=sink[1] if sink else 0.01,
                      sink_h0=sink[2] if sink else 1.0)


def lattice_params(c, prec, rho_ref=(0.0, 0.0), **tile):
    from paper_2607_06794_amd.sim import LatticeParams

    return LatticeParams(shape=c["shape"], periodic=c["periodic"], prec=prec, tau=c["tau"], G=c["G"],
                         body_force=c["body_force"], psi_solid=PSI_SOLID.copy(), evaporation=c["evaporation"],
                         rho_top=(0.0, 1.0), rho_ref=rho_ref, sink=c.get("sink"), **tile)


# The coupled step at length: a reduced form of the benchmark's droplet with
# five rods placed fully inside the liquid, their centres at most 12 above the
# wall (shared by the GPU parity test and the script that writes the oracle's
# expected values).  Rods kept clear of the liquid-vapour interface: a rod
# whose end pierces the interface makes the trajectory sensitive to rounding
# (a 1e-13 change of one initial density moves the rods by 1e-2 within 500
# steps in the oracle itself), and no two implementations then agree to 1e-12.
COUPLED_RODS = dict(length=24.0, radius=2.0, rho_rod=1.0, eps_att=1e-4, eps_rep=0.03, d0=5.0, r_cut=7.5,
                    eps_wall=0.03, d0_wall=3.0, n_sub=5)


def coupled_cap_case():
    spec = inputs.CapSpec(shape=(32, 48, 96), footprint=(84.0, 36.0), height=18.0, stripe=(90, 42), seed=2300)
    rho, mat = inputs.sessile_cap(spec)
    ins = inputs.cap_inside(spec)
    rods = inputs.place_rods(5, 24.0, 2.0, (96, 48, 32), inside=lambda x, y, z: ins(x, y, z) and z <= 12.0,
                             seed=2355, margin=1.0, gap=4.0, max_trials=200000)
    assert len(rods) == 5
    return dict(shape=spec.shape, periodic=(True, True, False), G=3.6, tau=(1.0, 1.0), rho=rho, mat=mat,
                evaporation=True, body_force=(0.0, 0.0, 0.0), rods=rods)
