"""Parity of the bead-spring filament update (HIP) against the FP64 oracle (GPU).

After N coupled steps (fluid step, then filament update), FP64 within 1e-12
and FP32 within 1e-5:
  bead positions   max |dX| / d0 (one bead diameter);
  bead velocities  max |dV| / (d0 per step), the same scale per time step;
  impulses         max |dI| / (m d0 per step), a bead moving one diameter
                   per step (the residual velocities of chains near their
                   rest shape are 1e-3 of that, so a relative error would
                   measure the stiff bond forces' rounding, not the update);
  populations      max |df| / max |f| at fluid nodes."""
import functools
import sys

import numpy as np
import pytest

from oracle import filaments as FL
from oracle import lbm
from tests import cases

pytestmark = pytest.mark.gpu

SPACING = 1.95  # near the zero-tension spacing of a straight chain


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def drop_case():
    """Periodic 24^3 box, droplet of radius 8; three chains of five beads
    inside it, cohesion on."""
    from paper_2607_06794_amd import inputs

    n = 24
    rho, mat = inputs.sphere_droplet((n, n, n), 8, noise=1e-4, seed=2500)
    c0 = (n - 1) / 2.0

    def inside(x, y, z):
        return (x - c0) ** 2 + (y - c0) ** 2 + (z - c0) ** 2 <= 6.0**2

    beads = inputs.place_filaments(3, 5, SPACING, (n, n, n), inside=inside, seed=2501)
    assert len(beads) == 15
    return dict(shape=(n, n, n), periodic=(True, True, True), rho=rho, mat=mat, evaporation=False, beads=beads,
                n_per=5, eps_coh=0.004, wall=None)


def cap_case():
    """Sessile cap on the striped wall with the reservoir plane on top; four
    chains of six beads, some low enough for the substrate's adhesion and
    friction."""
    from paper_2607_06794_amd import inputs

    spec = inputs.CapSpec(shape=(20, 24, 40), footprint=(30.0, 18.0), height=12.0, stripe=(34, 20), seed=2510)
    rho, mat = inputs.sessile_cap(spec)
    beads = inputs.place_filaments(4, 6, SPACING, (40, 24, 20), inside=inputs.cap_inside(spec), seed=2511, zmin=1.3,
                                   margin=0.5)
    assert len(beads) == 24
    return dict(shape=spec.shape, periodic=(True, True, False), rho=rho, mat=mat, evaporation=True, beads=beads,
                n_per=6, eps_coh=0.0, wall=0.5)


CASES = {"drop": drop_case, "cap": cap_case}


def fluid_params(c):
    return lbm.Params(shape=c["shape"], periodic=c["periodic"], tau=(1.0, 1.0), G=3.6, body_force=(0.0, 0.0, 0.0),
                      psi_solid=cases.PSI_SOLID.copy(), rho_top=(0.0, 1.0), evaporation=c["evaporation"])


@functools.lru_cache(maxsize=None)
def oracle_run(name, steps):
    c = CASES[name]()
    p = FL.FilParams(n_per=c["n_per"], eps_coh=c["eps_coh"], wall_z=c["wall"])
    nz, ny, nx = c["shape"]
    fil = FL.Filaments(c["beads"][:, :3], c["beads"][:, 3:], p, (nx, ny, nz), c["periodic"])
    run = FL.FilamentRun(c["rho"], c["mat"], fluid_params(c), fil)
    m0 = run.fluid_mass()
    run.step(steps)
    return run.f.copy(), fil.X.copy(), fil.V.copy(), run.last["impulse"].copy(), run.material, m0, run.fluid_mass(), \
        run.ledger.copy()


def gpu_run(name, prec, steps):
    from paper_2607_06794_amd.sim import Lattice, LatticeParams

    c = CASES[name]()
    say(f"[gpu] filaments case={name} prec={prec} steps={steps} beads={len(c['beads'])}")
    lp = LatticeParams(shape=c["shape"], periodic=c["periodic"], prec=prec, psi_solid=cases.PSI_SOLID.copy(),
                       evaporation=c["evaporation"], rho_top=(0.0, 1.0), wall_z=c["wall"],
                       n_fil=len(c["beads"]) // c["n_per"], fil_beads=c["n_per"], fil_eps_coh=c["eps_coh"])
    lat = Lattice(lp, c["rho"], c["mat"], beads=c["beads"])
    lat.coupled_step(steps)
    obs = lat.observables()
    b = lat.beads()
    _, f = lat.export()
    lat.close()
    return f, b, obs


@pytest.mark.parametrize("name,steps", [("drop", 120), ("cap", 80)])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_filaments_match_oracle(name, steps, prec, tol):
    fo, Xo, Vo, Io, mat, m0, m1, led = oracle_run(name, steps)
    fg, b, obs = gpu_run(name, prec, steps)
    c = CASES[name]()
    nz, ny, nx = c["shape"]
    d = b[:, :3] - Xo
    for a, n in ((0, nx), (1, ny), (2, nz)):
        if c["periodic"][a]:
            d[:, a] -= n * np.round(d[:, a] / n)
    ex = float(np.abs(d).max() / 2.0)
    d0, mass = 2.0, np.pi * 8.0 / 6.0
    ev = float(np.abs(b[:, 3:6] - Vo).max() / d0)
    ei = float(np.abs(b[:, 9:12] - Io).max() / (mass * d0))
    fluid = (mat == lbm.FLUID)[None, None]
    ef = cases.rel_err(np.where(fluid, fg, 0), np.where(fluid, fo, 0))
    say(f"[gpu] filaments {name} {prec}: X {ex:.2e} V {ev:.2e} impulse {ei:.2e} f {ef:.2e} status {obs['status']}")
    assert obs["status"] == 0
    assert ex <= tol and ev <= tol and ef <= tol and ei <= tol
    # each component's mass plus its reservoir ledger is kept (the impulses
    # move momentum only)
    tot0 = m0
    tot1 = obs["mass"] + obs["ledger"]
    assert np.all(np.abs(tot1 - tot0) <= (1e-12 if prec == "f64" else 2e-5) * tot0)
    assert np.all(np.abs(obs["ledger"] - led) <= (1e-9 if prec == "f64" else 1e-3) * np.abs(led).max() + 1e-12)


def test_filament_rejections():
    from paper_2607_06794_amd import _lib
    from paper_2607_06794_amd.sim import Lattice, LatticeParams

    c = drop_case()
    base = dict(shape=c["shape"], n_fil=3, fil_beads=5)
    with pytest.raises(_lib.LbError, match="FP64 or FP32"):
        Lattice(LatticeParams(prec="f16dev", **base), c["rho"], c["mat"], beads=c["beads"])
    with pytest.raises(_lib.LbError, match="Shan-Chen"):
        Lattice(LatticeParams(prec="f32", model="cg", **base), c["rho"], c["mat"], beads=c["beads"])
    with pytest.raises(_lib.LbError, match="LB_FIL_MAX_BEADS"):
        Lattice(LatticeParams(prec="f32", shape=c["shape"], n_fil=1000, fil_beads=5), c["rho"], c["mat"],
                beads=np.zeros((5000, 6)))
    lat = Lattice(LatticeParams(prec="f32", **base), c["rho"], c["mat"], beads=c["beads"])
    try:
        from paper_2607_06794_amd.sim import Batch

        with pytest.raises(_lib.LbError, match="filaments"):
            Batch([lat])
    finally:
        lat.close()


def test_full_size_cap_with_filaments_keeps_mass():
    """The benchmark's 256 x 128 x 64 cap with as many of 200 requested
    filaments of twelve beads (L = 24) as fit straight inside the liquid
    (89), FP32, 20 coupled steps: no NaN, non-positive density, bead-move or
    list bit, every component's mass plus its ledger kept, every bead still
    in the lattice's interior."""
    from paper_2607_06794_amd import inputs
    from paper_2607_06794_amd.sim import Lattice, LatticeParams

    case = cases.cap_case()
    spec = inputs.CapSpec()
    beads = inputs.place_filaments(200, 12, SPACING, (256, 128, 64), inside=inputs.cap_inside(spec), seed=2600,
                                   clearance=2.2, margin=0.5, zmin=1.5, max_trials=300000)
    nf = len(beads) // 12
    say(f"[gpu] full-size cap, {nf} filaments of 12 beads, FP32, 20 steps")
    assert nf >= 80
    lp = cases.lattice_params(case, "f32")
    lp.wall_z, lp.n_fil, lp.fil_beads, lp.fil_eps_coh = 0.5, nf, 12, 0.004
    lat = Lattice(lp, case["rho"], case["mat"], beads=beads)
    o0 = lat.observables()
    lat.coupled_step(20)
    o1 = lat.observables()
    b = lat.beads()
    lat.close()
    tot0 = o0["mass"] + o0["ledger"]
    tot1 = o1["mass"] + o1["ledger"]
    say(f"[gpu] mass closure {np.abs(tot1 - tot0) / tot0}, max |V| {np.abs(b[:, 3:6]).max():.3e}")
    assert o1["status"] & (1 | 2 | 8 | 32) == 0, o1["status"]
    assert np.all(np.abs(tot1 - tot0) <= 2e-5 * tot0)
    assert np.all(np.isfinite(b)) and b[:, 2].min() > 0.5 and b[:, 2].max() < 63.0
