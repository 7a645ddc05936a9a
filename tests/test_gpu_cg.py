"""Parity of the colour-gradient step (HIP) against the FP64 oracle (GPU).

Populations at fluid nodes after N steps: FP64 within 1e-12 and FP32 within
1e-5 relative (max |a - b| / max |b|); colour masses kept on the GPU."""
import functools
import sys

import numpy as np
import pytest

from oracle import cg as OC
from tests import cases

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def drop_case():
    """Periodic box with an off-centre droplet of component 1 and noise."""
    n = 20
    rng = np.random.default_rng(5150)
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    ins = (x - 9.3) ** 2 + (y - 10.1) ** 2 + (z - 9.8) ** 2 <= 36.0
    rho = np.zeros((2, n, n, n))
    rho[0] = np.where(ins, 1.0, 0.0) + rng.uniform(0, 1e-3, size=(n, n, n))
    rho[1] = np.where(ins, 0.0, 1.0) + rng.uniform(0, 1e-3, size=(n, n, n))
    return dict(shape=(n, n, n), periodic=(True, True, True), rho=rho, mat=np.zeros((n, n, n), np.uint8),
                tau=(1.0, 1.0), sigma=0.02, g=(0.0, 0.0, 0.0), theta=np.full(9, np.pi / 2))


def wall_case():
    """Cap on a striped wall (60 degrees on the stripe, 120 around it) under a
    lid of 90 degrees; unequal relaxation times and a small body force."""
    from paper_2607_06794_amd import inputs

    shape = (16, 14, 40)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    mat = np.zeros(shape, np.uint8)
    mat[0] = inputs.SURROUND
    mat[0][(np.abs(x[0] - 19.5) <= 9) & (np.abs(y[0] - 6.5) <= 4)] = inputs.STRIPE
    mat[-1] = 4
    ins = ((x - 19.5) / 11.0) ** 2 + ((y - 6.5) / 5.0) ** 2 + ((z - 0.5) / 7.0) ** 2 <= 1.0
    rho = np.zeros((2,) + shape)
    rho[0] = np.where(ins, 1.0, 0.0)
    rho[1] = np.where(ins, 0.0, 1.0)
    rho[:, mat != 0] = 0.0
    th = np.full(9, np.pi / 2)
    th[inputs.STRIPE], th[inputs.SURROUND] = np.deg2rad(60.0), np.deg2rad(120.0)
    return dict(shape=shape, periodic=(True, True, False), rho=rho, mat=mat, tau=(0.9, 1.15), sigma=0.015,
                g=(2e-6, 0.0, -1e-6), theta=th)


def ragged_case():
    """Odd extents in every direction, tau = 0.8."""
    shape = (13, 11, 17)
    rng = np.random.default_rng(5151)
    z, y, x = np.meshgrid(*(np.arange(v) for v in shape), indexing="ij")
    ins = (x - 8.0) ** 2 + (y - 5.0) ** 2 + (z - 6.0) ** 2 <= 14.0
    rho = np.zeros((2,) + shape)
    rho[0] = np.where(ins, 1.0, 0.02) + rng.uniform(0, 1e-3, size=shape)
    rho[1] = np.where(ins, 0.02, 1.0) + rng.uniform(0, 1e-3, size=shape)
    return dict(shape=shape, periodic=(True, True, True), rho=rho, mat=np.zeros(shape, np.uint8), tau=(0.8, 0.8),
                sigma=0.01, g=(0.0, 0.0, 0.0), theta=np.full(9, np.pi / 2))


CASES = {"drop": drop_case, "walls": wall_case, "ragged": ragged_case}


@functools.lru_cache(maxsize=None)
def oracle_run(name, steps):
    c = CASES[name]()
    p = OC.CGParams(shape=c["shape"], periodic=c["periodic"], tau=c["tau"], sigma=c["sigma"], beta=0.7,
                    body_force=c["g"], theta=c["theta"])
    run = OC.CGRun(c["rho"], c["mat"], p)
    m0 = run.masses()
    run.step(steps)
    return run.f, run.material, m0, run.masses()


def gpu_run(name, prec, steps):
    from paper_2607_06794_amd.sim import Lattice, LatticeParams

    c = CASES[name]()
    say(f"[gpu] colour gradient case={name} prec={prec} steps={steps} shape={c['shape']}")
    lp = LatticeParams(shape=c["shape"], periodic=c["periodic"], prec=prec, tau=c["tau"], body_force=c["g"],
                       model="cg", cg_sigma=c["sigma"], cg_beta=0.7, cg_grad_eps=1e-2, cg_theta=c["theta"])
    lat = Lattice(lp, c["rho"], c["mat"])
    o0 = lat.observables()
    lat.step(steps)
    obs = lat.observables()
    _, f = lat.export()
    lat.close()
    return f, o0, obs


@pytest.mark.parametrize("name,steps", [("drop", 150), ("walls", 120), ("ragged", 100)])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_cg_parity(name, steps, prec, tol):
    fo, mo, m0, m1 = oracle_run(name, steps)
    fg, o0, obs = gpu_run(name, prec, steps)
    fluid = (mo == 0)[None, None]
    ef = cases.rel_err(np.where(fluid, fg, 0), np.where(fluid, fo, 0))
    dm = np.abs(obs["mass"] - o0["mass"]) / o0["mass"]
    say(f"[gpu] cg {name} {prec}: rel err f {ef:.3e}, colour mass drift {dm}")
    assert ef <= tol
    assert obs["status"] == 0
    assert np.all(dm <= (1e-13 if prec == "f64" else 1e-5))


def test_cg_rejections():
    """Rods, the reservoir and 16-bit storage are refused for the colour
    gradient; a batch does not take such a lattice."""
    from paper_2607_06794_amd import _lib
    from paper_2607_06794_amd.sim import Lattice, LatticeParams

    c = drop_case()
    for kw in (dict(prec="f16dev"), dict(prec="bf16dev")):
        lp = LatticeParams(shape=c["shape"], model="cg", **kw)
        with pytest.raises(_lib.LbError, match="colour-gradient"):
            Lattice(lp, c["rho"], c["mat"])
    lp = LatticeParams(shape=c["shape"], model="cg", prec="f32", cg_beta=1.5)
    with pytest.raises(_lib.LbError, match="beta"):
        Lattice(lp, c["rho"], c["mat"])
