"""Pins of the bead-spring filament oracle: the paper's constants, energy
derivatives, closed forms of the substep integrator, conservation, exact
interpolation of linear fields, the exact-difference impulse, and planted
mistakes that the pins must catch."""
import json
import os

import numpy as np
import pytest

from oracle import filaments as FL
from oracle import lbm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def energies(d, p):
    """The paper's energies written out (Eqs. 9-12), for derivative checks."""
    return {
        "fene": -0.5 * p.k_s * p.R_m**2 * np.log(1.0 - d**2 / p.R_m**2) if d < p.R_m else np.inf,
        "wca": (p.eps * ((p.d0 / d) ** 12 - 2 * (p.d0 / d) ** 6) + p.eps) if d <= p.d0 else 0.0,
        "bend": 0.5 * p.k_b * (d - 2 * p.d0) ** 2,
    }


def test_constants_are_the_papers():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    p = FL.FilParams()
    assert (p.k_s, p.R_m, p.k_b) == (g["fene_ks"], g["fene_rm"], g["bend_kb"])
    assert (p.d0, p.eps, p.eps_s, p.n_sub) == (g["wca_d0"], g["wca_eps"], g["substrate_eps"], g["md_substeps"])


@pytest.mark.parametrize("d", [1.3, 1.7, 1.95, 2.0 - 1e-3, 2.2, 2.39])
def test_forces_are_minus_energy_derivatives(d):
    p = FL.FilParams(eps_coh=0.004)
    h = 1e-6
    for name, fn in (("fene", FL.fene_force), ("bend", FL.bend_force)):
        num = -(energies(d + h, p)[name] - energies(d - h, p)[name]) / (2 * h)
        assert fn(d, p) == pytest.approx(num, rel=1e-7, abs=1e-9), name
    if d + h < p.d0:
        num = -(energies(d + h, p)["wca"] - energies(d - h, p)["wca"]) / (2 * h)
        assert FL.wca_force(d, p) == pytest.approx(num, rel=1e-7, abs=1e-9)


def test_closed_form_values():
    p = FL.FilParams(eps_coh=0.004)
    # WCA and its force vanish at d0; the LJ minimum is at d0
    assert energies(2.0, p)["wca"] == pytest.approx(0.0, abs=1e-15)
    assert FL.wca_force(2.0, p) == pytest.approx(0.0, abs=1e-15)
    assert FL.cohesion_force(2.0, p) == 0.0 and FL.cohesion_force(3.0, p) == 0.0
    assert FL.cohesion_force(2.5, p) < 0.0  # attractive beyond the minimum
    # FENE: -k_s d / (1 - d^2/R_m^2); at d = R_m / sqrt(2) the denominator is 1/2
    d = 2.4 / np.sqrt(2.0)
    assert FL.fene_force(d, p) == pytest.approx(-2 * 0.3 * d, rel=1e-14)
    # bending at rest length 2 d0 = 4: no force
    assert FL.bend_force(4.0, p) == 0.0
    # substrate minimum at sigma = d0 / 2
    assert FL.substrate_force(1.0, p) == pytest.approx(0.0, abs=1e-15)
    assert FL.substrate_force(1.5, p) < 0.0 < FL.substrate_force(0.9, p)
    assert FL.substrate_force(2.6, p) == 0.0
    assert p.mass == pytest.approx(np.pi * 8.0 / 6.0)


def _vacuum_chain(n_per=6, spacing=1.9, seed=3, eps_coh=0.0, wall=None):
    rng = np.random.default_rng(seed)
    p = FL.FilParams(n_per=n_per, wall_z=wall, eps_coh=eps_coh, gamma=0.0, kappa_s=0.0)
    e = rng.normal(size=3)
    X = FL.straight_chains([[20.0, 20.0, 20.0]], [e], p) * (spacing / p.d0) + 20.0 * (1 - spacing / p.d0)
    X += rng.normal(scale=0.05, size=X.shape)
    V = rng.normal(scale=0.01, size=X.shape)
    return FL.Filaments(X, V, p, (40, 40, 40), (True, True, True))


def _energy(fil):
    p = fil.p
    n = fil.n_beads
    U = 0.0
    for a in range(n):
        for b in range(a + 1, n):
            d = float(np.linalg.norm(FL.min_image(fil.X[a] - fil.X[b], fil.box, fil.periodic)))
            e = energies(d, p)
            U += e["wca"]
            if b - a == 1:
                U += e["fene"]
            if b - a == 2:
                U += e["bend"]
    return U + 0.5 * p.mass * (fil.V**2).sum()


def _substeps(fil, n):
    p = fil.p
    dt = 1.0 / p.n_sub
    for _ in range(n):
        Fi, _ = fil.internal_forces()
        fil.V = fil.V + Fi / p.mass * dt
        fil.X = fil.X + fil.V * dt


def test_isolated_chain_conserves_momentum_and_energy():
    fil = _vacuum_chain()
    P0 = fil.V.sum(0).copy()
    E0 = _energy(fil)
    Es = []
    for _ in range(80):
        _substeps(fil, 5)
        Es.append(_energy(fil))
    assert np.abs(fil.V.sum(0) - P0).max() < 1e-15
    # symplectic Euler keeps the energy within O(omega dt) of its start
    # (bounded oscillation of the fast bond modes), with no drift
    Es = np.array(Es)
    assert np.max(np.abs(Es - E0)) < 0.05 * abs(E0)
    assert abs(Es[-10:].mean() - Es[:10].mean()) < 0.01 * abs(E0)


def test_chain_bending_straightens_a_kink():
    """A chain bent at its middle bead relaxes towards straight (bending
    springs between second neighbours, Eq. 11)."""
    p = FL.FilParams(n_per=3, wall_z=None, gamma=0.0, kappa_s=0.0)
    X = np.array([[10.0, 10.0, 10.0], [11.95, 10.0, 10.0], [11.95 + 1.95 * np.cos(1.0), 10.0 + 1.95 * np.sin(1.0), 10.0]])
    fil = FL.Filaments(X, np.zeros_like(X), p, (30, 30, 30), (True, True, True))
    Fi, _ = fil.internal_forces()
    # the end beads are pushed apart along their separation
    r = fil.X[2] - fil.X[0]
    assert Fi[2] @ r > 0 and Fi[0] @ r < 0


def _uniform_fluid(n, u, rho=(1.0, 0.03), periodic=(True, True, True)):
    mat = np.zeros((n, n, n), np.uint8)
    fp = lbm.Params(shape=(n, n, n), periodic=periodic, tau=(1.0, 1.0), G=3.6, body_force=(0.0, 0.0, 0.0),
                    psi_solid=np.zeros((9, 2)), rho_top=(0.0, 1.0), evaporation=False)
    return mat, fp


def test_drag_in_uniform_flow_matches_the_substep_closed_form():
    """One lattice step in a uniform flow: the fluid step keeps it uniform,
    the drag takes V to U + (V0 - U)(1 - gamma dt / m)^5, and the fluid gains
    exactly the momentum the bead lost."""
    n = 10
    U = np.array([0.02, -0.01, 0.005])
    mat, fp = _uniform_fluid(n, U)
    p = FL.FilParams(n_per=1, wall_z=None, kappa_s=0.0)
    V0 = np.array([[-0.03, 0.04, 0.01]])
    fil = FL.Filaments([[4.3, 5.6, 4.9]], V0, p, (n, n, n), (True, True, True))
    rho0 = np.stack([np.full((n, n, n), 1.0), np.full((n, n, n), 0.03)])
    run = FL.FilamentRun(rho0, mat, fp, fil)
    for k in range(2):
        run.f[k] = lbm.equilibrium(rho0[k], np.broadcast_to(U[:, None, None, None], (3, n, n, n)))
    P0 = run.fluid_momentum() + p.mass * fil.V.sum(0)
    run.step()
    a = 1.0 - p.gamma * 0.2 / p.mass
    expect = U + (V0[0] - U) * a**5
    assert np.abs(fil.V[0] - expect).max() < 1e-15
    assert np.abs(run.last["u"][0] - U).max() < 1e-15
    P1 = run.fluid_momentum() + p.mass * fil.V.sum(0)
    assert np.abs(P1 - P0).max() < 1e-13


def test_interpolation_is_exact_for_linear_fields():
    """A uniform two-component state carrying a velocity linear in x, y, z
    (no Shan-Chen force: uniform densities) and a linear colour: the gathered
    velocity and colour gradient are the field's value and slope."""
    n = 12
    mat = np.zeros((n, n, n), np.uint8)
    fp = lbm.Params(shape=(n, n, n), periodic=(True, True, True), tau=(1.0, 1.0), G=0.0,
                    body_force=(0.0, 0.0, 0.0), psi_solid=np.zeros((9, 2)), rho_top=(0.0, 1.0), evaporation=False)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    A = np.array([[1e-3, 2e-3, -1e-3], [0.5e-3, -1e-3, 2e-3], [-2e-3, 1e-3, 0.7e-3]])
    u = np.stack([A[a, 0] * x + A[a, 1] * y + A[a, 2] * z for a in range(3)])
    cA = 0.5 + 0.01 * x - 0.02 * y + 0.015 * z
    rho = np.stack([cA, 1.0 - cA])  # rho_A + rho_B = 1: C = 2 rho_A - 1 is linear
    p = FL.FilParams(n_per=1, wall_z=None)
    fil = FL.Filaments([[5.3, 4.6, 6.2]], [[0.0, 0.0, 0.0]], p, (n, n, n), (True, True, True))
    run = FL.FilamentRun(rho, mat, fp, fil)
    for k in range(2):
        run.f[k] = lbm.equilibrium(rho[k], u)
    sts, ub, gb = run.gather()
    X = fil.X[0]
    assert np.abs(ub[0] - A @ X).max() < 1e-15
    assert np.abs(gb[0] - 2 * np.array([0.01, -0.02, 0.015])).max() < 1e-14
    assert sum(w for *_, w in sts[0]) == pytest.approx(1.0, abs=1e-15)


def test_exact_difference_impulse_adds_momentum_and_keeps_mass():
    n = 6
    rng = np.random.default_rng(9)
    mat = np.zeros((n, n, n), np.uint8)
    fp = lbm.Params(shape=(n, n, n), periodic=(True, True, True), tau=(1.0, 1.0), G=3.6,
                    body_force=(0.0, 0.0, 0.0), psi_solid=np.zeros((9, 2)), rho_top=(0.0, 1.0), evaporation=False)
    rho = rng.uniform(0.05, 1.0, size=(2, n, n, n))
    run = FL.FilamentRun(rho, mat, fp, FL.Filaments(np.zeros((1, 3)), np.zeros((1, 3)), FL.FilParams(n_per=1), (n,) * 3,
                                                     (True,) * 3))
    run.f = run.f + rng.uniform(0, 1e-3, size=run.f.shape)
    node = (2, 3, 4)
    before = run.f[:, :, 2, 3, 4].copy()
    dp = np.array([1e-3, -2e-3, 5e-4])
    run.apply_impulse({node: dp})
    after = run.f[:, :, 2, 3, 4]
    for k in range(2):
        assert after[k].sum() == pytest.approx(before[k].sum(), abs=1e-15)
    dj = (after - before).sum(0) @ lbm.C
    assert np.abs(dj - dp).max() < 1e-16
    # each component takes the share of its density
    rk = before.sum(1)
    for k in range(2):
        assert np.abs((after[k] - before[k]) @ lbm.C - rk[k] / rk.sum() * dp).max() < 1e-16


def _droplet_run(wall=False, steps=6, eps_coh=0.005, n=14):
    from paper_2607_06794_amd import inputs

    rho, mat = inputs.sphere_droplet((n, n, n), 5, noise=1e-4, seed=77)
    periodic = (True, True, True)
    p = FL.FilParams(n_per=4, wall_z=None, eps_coh=eps_coh)
    fp = lbm.Params(shape=(n, n, n), periodic=periodic, tau=(1.0, 1.0), G=3.6, body_force=(0.0, 0.0, 0.0),
                    psi_solid=np.zeros((9, 2)), rho_top=(0.0, 1.0), evaporation=False)
    X = FL.straight_chains([[6.5, 6.2, 6.7], [6.4, 8.6, 6.1]], [[1, 0.2, 0.1], [0.9, -0.1, 0.3]], p) * 0.975
    fil = FL.Filaments(X, np.zeros_like(X), p, (n, n, n), periodic)
    return FL.FilamentRun(rho, mat, fp, fil)


def test_coupled_momentum_and_mass_are_conserved():
    """Periodic box, no wall: fluid momentum plus bead momentum and each
    component's mass are kept by the coupled step (drag, solvation and their
    reactions, the exact-difference impulse)."""
    run = _droplet_run()
    p = run.fil.p
    P0 = run.fluid_momentum() + p.mass * run.fil.V.sum(0)
    m0 = run.fluid_mass()
    for _ in range(6):
        run.step()
        P = run.fluid_momentum() + p.mass * run.fil.V.sum(0)
        assert np.abs(P - P0).max() < 1e-13
        assert np.abs(run.fluid_mass() - m0).max() < 1e-12 * m0.max()
    assert np.abs(run.last["impulse"]).max() > 1e-4  # the coupling is active


def test_solvation_pushes_beads_into_the_liquid():
    """A bead in the interface of a droplet of A is pushed along grad C,
    towards the droplet's centre."""
    run = _droplet_run(steps=0)
    run.f, _, _ = lbm.fluid_step(run.f, run.material, run.fp)
    run.fil.X = np.array([[6.5 + 5.0, 6.5, 6.5]])
    run.fil.V = np.zeros((1, 3))
    run.fil.p = FL.FilParams(n_per=1, wall_z=None)
    _, _, gb = run.gather()
    assert gb[0, 0] < 0 and abs(gb[0, 0]) > 10 * max(abs(gb[0, 1]), abs(gb[0, 2]))


def test_friction_decelerates_and_never_reverses():
    """A bead pressed on the wall (z = wall + 1, the substrate minimum) by a
    constant load slides to rest: each substep removes mu N dt / m of its
    tangential speed until it stops, and it does not move backwards."""
    p = FL.FilParams(n_per=1, wall_z=0.5, mu=0.5)
    fil = FL.Filaments([[5.0, 5.0, 1.5]], [[0.02, 0.0, 0.0]], p, (20, 20, 20), (True, True, False))
    load = np.array([[0.0, 0.0, -0.05]])
    Fs = np.zeros((1, 3))
    v = [0.02]
    for _ in range(40):
        Ff = fil.friction(load, Fs, fil.V)
        fil.V = fil.V + Ff / p.mass * 0.2
        v.append(fil.V[0, 0])
    dv = p.mu * 0.05 * 0.2 / p.mass
    assert v[1] == pytest.approx(0.02 - dv, rel=1e-14)
    assert min(v) >= 0.0 and v[-1] == 0.0


@pytest.mark.parametrize("mistake", ["reaction_sign", "no_solvation_reaction", "impulse_per_component_density"])
def test_planted_coupling_mistakes_are_caught(monkeypatch, mistake):
    """Each planted mistake in the coupled step breaks the momentum pin."""
    if mistake == "reaction_sign":
        monkeypatch.setattr(FL.FilamentRun, "reaction", staticmethod(lambda Fd, Fs: Fd + Fs))
    elif mistake == "no_solvation_reaction":
        monkeypatch.setattr(FL.FilamentRun, "reaction", staticmethod(lambda Fd, Fs: -Fd))
    else:
        def per_component(self, dp):
            # each component shifted by dp / rho_k instead of dp / rho
            for (z, y, x), d in dp.items():
                for k in range(2):
                    fk = self.f[k, :, z, y, x]
                    rk = fk.sum()
                    uk = (fk @ lbm.C) / rk
                    self.f[k, :, z, y, x] = fk + (lbm.equilibrium(np.array([rk]), (uk + d / rk)[:, None])
                                                  - lbm.equilibrium(np.array([rk]), uk[:, None]))[:, 0]

        monkeypatch.setattr(FL.FilamentRun, "apply_impulse", per_component)
    run = _droplet_run()
    p = run.fil.p
    P0 = run.fluid_momentum() + p.mass * run.fil.V.sum(0)
    worst = 0.0
    for _ in range(4):
        run.step()
        P = run.fluid_momentum() + p.mass * run.fil.V.sum(0)
        worst = max(worst, float(np.abs(P - P0).max()))
    assert worst > 1e-6, worst
