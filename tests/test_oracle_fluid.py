"""Pins of the FP64 fluid oracle against facts fixed outside the oracle.

Each test checks the oracle against lattice identities, closed forms,
conservation laws or textbook solutions -- never against a retyped copy of the
oracle's own formula.
"""
import numpy as np
import pytest

from oracle import lbm

RNG = np.random.default_rng(12345)


# ---------------------------------------------------------------- lattice --
def test_d3q19_isotropy_identities():
    """D3Q19 weights: sum w = 1, sum w c_a c_b = cs2 delta_ab, 4th-order isotropy."""
    C, W = lbm.C.astype(float), lbm.W
    assert C.shape == (19, 3)
    assert len({tuple(c) for c in lbm.C}) == 19
    assert np.isclose(W.sum(), 1.0, rtol=0, atol=1e-15)
    m2 = np.einsum("i,ia,ib->ab", W, C, C)
    assert np.allclose(m2, np.eye(3) / 3.0, atol=1e-15)
    assert np.allclose(np.einsum("i,ia->a", W, C), 0.0, atol=1e-16)
    assert np.isclose(np.sum(W * C[:, 0] ** 2 * C[:, 1] ** 2), 1.0 / 9.0, atol=1e-15)
    assert np.isclose(np.sum(W * C[:, 0] ** 4), 1.0 / 3.0, atol=1e-15)
    # third moment vanishes
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", W, C, C, C), 0.0, atol=1e-16)
    for i in range(19):
        assert (lbm.C[lbm.OPP[i]] == -lbm.C[i]).all()
    # speeds: 1 rest, 6 with |c|^2 = 1, 12 with |c|^2 = 2
    sp = (lbm.C**2).sum(1)
    assert (sp == 0).sum() == 1 and (sp == 1).sum() == 6 and (sp == 2).sum() == 12


def test_equilibrium_moments_exact():
    """Eq. 2 reproduces rho, rho u and rho cs2 I + rho u u exactly on D3Q19."""
    rho = RNG.uniform(0.01, 2.0, size=50)
    u = RNG.uniform(-0.1, 0.1, size=(3, 50))
    feq = lbm.equilibrium(rho, u)
    C = lbm.C.astype(float)
    assert np.allclose(feq.sum(0), rho, rtol=1e-14)
    assert np.allclose(np.einsum("ia,in->an", C, feq), rho * u, rtol=1e-13, atol=1e-16)
    P = np.einsum("ia,ib,in->abn", C, C, feq)
    want = rho[None, None] * (np.eye(3)[:, :, None] / 3.0 + u[:, None] * u[None, :])
    assert np.allclose(P, want, rtol=1e-13, atol=1e-16)


def test_moments_definition_eq3():
    """Eq. 3 on a hand-built population set: rho = sum f, j = sum f c."""
    f = np.zeros((19, 1))
    f[1] = 0.5  # +x
    f[7] = 0.25  # (1, 1, 0)
    f[6] = 0.125  # -z
    rho, j = lbm.moments(f)
    assert rho[0] == 0.875
    assert tuple(j[:, 0]) == (0.75, 0.25, -0.125)


# ------------------------------------------------------------------ force --
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_force_stencil_plane_wave_closed_form(axis):
    """For psi_B = sin(k x_a) the stencil sum is exactly cs2 sin(k) cos(k x_a).

    sum_i w_i sin(k(x + c_ia)) c_ia = cos(k x) sin(k) sum_i w_i c_ia^2 because
    c_ia in {-1, 0, 1}; with psi_A = 1 the force on A is -G times that.
    """
    n = 16
    shape = (n, n, n)
    k = 2 * np.pi / n
    grid = np.meshgrid(*[np.arange(n)] * 3, indexing="ij")  # z, y, x
    coord = grid[2 - axis]
    psi = np.zeros((2,) + shape)
    psi[0] = 1.0
    psi[1] = np.sin(k * coord)
    rho = psi.copy()
    p = lbm.Params(shape=shape, G=2.0)
    F = lbm.sc_force(psi, rho, p)
    want = -2.0 * (1.0 / 3.0) * np.sin(k) * np.cos(k * coord)
    assert np.allclose(F[0, axis], want, atol=1e-14)
    for b in range(3):
        if b != axis:
            assert np.allclose(F[0, b], 0.0, atol=1e-15)
    # force on B: -G psi_B * (gradient stencil of psi_A = const) = 0
    assert np.allclose(F[1], 0.0, atol=1e-15)


def test_force_body_force_term():
    """With G = 0 the force is rho_k g exactly."""
    shape = (4, 4, 4)
    rho = RNG.uniform(0.1, 1.0, size=(2,) + shape)
    p = lbm.Params(shape=shape, G=0.0, body_force=(1e-3, -2e-3, 5e-4))
    F = lbm.sc_force(rho, rho, p)
    for k in range(2):
        for a in range(3):
            assert np.allclose(F[k, a], rho[k] * p.body_force[a], rtol=1e-15)


def test_force_total_momentum_zero_periodic():
    """Cross-coupled forces cancel in total on a periodic lattice (Newton's third law)."""
    shape = (8, 8, 8)
    rho = RNG.uniform(0.05, 1.1, size=(2,) + shape)
    p = lbm.Params(shape=shape, G=3.6)
    F = lbm.sc_force(rho, rho, p)
    tot = F.sum(axis=(0, 2, 3, 4))
    assert np.allclose(tot, 0.0, atol=1e-12)
    # but each component alone is not balanced
    assert np.abs(F[0].sum(axis=(1, 2, 3))).max() > 1e-6


# -------------------------------------------------------------- collision --
def test_collision_invariants_unequal_tau():
    """Mass per component and total momentum sum_k(j_k) + sum_k(F_k) survive collision.

    Uses tau_A != tau_B so the velocity-shift weights 1/tau_k are exercised.
    """
    shape = (6, 5, 4)
    mat = np.zeros(shape, np.uint8)
    p = lbm.Params(shape=shape, tau=(0.8, 1.7), G=3.0, body_force=(1e-4, 0, -2e-4))
    rho0 = RNG.uniform(0.05, 1.0, size=(2,) + shape)
    f = lbm.initial_state(rho0) * RNG.uniform(0.9, 1.1, size=(2, 19) + shape)
    fnew, _, d = lbm.fluid_step(f, mat, p)
    rho, j, F = d["rho"], d["j"], d["F"]
    for k in range(2):
        r2, j2 = lbm.moments(fnew[k])
        assert np.allclose(r2, rho[k], rtol=1e-13)
    _, jA = lbm.moments(fnew[0])
    _, jB = lbm.moments(fnew[1])
    assert np.allclose(jA + jB, j[0] + j[1] + F[0] + F[1], atol=1e-14)


def test_rest_state_is_fixed_point():
    """Uniform densities at rest stay at rest.

    The force vanishes and opposite populations stay exactly equal, so every
    momentum is exactly zero; the densities can move only by the rounding of
    sum_i w_i rho (a few ulp, no drift).
    """
    shape = (6, 6, 6)
    mat = np.zeros(shape, np.uint8)
    rho0 = np.zeros((2,) + shape)
    rho0[0] = 0.7
    rho0[1] = 0.2
    run = lbm.Run(rho0, mat, lbm.Params(shape=shape, G=3.6))
    run.step(50)
    f50 = run.f.copy()
    run.step(50)
    for k in range(2):
        rho, j = lbm.moments(run.f[k])
        assert np.all(j == 0.0)
        assert np.abs(rho - rho0[k]).max() <= 1e-14 * rho0[k].max()
    assert np.all(run.last["F"] == 0.0)
    # the rounding settles: the state has become an exact fixed point
    assert np.array_equal(run.f, f50)


# ------------------------------------------------------------ conservation --
def _droplet(n, R, noise=0.0, seed=0):
    c = n / 2 - 0.5
    z, y, x = np.meshgrid(*[np.arange(n)] * 3, indexing="ij")
    ins = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2 <= R * R
    rho = np.zeros((2, n, n, n))
    rho[0] = np.where(ins, 1.0, 0.03)
    rho[1] = np.where(ins, 0.03, 1.0)
    if noise:
        rho += np.random.default_rng(seed).uniform(-noise, noise, size=rho.shape)
    return rho


def test_mass_and_momentum_conservation_periodic_droplet():
    n = 16
    rho0 = _droplet(n, 5, noise=1e-4, seed=3)
    mat = np.zeros((n, n, n), np.uint8)
    run = lbm.Run(rho0, mat, lbm.Params(shape=(n, n, n), G=3.6))
    m0 = run.masses()
    run.step(200)
    m1 = run.masses()
    assert np.all(np.abs(m1 - m0) / m0 < 1e-13)
    # total post-collision momentum equals the total force of the last step,
    # which vanishes: momentum stays at its initial value of zero
    _, jA = lbm.moments(run.f[0])
    _, jB = lbm.moments(run.f[1])
    P = (jA + jB).sum(axis=(1, 2, 3))
    assert np.abs(P).max() < 1e-12


def test_droplet_symmetries_preserved():
    """A droplet centred at (n/2 - 1/2) keeps its mirror and axis-exchange symmetry."""
    n = 16
    rho0 = _droplet(n, 5)
    mat = np.zeros((n, n, n), np.uint8)
    run = lbm.Run(rho0, mat, lbm.Params(shape=(n, n, n), G=3.6))
    run.step(60)
    rho, _ = lbm.fields(run.f, mat)
    a = rho[0]
    assert np.abs(a - a[:, :, ::-1]).max() < 1e-12
    assert np.abs(a - a[::-1]).max() < 1e-12
    assert np.abs(a - a.transpose(0, 2, 1)).max() < 1e-12
    assert np.abs(a - a.transpose(2, 1, 0)).max() < 1e-12
    # the droplet stays separated: A-rich inside, B-rich outside
    c = n // 2
    assert a[c, c, c] > 0.9 and a[0, 0, 0] < 0.05


@pytest.mark.slow
def test_laplace_law():
    """Delta p * R_eq is constant over R (Delta p = 2 gamma / R) in a fixed box."""
    n = 24
    G = 3.6
    vals = []
    for R in (5, 6, 7):
        rho0 = _droplet(n, R)
        mat = np.zeros((n, n, n), np.uint8)
        run = lbm.Run(rho0, mat, lbm.Params(shape=(n, n, n), G=G))
        run.step(700)
        rho, _ = lbm.fields(run.f, mat)
        P = lbm.pressure(rho, G)
        c = n // 2
        dp = P[c, c, c] - P[0, 0, 0]
        rin, rout = rho[0, c, c, c], rho[0, 0, 0, 0]
        Req = (3 * (rho[0].sum() - rout * n**3) / (4 * np.pi * (rin - rout))) ** (1 / 3)
        vals.append(dp * Req)
    vals = np.array(vals)
    assert np.all(vals > 0)
    assert (vals.max() - vals.min()) / vals.mean() < 0.02


@pytest.mark.slow
def test_poiseuille_profile():
    """G = 0, body force g along x between walls at z = 0 and z = H+1.

    Steady BGK + halfway bounce-back gives an exactly parabolic profile of the
    force-corrected velocity with curvature -g / nu, nu = cs2 (tau - 1/2);
    the wall slip is a small fraction of the peak velocity.
    """
    H = 12
    nz = H + 2
    g = 1e-6
    tau = 0.8
    mat = np.zeros((nz, 1, 1), np.uint8)
    mat[0] = 2
    mat[-1] = 2
    p = lbm.Params(shape=(nz, 1, 1), periodic=(True, True, False), tau=(tau, tau), G=0.0, body_force=(g, 0, 0))
    rho = np.zeros((2, nz, 1, 1))
    rho[0] = 1.0
    run = lbm.Run(rho, mat, p)
    run.step(4000)
    d = run.last
    u = lbm.physical_velocity(d["rho"], d["j"], d["F"])[0, 1:-1, 0, 0]
    z = np.arange(1, nz - 1, dtype=float)
    coef = np.polyfit(z, u, 2)
    nu = (tau - 0.5) / 3.0
    assert abs(2 * coef[0] / (-g / nu) - 1) < 1e-6
    assert np.abs(u - np.polyval(coef, z)).max() < 1e-9 * u.max()
    # symmetric about the channel centre and small slip at the hydrodynamic walls
    assert abs(-coef[1] / (2 * coef[0]) - (H + 1) / 2) < 1e-6
    ua = g / (2 * nu) * (z - 0.5) * (H + 0.5 - z)
    assert abs(u.max() - ua.max()) / ua.max() < 0.01


# ------------------------------------------------------------- evaporation --
def test_evaporation_ledger_closes():
    """sum_fluid rho_k(t) + ledger_k(t) = sum_fluid rho_k(0) with a reservoir top plane."""
    nz, ny, nx = 12, 8, 10
    mat = np.zeros((nz, ny, nx), np.uint8)
    mat[0] = 2
    mat[0, 2:6, 3:7] = 3
    mat[-1] = lbm.GHOST
    psi = np.zeros((9, 2))
    psi[2] = (0.6, 0.4)
    psi[3] = (0.3, 0.7)
    rho = np.zeros((2, nz, ny, nx))
    rho[0] = 0.03
    rho[1] = 1.0
    rho[0, 1:5] = 1.0
    rho[1, 1:5] = 0.03
    p = lbm.Params(shape=(nz, ny, nx), periodic=(True, True, False), G=3.6, psi_solid=psi, rho_top=(0.0, 1.0), evaporation=True)
    run = lbm.Run(rho, mat, p)
    m0 = run.masses()
    run.step(40)
    m1 = run.masses()
    assert np.all(np.abs(m1 + run.ledger - m0) < 1e-12 * m0)
    # component A does evaporate towards the dry reservoir
    assert run.ledger[0] > 0


def test_wall_bounce_back_conserves_mass():
    """Closed box (walls on every face, no reservoir): mass is conserved."""
    n = 8
    mat = np.full((n, n, n), 2, np.uint8)
    mat[1:-1, 1:-1, 1:-1] = 0
    psi = np.zeros((9, 2))
    psi[2] = (0.5, 0.5)
    rho = RNG.uniform(0.2, 0.8, size=(2, n, n, n))
    p = lbm.Params(shape=(n, n, n), periodic=(False, False, False), G=1.5, psi_solid=psi)
    run = lbm.Run(rho, mat, p)
    m0 = run.masses()
    run.step(30)
    assert np.all(np.abs(run.masses() - m0) < 1e-13 * m0)


def test_boundary_validation():
    mat = np.zeros((4, 4, 4), np.uint8)
    with pytest.raises(ValueError):
        lbm.Run(np.ones((2, 4, 4, 4)), mat, lbm.Params(shape=(4, 4, 4), periodic=(True, True, False)))
