"""Pins of the rod oracle: closed forms, brute force, library solvers, conservation."""
import json
import os

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import lbm
from oracle import rods as R

RNG = np.random.default_rng(2024)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_potential_constants_from_the_paper():
    """Eq. 10 / Eq. 12 constants printed in the paper (golden fixture)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    # WCA: U(d0) = 0 and U grows below d0; LJ minimum -eps at d0 (Eq. 12)
    d0, eps = g["wca_d0"], g["wca_eps"]
    p = R.RodParams(eps_att=0.0, eps_rep=eps, d0=d0)
    assert R.pair_energy(d0, p) == pytest.approx(0.0, abs=1e-15)
    assert R.pair_energy(0.9 * d0, p) > 0
    assert R.lj_form(d0, d0) == -1.0
    assert abs(R.lj_form_deriv(d0, d0)) < 1e-15
    # the paper's printed elongation parameter of the patch, Eq. 5
    rx, ry = g["patch_half_lengths"]
    assert (rx - ry) / (rx + ry) == pytest.approx(g["epsilon_printed"], abs=5e-4)


def test_pair_potential_closed_forms():
    p = R.RodParams(eps_att=2e-4, eps_rep=0.03, d0=5.0, r_cut=7.5)
    phic = R.lj_form(7.5, 5.0)
    assert phic == pytest.approx((5 / 7.5) ** 12 - 2 * (5 / 7.5) ** 6, rel=1e-15)
    assert phic == pytest.approx(-0.16788, abs=1e-5)  # (2/3)^12 - 2 (2/3)^6
    # minimum at d0 with value -eps (1 + phi(rc)); zero force there; zero energy at the cutoff
    assert R.pair_energy(5.0, p) == pytest.approx(-2e-4 * (1 + phic), rel=1e-12)
    assert R.pair_force_mag(5.0, p) == pytest.approx(0.0, abs=1e-15)
    assert R.pair_energy(7.5 - 1e-12, p) == pytest.approx(0.0, abs=1e-12)
    assert R.pair_energy(8.0, p) == 0.0
    # force is minus the derivative of the energy in every regime
    for d in (3.0, 4.5, 4.99, 5.5, 6.7, 7.4):
        h = 1e-6
        fd = -(R.pair_energy(d + h, p) - R.pair_energy(d - h, p)) / (2 * h)
        assert R.pair_force_mag(d, p) == pytest.approx(fd, rel=1e-5, abs=1e-12)
    # attractive between d0 and rc, repulsive below d0
    assert R.pair_force_mag(6.0, p) < 0 < R.pair_force_mag(4.0, p)


def test_segment_distance_matches_bounded_minimiser():
    """Closest points agree with L-BFGS-B on the squared distance over [0,1]^2."""
    for _ in range(300):
        p1, q1, p2, q2 = RNG.normal(size=(4, 3)) * RNG.uniform(0.5, 5.0)
        if RNG.uniform() < 0.2:  # near-parallel pairs
            q2 = p2 + (q1 - p1) * RNG.uniform(0.3, 2.0) + RNG.normal(size=3) * 1e-6
        d, c1, c2, s, t = R.segment_segment(p1, q1, p2, q2)
        fun = lambda v: float(np.sum((p1 + v[0] * (q1 - p1) - p2 - v[1] * (q2 - p2)) ** 2))
        best = min(
            (minimize(fun, x0, method="L-BFGS-B", bounds=[(0, 1), (0, 1)], options={"ftol": 1e-15, "gtol": 1e-12}).fun
             for x0 in ([0.5, 0.5], [0, 0], [1, 1], [0, 1], [1, 0])),
        )
        assert d <= np.sqrt(max(best, 0)) + 1e-9
        assert d == pytest.approx(np.sqrt(max(best, 0)), abs=1e-6)
        assert np.linalg.norm(c1 - c2) == pytest.approx(d, abs=1e-12)


def test_capsule_mask_against_sampled_axis():
    """Mask membership equals distance-to-axis <= R with the axis sampled densely."""
    shape = (20, 22, 24)
    for _ in range(3):
        q = RNG.normal(size=4)
        q /= np.linalg.norm(q)
        X = np.array([12.3, 10.7, 9.9]) + RNG.uniform(-1, 1, 3)
        rods = R.Rods([X], [q], [[0, 0, 0]], [[0, 0, 0]], R.RodParams(length=12.0, radius=2.0), (24, 22, 20), (1, 1, 1))
        rid = rods.mask(shape)
        a, b = rods.ends(0)
        samples = a + np.linspace(0, 1, 4001)[:, None] * (b - a)
        z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
        pts = np.stack([x, y, z], -1).reshape(-1, 3).astype(float)
        near = np.abs(pts - X).max(1) < 10
        dmin = np.full(len(pts), 1e9)
        for s in samples[::1]:
            dmin[near] = np.minimum(dmin[near], np.linalg.norm(pts[near] - s, axis=1))
        inside = (dmin <= 2.0 + 1e-9).reshape(shape)
        # sampling step 12/4000 bounds the distance error by 1.5e-3
        ambiguous = (np.abs(dmin - 2.0) < 2e-3).reshape(shape)
        assert np.array_equal((rid == 0) & ~ambiguous, inside & ~ambiguous)


def test_free_rotation_matches_rodrigues():
    """Angular momentum perpendicular to the axis: rotation by |omega| t about L."""
    p = R.RodParams(length=24, radius=2, eps_att=0, wall_z=None)
    q0 = np.array([1.0, 0, 0, 0])  # axis along z
    Lang = np.array([3.0, 4.0, 0.0])  # perpendicular to the axis
    rods = R.Rods([[10, 10, 10]], [q0], [[0, 0, 0]], [Lang], p, (100, 100, 100), (1, 1, 1))
    Ipar, Iperp = p.inertia
    w = Lang / Iperp
    nsteps = 7
    for _ in range(nsteps):
        rods.integrate(np.zeros((1, 3)), np.zeros((1, 3)))
    theta = np.linalg.norm(w) * nsteps
    qexp = np.concatenate([[np.cos(theta / 2)], np.sin(theta / 2) * w / np.linalg.norm(w)])
    assert np.allclose(rods.q[0], R.quat_mul(qexp, q0), atol=1e-13)
    assert abs(np.linalg.norm(rods.q[0]) - 1) < 1e-14
    assert np.allclose(rods.L[0], Lang)  # no torque: angular momentum conserved
    # closed-form inertia of a solid cylinder
    m = np.pi * 4 * 24
    assert p.mass == pytest.approx(m) and Ipar == pytest.approx(m * 2) and Iperp == pytest.approx(m * (12 + 576) / 12)


def test_pair_forces_newton_and_wall():
    """Internal pair forces sum to zero; the wall pushes a low rod up; far rods feel nothing."""
    p = R.RodParams(eps_att=1e-3, wall_z=0.5)
    qx = np.array([np.cos(np.pi / 4), 0, np.sin(np.pi / 4), 0])  # axis along x
    tilt = np.array([np.cos(0.6), 0.2 * np.sin(0.6), np.sin(0.6), 0.1])
    tilt /= np.linalg.norm(tilt)
    for sep, want in ((4.5, "repel"), (6.2, "attract")):
        rods = R.Rods([[20, 20, 3.2], [21, 20 + sep, 12.0]], [qx, tilt], np.zeros((2, 3)), np.zeros((2, 3)), p,
                      (64, 64, 40), (1, 1, 0))
        rods.X[1] = [21, 20 + sep, 3.2]
        rods.q[1] = qx
        F, T = rods.contact_forces()
        h = 3.2 - 0.5
        wall = R.wall_force_mag(h, p)
        assert wall > 0
        assert np.allclose(F[:, 2], wall, rtol=1e-14)  # both rods sit at the same height
        assert abs(F[0, 1] + F[1, 1]) < 1e-18 and abs(F[0, 0] + F[1, 0]) < 1e-18
        if want == "repel":
            assert F[0, 1] < 0 < F[1, 1]
        else:
            assert F[0, 1] > 0 > F[1, 1]
        assert F[0, 1] == pytest.approx(-R.pair_force_mag(sep, p), rel=1e-12)
    far = R.Rods([[5, 5, 20], [40, 40, 20]], [qx, tilt], np.zeros((2, 3)), np.zeros((2, 3)), p, (64, 64, 40), (1, 1, 0))
    F2, _ = far.contact_forces()
    assert np.all(F2 == 0)


def _uniform_case(shape, rod_pos, V, q=None, L=12.0, omega=(0, 0, 0)):
    nz, ny, nx = shape
    rho = np.zeros((2,) + shape)
    rho[0] = 1.0 + RNG.uniform(-1e-3, 1e-3, size=shape)
    rho[1] = 0.03 + RNG.uniform(-1e-4, 1e-4, size=shape)
    mat = np.zeros(shape, np.uint8)
    psi = np.zeros((9, 2))
    psi[lbm.ROD] = (0.6, 0.25)
    fp = lbm.Params(shape=shape, G=3.6, psi_solid=psi)
    p = R.RodParams(length=L, radius=2.0, eps_att=0, wall_z=None)
    q = q if q is not None else np.array([np.cos(0.4), 0.3 * np.sin(0.4), np.sin(0.4) * 0.9539392, 0])
    q = q / np.linalg.norm(q)
    Ipar, Iperp = p.inertia
    rods = R.Rods([rod_pos], [q], [V], [np.array(omega) * Iperp], p, (nx, ny, nz), (1, 1, 1))
    return rho, mat, fp, rods


def test_coupled_momentum_and_mass_conservation():
    """Periodic box, one moving rod: fluid + rod momentum and fluid + exchanged mass conserved."""
    shape = (16, 16, 24)
    rho, mat, fp, rods = _uniform_case(shape, [11.3, 7.6, 8.2], [0.05, -0.03, 0.02], omega=(0, 0.004, 0.002))
    run = R.CoupledRun(rho, mat, fp, rods)
    P0 = run.total_momentum()
    M0 = run.fluid_mass()
    events = 0
    for _ in range(25):
        run.step()
        events += run.last["covered"] + run.last["uncovered"]
    P1 = run.total_momentum()
    assert events > 10  # cover / uncover really happened
    assert np.abs(P1 - P0).max() < 1e-11
    assert np.allclose(run.fluid_mass() + run.solid, M0, rtol=1e-13)


def test_resting_rod_is_static_bounce_back():
    """With V = Omega = 0 the moving bounce-back adds nothing: the fluid step
    equals the plain step with the rod nodes as static solids of the same psi."""
    shape = (12, 12, 16)
    rho, mat, fp, rods = _uniform_case(shape, [8.0, 6.0, 6.0], [0, 0, 0], L=8.0)
    run = R.CoupledRun(rho, mat, fp, rods)
    static = run.material.copy()
    static[static == lbm.ROD] = 5
    psi = fp.psi_solid.copy()
    psi[5] = psi[lbm.ROD]
    fp2 = lbm.Params(shape=shape, G=fp.G, psi_solid=psi)
    f_static, _, _ = lbm.fluid_step(run.f.copy(), static, fp2)
    run.rods.p.n_sub = 1
    run.step()
    # the rod has not moved a full node: masks agree
    assert run.last["covered"] == 0 and run.last["uncovered"] == 0
    assert np.array_equal(run.f, f_static)


# --------------------------------------------------------------------------
# moving bounce-back: Ladd's rule leaves a co-moving equilibrium unchanged
# --------------------------------------------------------------------------


def _comoving_links(V, omega, seed=11):
    """Fluid at f*_k = f^eq(rho_k(x), u(x)) with u(x) = V + Omega x (x - X), the
    rigid velocity field of the rod extended over the whole box (random rho_k).
    For every rod link (fluid x, source x - c_i a rod node) the pull with
    Ladd's moving bounce-back must return f^eq_i(rho_k(x), u(x)): the odd part
    of Eq. 2 is w_i rho (c_i . u) / c_s^2, so f^eq_i - f^eq_ibar =
    2 w_i rho (c_i . u) / c_s^2 exactly, and c_i . u_b is the same at x, at the
    link midpoint and at the rod node for a rigid motion (c_i . (Omega x c_i) = 0).
    Returns (pulled populations, expected, link mask, run, dP, dsolid)."""
    shape = (14, 16, 22)
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    rho = np.zeros((2,) + shape)
    rho[0] = 1.0 + rng.uniform(-0.05, 0.05, size=shape)
    rho[1] = 0.03 + rng.uniform(-0.01, 0.01, size=shape)
    mat = np.zeros(shape, np.uint8)
    fp = lbm.Params(shape=shape, G=0.0, psi_solid=np.zeros((9, 2)))
    p = R.RodParams(length=12.0, radius=2.0, eps_att=0, wall_z=None)
    q = np.array([np.cos(0.45), 0.5 * np.sin(0.45), 0.3 * np.sin(0.45), np.sqrt(0.66) * np.sin(0.45)])
    Iperp = p.inertia[1]
    Lang = np.asarray(omega, dtype=float) * Iperp  # omega perpendicular to the axis below
    rods = R.Rods([[10.7, 8.3, 6.6]], [q], [V], [Lang], p, (nx, ny, nz), (1, 1, 1))
    run = R.CoupledRun(rho, mat, fp, rods)
    w = rods.omega(0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.stack([x, y, z]).astype(float) - rods.X[0][:, None, None, None]
    for a, n in enumerate((nx, ny, nz)):
        d[a] -= n * np.round(d[a] / n)
    u = np.asarray(V, float)[:, None, None, None] + np.cross(w, d, axis=0)
    fluid = run.material == lbm.FLUID
    feq = np.stack([lbm.equilibrium(rho[k], u) for k in range(2)])
    run.f = np.where(fluid, feq, 0.0)
    rho_t = np.array([run.f[k].sum(axis=0) for k in range(2)])
    f, _ = lbm.pull_stream(run.f, run.material, fp)
    dP, dT, dsolid = run.moving_bounce_back(run.f, f, rho_t)
    link = np.zeros((lbm.Q,) + shape, bool)
    for i in range(1, lbm.Q):
        link[i] = fluid & (lbm._shift(run.material, lbm.C[i]) == lbm.ROD)
    return f, feq, link, run, dP, dsolid


@pytest.mark.parametrize("V,omega", [((0.04, -0.03, 0.02), (0.0, 0.0, 0.0)),
                                     ((0.0, 0.0, 0.0), (0.004, -0.006, 0.0)),
                                     ((0.01, 0.02, -0.015), (-0.003, 0.002, 0.005))])
def test_moving_bounce_back_returns_comoving_equilibrium(V, omega):
    f, feq, link, run, _, _ = _comoving_links(V, omega)
    assert link.sum() > 300
    for k in range(2):
        got = f[k][link]
        want = feq[k][link]
        assert np.abs(got - want).max() <= 1e-15 * np.abs(want).max() * 8
    # the added terms are not trivially zero here
    rho_t = np.array([run.f[k].sum(axis=0) for k in range(2)])
    adds = [abs(R.CoupledRun.link_term(i, 1.0, run.rods.velocity_at(0, [5.0, 5.0, 5.0]))) for i in range(1, 19)]
    assert max(adds) > 1e-4 and rho_t[0].max() > 0.9


def test_moving_bounce_back_uniform_flow_exerts_no_force():
    """Uniform densities, rod and fluid translating together: every lattice
    line enters and leaves the closed rod surface equally often, and each
    link carries -c_i times a term even in c_i, so the net load is zero
    (Galilean invariance of the exchange)."""
    shape = (14, 16, 22)
    f, feq, link, run, dP, dsolid = _comoving_links((0.03, 0.01, -0.02), (0, 0, 0))
    # rebuild with uniform densities
    nz, ny, nx = shape
    rho = np.zeros((2,) + shape)
    rho[0], rho[1] = 1.0, 0.03
    u = np.array([0.03, 0.01, -0.02])[:, None, None, None] * np.ones((3,) + shape)
    fluid = run.material == lbm.FLUID
    run.f = np.where(fluid, np.stack([lbm.equilibrium(rho[k], u) for k in range(2)]), 0.0)
    rho_t = np.array([run.f[k].sum(axis=0) for k in range(2)])
    f2, _ = lbm.pull_stream(run.f, run.material, run.fp)
    dP, dT, dsolid = run.moving_bounce_back(run.f, f2, rho_t)
    for i in range(1, lbm.Q):
        assert link[i].sum() == link[lbm.OPP[i]].sum()
    assert np.abs(dP).max() < 1e-13
    # mass pushed by the moving surface: sum over links of 2 w_i rho c_i.u/cs2 = 0 too
    assert np.abs(dsolid).max() < 1e-13


@pytest.mark.parametrize("mistake", ["sign", "factor6", "no_rotation", "density_one"])
def test_planted_bounce_back_mistakes_are_caught(monkeypatch, mistake):
    """Plant a wrong moving bounce-back term in the oracle: the co-moving pin fails."""
    right = R.CoupledRun.link_term

    def wrong(i, rho_k, ub):
        if mistake == "sign":
            return -right(i, rho_k, ub)
        if mistake == "factor6":
            return 3.0 * right(i, rho_k, ub)
        if mistake == "density_one":
            return right(i, 1.0, ub)
        return right(i, rho_k, ub)

    monkeypatch.setattr(R.CoupledRun, "link_term", staticmethod(wrong))
    if mistake == "no_rotation":
        monkeypatch.setattr(R.Rods, "velocity_at", lambda self, r, x: self.V[r].copy())
    worst = 0.0
    for V, om in (((0.04, -0.03, 0.02), (0, 0, 0)), ((0.0, 0.0, 0.0), (0.004, -0.006, 0.0))):
        f, feq, link, _, _, _ = _comoving_links(V, om)
        worst = max(worst, max(np.abs(f[k][link] - feq[k][link]).max() for k in range(2)))
    assert worst > 1e-6


def test_link_velocity_is_the_same_anywhere_on_the_link():
    """c_i . u_b and the torque arm (x_b - X) x (-c_i g) are identical for x_b at
    the fluid node, at the link midpoint and at the rod node (rigid motion),
    so the choice of the midpoint only fixes the rounding."""
    rods = R.Rods([[10.0, 9.0, 8.0]], [[0.9, 0.1, 0.3, 0.2]], [[0.01, -0.02, 0.03]], [[3.0, -2.0, 5.0]],
                  R.RodParams(length=12.0, wall_z=None), (30, 30, 30), (1, 1, 1))
    rods.q[0] /= np.linalg.norm(rods.q[0])
    x = np.array([13.0, 11.0, 9.0])
    for i in range(1, lbm.Q):
        ci = lbm.C[i].astype(float)
        vals = [ci @ rods.velocity_at(0, x - s * ci) for s in (0.0, 0.5, 1.0)]
        assert np.ptp(vals) < 1e-16
        arms = [np.cross(x - s * ci - rods.X[0], -ci * 0.7) for s in (0.0, 0.5, 1.0)]
        assert np.abs(np.array(arms) - arms[0]).max() < 1e-14


# --------------------------------------------------------------------------
# rigid-body substeps: closed forms of the symplectic Euler scheme
# --------------------------------------------------------------------------


def _single_rod(n_sub=5, q=None, L=(0, 0, 0), V=(0, 0, 0)):
    p = R.RodParams(length=24.0, radius=2.0, eps_att=0, wall_z=None, n_sub=n_sub)
    q = np.array([1.0, 0, 0, 0]) if q is None else np.asarray(q, float) / np.linalg.norm(q)
    return R.Rods([[40.0, 41.0, 42.0]], [q], [V], [L], p, (100, 100, 100), (0, 0, 0)), p


def test_constant_force_matches_symplectic_euler_closed_form():
    """F fixed over N steps of n substeps (dt = 1/n): V_m = V0 + m a dt and,
    the position using the updated velocity, X_m = X0 + m V0 dt + a dt^2 m(m+1)/2."""
    F = np.array([[0.7, -0.4, 0.25]])
    V0 = np.array([0.01, 0.02, -0.03])
    rods, p = _single_rod(V=V0)
    X0 = rods.X[0].copy()
    N = 6
    for _ in range(N):
        rods.integrate(F, np.zeros((1, 3)))
    m, dt, a = N * p.n_sub, 1.0 / p.n_sub, F[0] / p.mass
    assert np.allclose(rods.V[0], V0 + m * a * dt, rtol=1e-14, atol=1e-17)
    Xw = X0 + m * V0 * dt + a * dt * dt * m * (m + 1) / 2
    assert np.abs(rods.X[0] - Xw).max() < 1e-12
    # the other order (position first) would give m(m-1)/2: distinguishable here
    assert np.abs(a * dt * dt * m).max() > 1e-5


def test_axial_torque_spins_with_the_parallel_inertia():
    """A constant torque along the axis: L_m = m T dt, omega = L / I_par, the
    axis stays put and the rotation angle is |T| dt^2 m(m+1) / (2 I_par)
    (omega taken after the L update)."""
    q0 = np.array([np.cos(0.3), 0.0, np.sin(0.3), 0.0])
    rods, p = _single_rod(q=q0)
    e = R.axis(rods.q[0])
    Tq = 0.2 * e
    N = 4
    for _ in range(N):
        rods.integrate(np.zeros((1, 3)), Tq[None])
    m, dt = N * p.n_sub, 1.0 / p.n_sub
    Ipar, _ = p.inertia
    theta = np.linalg.norm(Tq) * dt * dt * m * (m + 1) / (2 * Ipar)
    qw = R.quat_mul(np.concatenate([[np.cos(theta / 2)], np.sin(theta / 2) * e]), q0)
    assert min(np.abs(rods.q[0] - qw).max(), np.abs(rods.q[0] + qw).max()) < 1e-13
    assert np.allclose(R.axis(rods.q[0]), e, atol=1e-14)
    assert np.allclose(rods.L[0], m * dt * Tq, rtol=1e-14)
    assert theta > 1e-3


def _free_top_exact(q0, Lang, p, t):
    """Torque-free symmetric top: the orientation is a rotation about L at
    |L| / I_perp after a spin about the initial axis e0 at (L . e0)(1/I_par -
    1/I_perp):  q(t) = exp(t L / I_perp) exp(t b e0) q0 (space-frame rotations)."""
    Ipar, Iperp = p.inertia
    e0 = R.axis(q0)
    b = (1.0 / Ipar - 1.0 / Iperp) * (Lang @ e0)

    def qexp(w):
        n = np.linalg.norm(w)
        return np.concatenate([[np.cos(0.5 * n)], np.sin(0.5 * n) * w / n])

    return R.quat_mul(R.quat_mul(qexp(t * Lang / Iperp), qexp(t * b * e0)), q0)


def _free_top(n_sub, steps, omega_fn=None):
    q0 = np.array([np.cos(0.35), np.sin(0.35) * 0.6, np.sin(0.35) * 0.8, 0.0])
    p0 = R.RodParams(length=24.0, radius=2.0)
    Lang = np.array([0.3, -0.2, 0.5]) * p0.inertia[1] * 0.02  # oblique to the axis
    rods, p = _single_rod(n_sub=n_sub, q=q0, L=Lang)
    if omega_fn is not None:
        rods.omega = lambda r: omega_fn(rods, r)
    for _ in range(steps):
        rods.integrate(np.zeros((1, 3)), np.zeros((1, 3)))
    qe = _free_top_exact(q0, Lang, p, steps)
    err = min(np.abs(rods.q[0] - qe).max(), np.abs(rods.q[0] + qe).max())
    return err, rods, Lang, qe


def test_free_symmetric_top_precesses_about_L():
    """L oblique to the axis, no torque: L is kept exactly, the axis precesses
    about L at |L| / I_perp and the body spins about its axis at
    (L . e)(1/I_par - 1/I_perp).  The exponential map with omega frozen over a
    substep is first order: the error halves when the substeps double."""
    e5, rods, Lang, qe = _free_top(5, 20)
    e10, _, _, _ = _free_top(10, 20)
    assert np.array_equal(rods.L[0], Lang)
    assert e5 < 1e-3
    assert 0.45 < e10 / e5 < 0.55
    # the axis direction alone is within the same bound of the precessed axis
    assert np.abs(R.axis(rods.q[0]) - R.axis(qe)).max() < 2e-3


def test_planted_rigid_body_mistakes_are_caught():
    """Drop the (1/I_par - 1/I_perp)(L.e)e term, or use I_par for every axis:
    the free-top pin misses by 70x and 1000x."""
    def no_par(rods, r):
        return rods.L[r] / rods.p.inertia[1]

    def all_par(rods, r):
        return rods.L[r] / rods.p.inertia[0]

    for fn in (no_par, all_par):
        err, _, _, _ = _free_top(5, 20, fn)
        assert err > 0.01  # the correct scheme is within 1e-3 (2.3e-4)


def test_planted_position_first_order_is_caught():
    """X updated with the old velocity (position before velocity) misses the
    closed form of the constant-force pin."""
    F = np.array([[0.7, -0.4, 0.25]])
    rods, p = _single_rod()
    X0 = rods.X[0].copy()

    def integrate_x_first(F_hyd, T_hyd):
        dt = 1.0 / p.n_sub
        for _ in range(p.n_sub):
            rods.X = rods.X + rods.V * dt
            rods.V = rods.V + F_hyd / p.mass * dt

    for _ in range(6):
        integrate_x_first(F, np.zeros((1, 3)))
    m, dt, a = 6 * p.n_sub, 1.0 / p.n_sub, F[0] / p.mass
    Xw = X0 + a * dt * dt * m * (m + 1) / 2
    assert np.abs(rods.X[0] - Xw).max() > 1e-5


# --------------------------------------------------------------------------
# refill of uncovered nodes: enclosed pockets between touching capsules
# --------------------------------------------------------------------------


def _stub_run(periodic):
    run = R.CoupledRun.__new__(R.CoupledRun)
    run.fp = lbm.Params(shape=(9, 9, 9), periodic=periodic)
    return run


def test_refill_density_rings_by_hand():
    shape = (9, 9, 9)
    stay = np.zeros(shape, bool)
    rho = np.zeros((2,) + shape)
    run = _stub_run((True, True, True))
    x, y, z = 4, 4, 4
    # first ring: two fluid neighbours -> their mean, s = 1
    stay[z, y, x + 1] = stay[z + 1, y + 1, x] = True
    rho[:, z, y, x + 1] = (0.9, 0.05)
    rho[:, z + 1, y + 1, x] = (1.1, 0.01)
    rb, s = run.refill_density((x, y, z), stay, rho, 6)
    assert s == 1 and np.allclose(rb, (1.0, 0.03), rtol=1e-15)
    # none in the first ring, three in the second (x + 2 c_i), one node off
    # every ray (x + (1, 2, 0)) ignored
    stay[:] = False
    for (dx, dy, dz), v in (((2, 0, 0), 0.8), ((0, -2, 2), 1.0), ((-2, 2, 0), 1.2), ((1, 2, 0), 9.0)):
        stay[z + dz, y + dy, x + dx] = True
        rho[:, z + dz, y + dy, x + dx] = (v, 0.1 * v)
    rb, s = run.refill_density((x, y, z), stay, rho, 6)
    assert s == 2 and np.allclose(rb, (1.0, 0.1), rtol=1e-15)
    # periodic wrap at s = 3 through the low x face (node at x = 1, fluid at x = 7)
    stay[:] = False
    stay[z, y, 7] = True
    rho[:, z, y, 7] = (0.7, 0.2)
    rb, s = run.refill_density((1, y, z), stay, rho, 6)
    assert s == 3 and np.array_equal(rb, (0.7, 0.2))
    rb, s = run.refill_density((1, y, z), stay, rho, 2)
    assert s == 0 and np.array_equal(rb, (0.0, 0.0))
    # a closed z end is not wrapped: the node at z = 1 sees nothing through z < 0
    closed = _stub_run((True, True, False))
    stay[:] = False
    stay[8, 4, 4] = True  # would be x - 2 c_z through a wrap from z = 1
    rho[:, 8, 4, 4] = (1.0, 1.0)
    assert closed.refill_density((4, 4, 1), stay, rho, 6)[1] == 0
    assert run.refill_density((4, 4, 1), stay, rho, 6)[1] == 2


POCKET = dict(
    X=[[9.020064, 10.320612, 7.641499], [13.387424, 8.764085, 11.020971], [8.59099, 6.644925, 9.48745],
       [9.340319, 6.46289, 7.132206], [12.149523, 9.100366, 6.180325]],
    Q=[[0.533138, -0.201023, -0.821799, 0.0], [0.197892, -0.752418, 0.628256, 0.0], [0.186819, -0.974079, -0.127552, 0.0],
       [0.487011, -0.435238, -0.757224, 0.0], [0.954717, 0.106518, 0.277794, 0.0]],
    V0=[-0.155726, 0.125496, -0.000284])


def pocket_run():
    """Five overlapping capsules (heavy, no pair forces) in uniform liquid; the
    first slides out of a node that the other four enclose, so the node has no
    fluid neighbour when it is uncovered."""
    shape = (18, 18, 22)
    rho = np.zeros((2,) + shape)
    rho[0], rho[1] = 1.0, 0.03
    mat = np.zeros(shape, np.uint8)
    psi = np.zeros((9, 2))
    psi[lbm.ROD] = (0.6, 0.25)
    fp = lbm.Params(shape=shape, G=3.6, psi_solid=psi)
    q = np.array(POCKET["Q"])
    q /= np.linalg.norm(q, axis=1)[:, None]
    V = np.zeros((5, 3))
    V[0] = POCKET["V0"]
    p = R.RodParams(length=12.0, radius=2.0, wall_z=None, eps_rep=1e-12, eps_att=0.0, rho_rod=1e6)
    rods = R.Rods(POCKET["X"], q, V, np.zeros((5, 3)), p, (22, 18, 18), (1, 1, 1))
    return R.CoupledRun(rho, mat, fp, rods)


def test_enclosed_pocket_refill_keeps_every_fluid_node_filled():
    run = pocket_run()
    M0 = run.fluid_mass()
    P0 = run.total_momentum()
    run.step()
    assert run.last["uncovered"] > 0 and run.last["far_refills"] >= 1
    fl = run.material == lbm.FLUID
    rho = np.array([run.f[k].sum(axis=0) for k in range(2)])
    assert np.all(rho[:, fl] > 0.0)
    assert np.allclose(run.fluid_mass() + run.solid, M0, rtol=1e-13)
    assert np.abs(run.total_momentum() - P0).max() <= 1e-14 * np.abs(P0).max()  # heavy rods: round-off of |P|


def test_planted_first_ring_only_refill_leaves_an_empty_node(monkeypatch):
    """The first-ring rule alone gives the enclosed node rho_bar = 0: an empty
    fluid node, which the next fluid step cannot fill while all its
    neighbours are rod nodes -- the non-positive density the sweep droplets
    raised."""
    right = R.CoupledRun.refill_density

    def first_ring_only(self, node, stay, rho, reach):
        return right(self, node, stay, rho, 1)

    monkeypatch.setattr(R.CoupledRun, "refill_density", first_ring_only)
    run = pocket_run()
    run.step()
    fl = run.material == lbm.FLUID
    rho = np.array([run.f[k].sum(axis=0) for k in range(2)])
    assert np.any(rho[0][fl] == 0.0) and np.any(rho[1][fl] == 0.0)
