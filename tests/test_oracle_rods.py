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
