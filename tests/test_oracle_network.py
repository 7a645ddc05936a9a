"""Pins of the resistor-network oracle (Eqs. 15-18) against closed forms and
identities of linear resistor networks."""
import numpy as np
import pytest

from oracle import network as N


def chain(x0, x1, s, y=0.0, z=0.0):
    xs = np.arange(x0, x1 + 1e-9, s)
    return np.stack([xs, np.full_like(xs, y), np.full_like(xs, z)], axis=1)


def test_straight_chain_closed_form():
    # spacing 1.5 with r_c = 2.1 joins nearest neighbours only: resistors of
    # 1.5 in series between the last source bead and the first sink bead
    pos = chain(0.0, 30.0, 1.5)
    x_src, x_snk = 5.0, 25.0
    o = N.kirchhoff(pos, 2.1, x_src, x_snk, dV=1.0)
    x = pos[:, 0]
    x_ls, x_fs = x[x < x_src].max(), x[x > x_snk].min()
    I = 1.0 / (x_fs - x_ls)
    assert o["edges"] == len(pos) - 1
    assert abs(o["I_tot"] - I) < 1e-13
    assert abs(o["kappa"] - I * (x_snk - x_src)) < 1e-12
    free = (x >= x_src) & (x <= x_snk)
    # potential falls linearly along the chain; every free bead carries I
    assert np.allclose(o["V"][free], (x_fs - x[free]) / (x_fs - x_ls), atol=1e-13)
    assert np.allclose(o["I"][free], I, atol=1e-13)
    assert abs(o["I"][np.argmax(np.where(x < x_src, x, -1))] - 0.5 * I) < 1e-13


def test_ideal_chain_gives_kappa_one():
    # beads exactly on both electrode planes' neighbours: the gap equals L
    s = 1.0
    pos = chain(-3.0, 23.0, s)
    o = N.kirchhoff(pos, 1.5, -0.5, 20.5)  # last source bead x = -1, first sink x = 21
    assert abs(o["I_tot"] - 1.0 / 22.0) < 1e-14
    assert abs(o["kappa"] - 21.0 / 22.0) < 1e-13


def test_parallel_chains_add():
    a = chain(0.0, 30.0, 1.5, y=0.0)
    b = chain(0.0, 30.0, 1.5, y=10.0)
    one = N.kirchhoff(a, 2.1, 5.0, 25.0)
    two = N.kirchhoff(np.concatenate([a, b]), 2.1, 5.0, 25.0)
    assert abs(two["I_tot"] - 2.0 * one["I_tot"]) < 1e-13


def test_balanced_bridge_carries_no_current():
    S, T = [0.0, 0.0, 0.0], [4.0, 0.0, 0.0]
    A, B = [2.0, 1.2, 0.0], [2.0, -1.2, 0.0]
    pos = np.array([S, A, B, T])
    o = N.kirchhoff(pos, 2.6, 0.5, 3.5)
    r = np.hypot(2.0, 1.2)
    assert o["edges"] == 5  # S-A, S-B, A-B, A-T, B-T (S-T = 4 is out of range)
    assert abs(o["V"][1] - 0.5) < 1e-14 and abs(o["V"][2] - 0.5) < 1e-14
    assert abs(o["I_tot"] - 1.0 / r) < 1e-14  # two branches of 2 r in parallel
    assert abs(o["I"][1] - 0.5 / r) < 1e-14


def test_floating_and_one_sided_clusters():
    main = chain(0.0, 30.0, 1.5)
    floating = np.array([[15.0, 20.0, 0.0], [16.0, 20.0, 0.0]])   # touches no electrode
    src_only = np.array([[1.0, -20.0, 0.0], [3.0, -20.0, 0.0], [5.0, -20.0, 0.0], [7.0, -20.0, 0.0]])
    pos = np.concatenate([main, floating, src_only])
    o = N.kirchhoff(pos, 2.1, 5.0, 25.0)
    ref = N.kirchhoff(main, 2.1, 5.0, 25.0)
    n = len(main)
    assert abs(o["I_tot"] - ref["I_tot"]) < 1e-14
    assert np.all(o["V"][n:n + 2] == 0.0) and np.all(o["I"][n:n + 2] == 0.0)
    # the source-side dangling chain sits at the source potential, no current
    assert np.allclose(o["V"][n + 2:], 1.0, atol=1e-14) and np.allclose(o["I"][n + 2:], 0.0, atol=1e-14)


def random_network(seed, n=600, box=(40.0, 12.0, 6.0)):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, (n, 3)) * np.array(box)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_power_balance_and_conservation(seed):
    pos = random_network(seed)
    o = N.kirchhoff(pos, 2.1, 8.0, 32.0, dV=1.0)
    assert o["I_tot"] > 1e-3  # the network spans the gap: the identities below are not 0 = 0
    i, j, g = N.edges(pos, 2.1)
    dv = o["V"][i] - o["V"][j]
    # Tellegen: the power the source delivers is dissipated in the resistors
    assert abs(o["I_tot"] * 1.0 - np.sum(g * dv * dv)) <= 1e-10 * max(1.0, abs(o["I_tot"]))
    # the current leaving the source enters the sink
    snk = pos[:, 0] > 32.0
    into = np.sum(np.where(snk[j] & ~snk[i], g * dv, 0.0)) - np.sum(np.where(snk[i] & ~snk[j], g * dv, 0.0))
    assert abs(into - o["I_tot"]) <= 1e-10 * max(1.0, abs(o["I_tot"]))
    # Kirchhoff's current law at the free beads that were solved
    net = np.zeros(len(pos))
    np.add.at(net, i, g * dv)
    np.add.at(net, j, -g * dv)
    free = (pos[:, 0] >= 8.0) & (pos[:, 0] <= 32.0)
    assert np.abs(net[free]).max() < 1e-10
    # Eq. 15 from the edge currents; potentials between the electrode values
    I = np.zeros(len(pos))
    np.add.at(I, i, 0.5 * np.abs(g * dv))
    np.add.at(I, j, 0.5 * np.abs(g * dv))
    assert np.allclose(I, o["I"], atol=1e-14)
    assert o["V"].min() >= -1e-12 and o["V"].max() <= 1.0 + 1e-12


def test_mirror_symmetry():
    pos = random_network(5)
    a = N.kirchhoff(pos, 2.1, 8.0, 32.0)
    m = pos.copy()
    m[:, 0] = 40.0 - m[:, 0]
    b = N.kirchhoff(m, 2.1, 8.0, 32.0)  # electrodes swap ends
    assert abs(a["I_tot"] - b["I_tot"]) < 1e-10 * max(1.0, a["I_tot"])


def test_rod_beads_layout():
    X = np.array([[10.0, 5.0, 3.0], [20.0, 6.0, 2.0]])
    e = np.array([[1.0, 0.0, 0.0], [0.0, 0.6, 0.8]])
    p, nb = N.rod_beads(X, e, half=10.0, spacing=1.0)
    assert nb == 21 and p.shape == (42, 3)
    assert np.allclose(p[0], X[0] - 10.0 * e[0]) and np.allclose(p[20], X[0] + 10.0 * e[0])
    assert np.allclose(np.linalg.norm(np.diff(p[21:], axis=0), axis=1), 1.0)
    assert N.rod_beads(X, e, half=0.2, spacing=1.0)[1] == 2  # at least two beads
