"""Pins of the oracle's evaporation sink (Eq. 8; Methods, evaporation
paragraph) against closed forms and invariants."""
import numpy as np
import pytest

from oracle import lbm
from tests import cases


def _film(shape=(12, 6, 8), hf=4, J0=1e-3, K=0.01, h0=8.0, sink=True):
    """A flat liquid film of hf nodes (z = 1 .. hf) on a wall, gas above, a
    lid on top, periodic in x and y."""
    nz, ny, nx = shape
    mat = np.zeros(shape, np.uint8)
    mat[0] = 2
    mat[-1] = 2
    rho = np.zeros((2,) + shape)
    rho[0, 1:hf + 1], rho[1, 1:hf + 1] = 1.0, 0.03
    rho[0, hf + 1:-1], rho[1, hf + 1:-1] = 0.03, 1.0
    p = lbm.Params(shape=shape, periodic=(True, True, False), G=3.6, psi_solid=np.full((9, 2), 0.5),
                   sink=sink, sink_J0=J0, sink_K=K, sink_h0=h0)
    return rho, mat, p


def test_flat_film_loses_the_flux_of_eq8_per_column():
    # one interface node per column (the film's top node, gas above), every
    # column h = hf nodes high: one step moves nx ny J0 / (K + hf / h0) of
    # component A into component B, and nothing else changes
    hf, J0, K, h0 = 4, 1e-3, 0.01, 8.0
    rho, mat, p = _film(hf=hf, J0=J0, K=K, h0=h0)
    _, _, q = _film(hf=hf, J0=J0, K=K, h0=h0, sink=False)
    on = lbm.Run(rho, mat, p).step(1)
    off = lbm.Run(rho, mat, q).step(1)
    nz, ny, nx = mat.shape
    moved = nx * ny * J0 / (K + hf / h0)
    m_on, m_off = on.masses(), off.masses()
    assert m_off[0] - m_on[0] == pytest.approx(moved, rel=1e-12)
    assert m_on[1] - m_off[1] == pytest.approx(moved, rel=1e-12)
    assert on.ledger[0] - off.ledger[0] == pytest.approx(moved, rel=1e-12)
    assert off.ledger[1] - on.ledger[1] == pytest.approx(moved, rel=1e-12)
    # only the rest populations of the film's top plane differ
    d = on.f - off.f
    assert np.all(d[:, 1:] == 0.0)
    dz = np.abs(d[0, 0]).reshape(nz, -1).max(axis=1)
    assert np.all(dz[np.arange(nz) != hf] == 0.0) and dz[hf] == pytest.approx(J0 / (K + hf / h0), rel=1e-12)


def test_sink_is_capped_at_the_rest_population():
    # a flux far above the rest population empties it: f*_0^A = 0 on the
    # interface nodes, its content now in f*_0^B
    rho, mat, p = _film(J0=10.0)
    _, _, q = _film(sink=False)
    on = lbm.Run(rho, mat, p).step(1)
    off = lbm.Run(rho, mat, q).step(1)
    hf = 4
    assert np.all(on.f[0, 0, hf] == 0.0)
    assert np.allclose(on.f[1, 0, hf], off.f[1, 0, hf] + off.f[0, 0, hf], rtol=1e-15, atol=0)


def test_zero_flux_is_the_plain_method():
    c = cases.sink_case(J0=0.0)
    p = cases.oracle_params(c)
    q = cases.oracle_params(dict(c, sink=None))
    a = lbm.Run(c["rho"], c["mat"], p).step(3)
    b = lbm.Run(c["rho"], c["mat"], q).step(3)
    assert np.array_equal(a.f, b.f) and np.array_equal(a.ledger, b.ledger)


def test_sink_ledger_closes_and_total_mass_is_kept():
    c = cases.sink_case(J0=5e-4)
    p = cases.oracle_params(c)
    run = lbm.Run(c["rho"], c["mat"], p)
    m0 = run.masses()
    run.step(25)
    m = run.masses()
    assert run.ledger[0] > 0 and run.ledger[1] == pytest.approx(-run.ledger[0], rel=1e-12)
    assert np.allclose(m + run.ledger, m0, rtol=1e-13, atol=0)
    assert m.sum() == pytest.approx(m0.sum(), rel=1e-13)


def test_flux_is_highest_where_the_droplet_is_thin():
    # Eq. 8 on a cap: per interface node the moved mass falls with the local
    # height, so the thin rim loses more per node than the apex
    c = cases.sink_case(J0=5e-4)
    p = cases.oracle_params(c)
    q = cases.oracle_params(dict(c, sink=None))
    run = lbm.Run(c["rho"], c["mat"], p)
    f0 = run.f.copy()
    on, _, d = lbm.fluid_step(f0, c["mat"], p)
    off, _, _ = lbm.fluid_step(f0, c["mat"], q)
    delta = (off[0, 0] - on[0, 0])  # [z, y, x]
    h = lbm.column_heights(lbm.fields(f0, c["mat"])[0], c["mat"])
    col = delta.sum(axis=0)
    iface = lbm.interface_nodes(d["rho"], c["mat"], p).sum(axis=0)
    per_node = np.where(iface > 0, col / np.maximum(iface, 1), np.nan)
    thin = per_node[(h > 0) & (h <= 2) & (iface > 0)]
    thick = per_node[(h >= h.max() - 1) & (iface > 0)]
    assert thin.size and thick.size and np.nanmin(thin) > np.nanmax(thick)
