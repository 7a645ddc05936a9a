"""Parity of the deposit's resistor network (HIP, lb_kirchhoff and
lb_rod_beads) against the FP64 oracle (GPU).

The conjugate-gradient solve stops at a relative residual of 1e-13; the
potentials then agree with the oracle's direct solve to 1e-9 (the condition
number of these bead Laplacians is below 1e4), and the edge decision is
taken on the same FP64 squared distance on both sides, so the edge counts
agree exactly."""
import numpy as np
import pytest

from oracle import network as N
from oracle import rods as R
from tests import cases

pytestmark = pytest.mark.gpu

TOL = 1e-13


def say(*a):
    print(*a, flush=True)


def gpu(pos, r_c, x_src, x_snk, **kw):
    import torch

    from paper_2607_06794_amd.sim import kirchhoff

    t = torch.tensor(np.asarray(pos, float).reshape(-1, 3), dtype=torch.float64, device="cuda:0")
    o = kirchhoff(t, r_c, x_src, x_snk, tol=kw.pop("tol", TOL), **kw)
    torch.cuda.synchronize()
    o["V"], o["I"] = o["V"].cpu().numpy(), o["I"].cpu().numpy()
    return o


def compare(pos, r_c, x_src, x_snk):
    g = gpu(pos, r_c, x_src, x_snk)
    o = N.kirchhoff(pos, r_c, x_src, x_snk)
    say(f"[gpu] network n={len(pos)} edges {g['edges']}/{o['edges']} iters {g['iterations']} "
        f"res {g['rel_residual']:.1e} I_tot {g['I_tot']:.12g} vs {o['I_tot']:.12g}")
    assert g["edges"] == o["edges"] and g["n_source"] == o["n_source"] and g["n_sink"] == o["n_sink"]
    assert np.abs(g["V"] - o["V"]).max() <= 1e-9
    assert np.abs(g["I"] - o["I"]).max() <= 1e-9 * max(1.0, np.abs(o["I"]).max())
    assert abs(g["I_tot"] - o["I_tot"]) <= 1e-9 * max(1.0, abs(o["I_tot"]))
    assert abs(g["I_ref"] - o["I_ref"]) <= 1e-15 and abs(g["kappa"] - o["kappa"]) <= 1e-9 * max(1.0, abs(o["kappa"]))
    return g, o


def chain(x0, x1, s, y=0.0):
    xs = np.arange(x0, x1 + 1e-9, s)
    return np.stack([xs, np.full_like(xs, y), np.zeros_like(xs)], axis=1)


def test_chain_closed_form():
    g, _ = compare(chain(0.0, 30.0, 1.5), 2.1, 5.0, 25.0)
    assert abs(g["I_tot"] - 1.0 / 21.0) < 1e-12  # last source bead 4.5, first sink bead 25.5


@pytest.mark.parametrize("seed,n", [(0, 600), (1, 600), (3, 5000)])
def test_random_networks_match_oracle(seed, n):
    # several 256-bead tiles and a ragged tail; mean degree ~6.5 spans the gap
    rng = np.random.default_rng(seed)
    box = np.array([40.0, 12.0, 6.0]) * (n / 600.0) ** (1.0 / 3.0)
    pos = rng.uniform(0.0, 1.0, (n, 3)) * box
    g, o = compare(pos, 2.1, 0.2 * box[0], 0.8 * box[0])
    assert o["I_tot"] > 1e-3


def test_degenerate_networks():
    import torch

    from paper_2607_06794_amd import _lib
    from paper_2607_06794_amd.sim import kirchhoff

    # no beads at all
    e = kirchhoff(torch.zeros((0, 3), dtype=torch.float64, device="cuda:0"), 2.1, 1.0, 2.0)
    assert e["I_tot"] == 0.0 and e["edges"] == 0 and abs(e["I_ref"] - 1.0) < 1e-15
    # source bead next to a sink bead, nothing free in between
    g, _ = compare(np.array([[0.0, 0, 0], [1.5, 0, 0]]), 2.1, 0.5, 1.0)
    assert abs(g["I_tot"] - 1.0 / 1.5) < 1e-15 and g["iterations"] == 0
    # floating pair and a source-side dangling chain next to a spanning chain
    pos = np.concatenate([chain(0.0, 30.0, 1.5), [[15.0, 20.0, 0.0], [16.0, 20.0, 0.0]],
                          chain(1.0, 7.0, 2.0, y=-20.0)])
    compare(pos, 2.1, 5.0, 25.0)
    # too many neighbours: 70 beads within r_c of each other
    rng = np.random.default_rng(9)
    dense = torch.tensor(rng.uniform(0.0, 0.5, (70, 3)), dtype=torch.float64, device="cuda:0")
    with pytest.raises(_lib.LbError):
        kirchhoff(dense, 2.1, 0.1, 0.4)
    # iteration limit reached: reported, not hidden
    rng = np.random.default_rng(1)
    pos = torch.tensor(rng.uniform(0.0, 1.0, (600, 3)) * np.array([40.0, 12.0, 6.0]), device="cuda:0")
    with pytest.raises(_lib.LbError):
        kirchhoff(pos, 2.1, 8.0, 32.0, max_iter=2)


def test_rod_beads_match_oracle_layout():
    from paper_2607_06794_amd.sim import Lattice
    from tests.test_gpu_rods import ROD, periodic_case, rod_params

    c = periodic_case()
    lp = cases.lattice_params(dict(c, G=3.6, tau=(1.0, 1.0), body_force=(0, 0, 0)), "f64")
    rp = rod_params(c)
    lp.rod_length, lp.rod_radius = rp["length"], rp["radius"]
    lat = Lattice(lp, c["rho"], c["mat"], rods=c["rods"])
    beads = lat.rod_beads(1.0).cpu().numpy()
    lat.close()
    rods = np.array(c["rods"], dtype=np.float64)  # the inputs both sides were given
    rods[:, 3:7] /= np.linalg.norm(rods[:, 3:7], axis=1)[:, None]
    half = 0.5 * ROD["length"] - ROD["radius"]
    axes = np.array([R.axis(q) for q in rods[:, 3:7]])
    ref, nb = N.rod_beads(rods[:, :3], axes, half, 1.0)
    assert beads.shape == ref.shape and nb == 9
    assert np.abs(beads - ref).max() < 1e-12
    # the network of these beads: every rod a chain of 1/r resistors
    compare(ref, 1.5, 4.0, 24.0)
