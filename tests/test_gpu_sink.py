"""Evaporation sink of Eq. 8 (Methods, evaporation paragraph) in the fused
step against the FP64 oracle (GPU).

The sink runs with FP32 storage, or FP64 with tau = 1.  Tolerances as for
the plain step: FP64 1e-12 and FP32 1e-5 relative (max |a - b| / max |b|
over the populations) against the FP64 oracle, ledgers to 1e-12 / 1e-5
relative; populations of two tilings bit for bit (the column heights are
integer counts).
"""
import functools
import sys

import numpy as np
import pytest

from oracle import lbm
from tests import cases

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sink_cap(J0=5e-4):
    # two x tiles with a ragged tail (72 = 64 + 8), lid on top
    return cases.sink_case(shape=(20, 24, 72), footprint=(44.0, 14.0), height=9.0, stripe=(50, 18), seed=2101, J0=J0)


@functools.lru_cache(maxsize=None)
def oracle_run(steps):
    c = sink_cap()
    run = lbm.Run(c["rho"], c["mat"], cases.oracle_params(c))
    m0 = run.masses()
    run.step(steps)
    return run.f, run.ledger.copy(), m0


def gpu_run(prec, steps, retile=None, **tile):
    from paper_2607_06794_amd.sim import Lattice

    c = sink_cap()
    say(f"[gpu] sink cap {c['shape']} prec={prec} steps={steps} tile={tile} retile={retile}")
    lat = Lattice(cases.lattice_params(c, prec, **tile), c["rho"], c["mat"])
    if retile is None:
        lat.step(steps)
    else:
        at, (ty, rp, zc) = retile
        lat.step(at)
        lat.set_tiles(ty, rp, zc)
        lat.step(steps - at)
    obs = lat.observables()
    _, f = lat.export()
    lat.close()
    return f, obs


@pytest.mark.parametrize("tile,retile", [((8, 1, 8), None), ((8, 1, 8), (12, (4, 1, 4))), ((16, 2, 8), None)])
def test_sink_fp64_matches_oracle(tile, retile):
    # the 64 x 8 tile with one row per thread runs the two-rows-per-thread
    # instantiation in FP64 (same tiling); the retile changes the z chunks
    # mid-run, so the column heights are counted afresh
    steps = 30
    fo, led_o, m0 = oracle_run(steps)
    ty, rp, zc = tile
    f, obs = gpu_run("f64", steps, retile=retile, tile_y=ty, rows_per_thread=rp, zchunk=zc)
    ef = cases.rel_err(f, fo)
    say(f"[gpu] sink f64 tile={tile} retile={retile}: rel err f {ef:.3e} ledger {obs['ledger']} oracle {led_o}")
    assert ef <= 1e-12
    assert led_o[0] > 0
    assert np.allclose(obs["ledger"], led_o, rtol=1e-12, atol=0)
    assert np.allclose(obs["mass"] + obs["ledger"], m0, rtol=1e-13, atol=0)
    assert obs["status"] == 0


@pytest.mark.parametrize("retile", [None, (12, (4, 1, 4))])
def test_sink_matches_oracle(retile):
    # the retile case changes the z chunks mid-run: the column heights are
    # counted afresh and the ledger pairs folded
    steps = 30
    fo, led_o, m0 = oracle_run(steps)
    f, obs = gpu_run("f32", steps, retile=retile, tile_y=8, rows_per_thread=1, zchunk=8)
    ef = cases.rel_err(f, fo)
    say(f"[gpu] sink f32 retile={retile}: rel err f {ef:.3e} ledger {obs['ledger']} oracle {led_o}")
    assert ef <= 1e-5
    assert led_o[0] > 0
    assert np.allclose(obs["ledger"], led_o, rtol=1e-5, atol=0)
    assert np.allclose(obs["mass"] + obs["ledger"], m0, rtol=1e-6, atol=0)
    assert obs["status"] == 0


def test_sink_is_tile_invariant():
    a, oa = gpu_run("f32", 20, tile_y=8, rows_per_thread=1, zchunk=4)
    b, ob = gpu_run("f32", 20, tile_y=16, rows_per_thread=2, zchunk=20)
    assert np.array_equal(a, b)
    assert np.allclose(oa["ledger"], ob["ledger"], rtol=1e-6, atol=0)


def test_sink_rejected_where_unsupported():
    from paper_2607_06794_amd import _lib
    from paper_2607_06794_amd.sim import Batch, Lattice

    c = sink_cap()
    with pytest.raises(_lib.LbError, match="sink"):
        Lattice(cases.lattice_params(c, "f16dev"), c["rho"], c["mat"])
    ct = dict(c, tau=(1.0, 0.8))
    with pytest.raises(_lib.LbError, match="sink"):
        Lattice(cases.lattice_params(ct, "f64"), ct["rho"], ct["mat"])
    lat = Lattice(cases.lattice_params(c, "f32"), c["rho"], c["mat"])
    with pytest.raises(_lib.LbError, match="sink"):
        Batch([lat])
    lat.close()


def test_sink_with_unequal_relaxation_times():
    # tau != 1 keeps the populations in registers and marches without the
    # software pipeline: the same sink on that path
    from paper_2607_06794_amd.sim import Lattice

    c = dict(sink_cap(), tau=(1.0, 0.8))
    run = lbm.Run(c["rho"], c["mat"], cases.oracle_params(c))
    run.step(12)
    say(f"[gpu] sink cap tau={c['tau']} f32 12 steps")
    lat = Lattice(cases.lattice_params(c, "f32"), c["rho"], c["mat"])
    lat.step(12)
    obs = lat.observables()
    _, f = lat.export()
    lat.close()
    ef = cases.rel_err(f, run.f)
    say(f"[gpu] sink tau != 1: rel err f {ef:.3e} ledger {obs['ledger']} oracle {run.ledger}")
    assert ef <= 1e-5
    assert np.allclose(obs["ledger"], run.ledger, rtol=1e-5, atol=0)
