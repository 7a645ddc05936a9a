"""Parity of the HIP fused step against the FP64 oracle (GPU).

Tolerances: FP64 path 1e-12 and FP32 path 1e-5 relative (max |a-b| / max |b|
per field) after the stated number of steps; integer-like results (bitwise
tile invariance) exact.
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


@functools.lru_cache(maxsize=None)
def oracle_run(name, steps):
    c = CASES[name]()
    run = lbm.Run(c["rho"], c["mat"], cases.oracle_params(c))
    run.step(steps)
    rho, _ = lbm.fields(run.f, run.material)
    return run.f, rho, run.ledger.copy(), run.masses()


def gpu_run(name, prec, steps, rho_ref=(0.0, 0.0), **tile):
    """GPU run of a case; the observables carry mass0, the stored state's
    masses at step 0 (after the initial store into the storage format)."""
    from paper_2607_06794_amd.sim import Lattice

    c = CASES[name]()
    say(f"[gpu] case={name} prec={prec} steps={steps} rho_ref={rho_ref} tile={tile} shape={c['shape']}")
    lat = Lattice(cases.lattice_params(c, prec, rho_ref=rho_ref, **tile), c["rho"], c["mat"])
    m0 = lat.observables()["mass"]
    lat.step(steps)
    obs = lat.observables()
    obs["mass0"] = m0
    rho, f = lat.export()
    lat.close()
    return f, rho, obs


def small_cap():
    return cases.cap_case(shape=(20, 24, 72), footprint=(44.0, 14.0), height=9.0, stripe=(50, 18), seed=2001)


CASES = {
    "cfg1": lambda: cases.sphere_case(32, 8, seed=1000),
    "cap_small": small_cap,
    "ragged": lambda: _ragged(),
    "tau": lambda: cases.sphere_case(16, 5, seed=7, tau=(0.8, 1.3)),
}


def _ragged():
    from paper_2607_06794_amd import inputs

    shape = (11, 13, 70)
    rho, mat = inputs.sphere_droplet(shape, 4.5, noise=1e-3, seed=11)
    return dict(shape=shape, periodic=(True, True, True), G=3.6, tau=(1.0, 1.0), rho=rho, mat=mat,
                evaporation=False, body_force=(0.0, 0.0, 0.0))


def _fluid(mat):
    return (mat == 0)[None, None]


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_sphere_droplet_1000_steps(prec, tol):
    """32^3 periodic droplet R = 8, G = 3.6, noise 1e-4, 1000 steps."""
    fo, ro, _, mo = oracle_run("cfg1", 1000)
    fg, rg, obs = gpu_run("cfg1", prec, 1000)
    ef, er = cases.rel_err(fg, fo), cases.rel_err(rg, ro)
    say(f"[gpu] cfg1 {prec}: rel err f {ef:.3e} rho {er:.3e}")
    assert ef <= tol and er <= tol
    # mass per component conserved (no evaporation)
    m0 = CASES["cfg1"]()["rho"].sum(axis=(1, 2, 3))
    assert np.all(np.abs(obs["mass"] - m0) / m0 < (1e-13 if prec == "f64" else 1e-5))
    assert np.all(np.abs(obs["momentum"]) < (1e-11 if prec == "f64" else 1e-3))


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_sessile_cap_walls_reservoir(prec, tol):
    """Cap on a striped wall with the reservoir plane: bounce-back, ghost psi, ledger."""
    steps = 300
    fo, ro, lo, mo = oracle_run("cap_small", steps)
    fg, rg, obs = gpu_run("cap_small", prec, steps)
    ef, er = cases.rel_err(fg, fo), cases.rel_err(rg, ro)
    el = np.abs(obs["ledger"] - lo).max() / np.abs(lo).max()
    say(f"[gpu] cap_small {prec}: rel err f {ef:.3e} rho {er:.3e} ledger {el:.3e}")
    assert ef <= tol and er <= tol
    assert el <= (1e-11 if prec == "f64" else 1e-4)
    # ledger closure on the GPU: mass + ledger = initial mass
    c = CASES["cap_small"]()
    m0 = np.where(c["mat"] == 0, c["rho"], 0).sum(axis=(1, 2, 3))
    assert np.all(np.abs(obs["mass"] + obs["ledger"] - m0) / m0 < (1e-12 if prec == "f64" else 1e-5))


def test_ragged_shape_and_tile_invariance():
    """70 x 13 x 11 periodic lattice (ragged tiles): parity and bitwise tile invariance."""
    steps = 60
    fo, ro, _, _ = oracle_run("ragged", steps)
    ref = None
    for tile in [dict(tile_y=4, rows_per_thread=1), dict(tile_y=8, rows_per_thread=1),
                 dict(tile_y=8, rows_per_thread=2), dict(tile_y=16, rows_per_thread=2),
                 dict(tile_y=8, rows_per_thread=2, zchunk=3), dict(tile_y=8, rows_per_thread=1, zchunk=11)]:
        fg, rg, _ = gpu_run("ragged", "f64", steps, **tile)
        assert cases.rel_err(fg, fo) <= 1e-12
        if ref is None:
            ref = fg
        else:
            assert np.array_equal(fg, ref), tile


def test_unequal_tau():
    """tau = (0.8, 1.3): the general BGK path with populations held in registers."""
    steps = 100
    fo, ro, _, _ = oracle_run("tau", steps)
    fg, rg, _ = gpu_run("tau", "f64", steps, tile_y=8, rows_per_thread=1)
    assert cases.rel_err(fg, fo) <= 1e-12
    fg4, _, _ = gpu_run("tau", "f64", steps, tile_y=4, rows_per_thread=1)
    assert np.array_equal(fg4, fg)


def test_poiseuille_body_force_channel():
    """G = 0 channel with body force between walls: parity and the parabolic profile."""
    from paper_2607_06794_amd import inputs

    shape = (14, 5, 64)
    rho, mat = inputs.channel(shape)
    c = dict(shape=shape, periodic=(True, True, False), G=0.0, tau=(0.8, 0.8), rho=rho, mat=mat,
             evaporation=False, body_force=(1e-6, 0.0, 0.0))
    CASES["channel"] = lambda: c
    steps = 400
    fo, ro, _, _ = oracle_run("channel", steps)
    fg, rg, _ = gpu_run("channel", "f64", steps, tile_y=4, rows_per_thread=1)
    assert cases.rel_err(fg, fo) <= 1e-12


def test_full_size_cap_two_steps_parity_f32():
    """Full 256 x 128 x 64 cap in the benchmark's launch configuration: two
    FP32 steps against two oracle steps from the same inputs (populations to
    the FP32 bar, ledger), ledger closure on the GPU."""
    from paper_2607_06794_amd.sim import Lattice

    c = cases.cap_case()
    say("[gpu] full-size cap: 2 steps f32")
    lat = Lattice(cases.lattice_params(c, "f32"), c["rho"], c["mat"])
    lat.step(2)
    o2 = lat.observables()
    _, fg2 = lat.export()
    lat.close()
    run = lbm.Run(c["rho"], c["mat"], cases.oracle_params(c))
    run.step(2)
    ef = cases.rel_err(fg2, run.f)
    say(f"[gpu] full-size two-step rel err f {ef:.3e}")
    assert ef <= 1e-6
    assert np.allclose(o2["ledger"], run.ledger, rtol=1e-5, atol=1e-6)
    m0 = np.where(c["mat"] == 0, c["rho"], 0).sum(axis=(1, 2, 3))
    assert np.all(np.abs(o2["mass"] + o2["ledger"] - m0) / m0 < 1e-5)


# Bounds of the 16-bit storage errors after 10^4 steps, fixed before the runs
# were measured, from the rounding model of the storage: stochastic rounding
# of every stored value at every step (the kernel's rounding with its
# hash-based random bits; tests/golden/make_config3_oracle.py runs the FP64
# oracle with it, three seeds per form).
# * the mass of each component random-walks: drift within 5 sigma_M of the
#   closed form in tests/golden/errors.py (rounding_walk);
# * the droplet drifts (16-bit storage keeps neither the total momentum nor
#   its position): within K_MODEL times the largest drift of the model runs;
# * once that drift is translated back, the density errors (whole field and
#   per phase, max and RMS) within K_MODEL times the model runs' largest.
# The pointwise errors without the alignment are reported beside them: after
# 10^4 steps they measure where the drifting droplet sits.
K_MODEL = 4.0
ALIGNED_KEYS = ("rho_A", "rho_B", "liquid_rho_A", "liquid_rho_B", "gas_rho_A", "gas_rho_B", "interface_rho_A",
                "interface_rho_B")


@pytest.mark.parametrize("prec,rho_ref", [("f16dev", 0.0), ("bf16dev", 0.0), ("f16dev", 1.0), ("bf16dev", 1.0)])
def test_16bit_storage_error_at_1e4_steps(prec, rho_ref):
    """32^3 droplet, 10^4 steps, populations stored in 16 bits with stochastic
    rounding (rho_ref = 0: f_i; rho_ref = 1: f_i - w_i, the deviation from the
    lattice weights), FP32 compute, against the FP64 oracle's fields."""
    import json

    from tests.golden import errors as G

    fmt = "f16" if prec == "f16dev" else "bf16"
    gold = np.load(G.CONFIG3_ORACLE)
    rho_o, u_o = gold["rho"].astype(np.float64), gold["u"].astype(np.float64)
    runs = json.load(open(G.CONFIG3_MODEL))["forms"][f"{fmt}|rho_ref={rho_ref:g}"]
    fg, rg, obs = gpu_run("cfg1", prec, 10000, rho_ref=(rho_ref, rho_ref), rounding="stochastic")
    assert obs["status"] == 0
    ug = G.velocity(rg, fg)
    raw = G.field_errors(rg, ug, rho_o, u_o, obs["mass"], gold["mass"])
    # mass drift from the stored initial state (round to nearest at lb_init)
    raw["mass_rel"] = [float(abs(obs["mass"][k] - obs["mass0"][k]) / obs["mass0"][k]) for k in range(2)]
    al = G.aligned_errors(rg, ug, rho_o, u_o)
    sig_m = G.rounding_walk(rho_o, rho_ref, fmt, 10000)
    mdisp = max(float(np.linalg.norm(r["aligned"]["displacement"])) for r in runs)
    tag = f"[gpu] {prec} rho_ref={rho_ref:g}"
    for key in ("rho_A", "rho_B", "u") + ALIGNED_KEYS[2:]:
        mm = max(r["aligned"][key]["max"] for r in runs)
        mr = max(r["aligned"][key]["rms"] for r in runs)
        say(f"{tag} {key}: max {raw[key]['max']:.3e} rms {raw[key]['rms']:.3e} | aligned max {al[key]['max']:.3e} "
            f"rms {al[key]['rms']:.3e} (model <= {mm:.3e} / {mr:.3e})")
    d = float(np.linalg.norm(al["displacement"]))
    say(f"{tag} mass drift {raw['mass_rel']} (5 sigma {[5 * v for v in sig_m]}), droplet drift {d:.3f} "
        f"(model runs up to {mdisp:.3f})")
    for k in range(2):
        assert raw["mass_rel"][k] <= 5.0 * sig_m[k]
    assert d <= K_MODEL * mdisp
    for key in ALIGNED_KEYS:
        for m in ("max", "rms"):
            assert al[key][m] <= K_MODEL * max(r["aligned"][key][m] for r in runs), (key, m)


@pytest.mark.parametrize("prec", ["f16dev", "bf16dev"])
def test_16bit_nearest_rounding_drifts_the_mass(prec):
    """Round to nearest even, 2000 steps: the stored values cluster (the bulk
    phases hold nearly equal populations), so the rounding errors share a
    sign and the mass drifts far beyond the stochastic-rounding walk -- the
    reason the storage forms round stochastically."""
    from tests.golden import errors as G

    fmt = "f16" if prec == "f16dev" else "bf16"
    rho0 = CASES["cfg1"]()["rho"]
    _, rn, on = gpu_run("cfg1", prec, 2000)
    _, rs, os_ = gpu_run("cfg1", prec, 2000, rounding="stochastic")
    sig_m = G.rounding_walk(rho0, 0.0, fmt, 2000)
    # drift from the stored initial state (the oracle keeps the mass exactly)
    dn = np.abs(on["mass"] - on["mass0"]) / on["mass0"]
    ds = np.abs(os_["mass"] - os_["mass0"]) / os_["mass0"]
    say(f"[gpu] {prec} 2000 steps: mass drift nearest {dn}, stochastic {ds}, sigma {sig_m}")
    assert np.all(ds <= 5.0 * np.asarray(sig_m))
    assert np.max(dn / np.asarray(sig_m)) > 10.0


def test_deviation_storage_fp64_parity():
    """The deviation arithmetic (rho_ref = 1) is exact up to rounding: FP64 parity at 1e-12."""
    fo, ro, _, _ = oracle_run("cfg1", 1000)
    fg, rg, _ = gpu_run("cfg1", "f64", 1000, rho_ref=(1.0, 1.0))
    assert cases.rel_err(fg, fo) <= 1e-12 and cases.rel_err(rg, ro) <= 1e-12


def test_tile_switching_mid_run_and_autotune(tmp_path):
    """Changing tiles between steps (and the autotuner's trial steps) keeps the
    populations bitwise identical to a fixed-tile run; the ledger agrees to
    FP64 rounding (its per-tile slots are folded in a fixed order)."""
    from paper_2607_06794_amd.sim import Lattice

    c = small_cap()
    ref = Lattice(cases.lattice_params(c, "f64", tile_y=8, rows_per_thread=1, zchunk=5), c["rho"], c["mat"])
    ref.step(40)
    o_ref = ref.observables()
    _, f_ref = ref.export()
    ref.close()
    lat = Lattice(cases.lattice_params(c, "f64", tile_y=4, rows_per_thread=1), c["rho"], c["mat"])
    for i, (ty, rp, zc) in enumerate([(8, 2, 0), (16, 2, 7), (4, 1, 20), (8, 1, 3)]):
        lat.step(5)
        lat.set_tiles(ty, rp, zc)
    lat.step(20)
    o = lat.observables()
    _, f = lat.export()
    lat.close()
    assert np.array_equal(f, f_ref)
    assert np.allclose(o["ledger"], o_ref["ledger"], rtol=1e-14, atol=1e-12)
    # autotune: returns a supported shape, caches it, and the run stays on the oracle trajectory
    lat = Lattice(cases.lattice_params(c, "f32"), c["rho"], c["mat"])
    t = lat.autotune(trial_steps=2, cache=str(tmp_path / "tiles.json"))
    assert (t["tile_y"], t["rows_per_thread"]) in {(4, 1), (8, 1), (8, 2), (16, 2)} and t["us_per_step"] > 0
    steps_done = lat.observables()["step"]
    lat.close()
    lat = Lattice(cases.lattice_params(c, "f32"), c["rho"], c["mat"])
    t2 = lat.autotune(trial_steps=2, cache=str(tmp_path / "tiles.json"))
    assert t2["cached"] and t2["tile_y"] == t["tile_y"] and t2["zchunk"] == t["zchunk"]
    lat.close()
    fo, _, _, _ = oracle_run("cap_small", steps_done)
    lat = Lattice(cases.lattice_params(c, "f32"), c["rho"], c["mat"])
    lat.autotune(trial_steps=2, cache=str(tmp_path / "other.json"))
    _, fg = lat.export()
    lat.close()
    assert cases.rel_err(fg, fo) <= 1e-5


def test_largest_lattice_sampled_nodes_f32():
    # A periodic lattice at the library's size limit: one component's 19
    # arrays span just under 4 GiB, the reach of the 32-bit byte offsets of
    # the step's buffer accesses.  Two FP32 steps; populations at sampled
    # nodes (the first and last node among them) against the oracle run on
    # a 13^3 periodic sub-box of the initial state around each node (after
    # two steps the sub-box's wrap error has moved 4 nodes in from its faces,
    # so the centre is exact).
    import ctypes as ct

    import torch

    from paper_2607_06794_amd import _lib
    from paper_2607_06794_amd.sim import Lattice, LatticeParams, _stream_ptr

    nz, ny, nx = 215, 512, 512
    n = nz * ny * nx
    say(f"[gpu] largest lattice {nx}x{ny}x{nz} ({n} nodes) f32, 2 steps")
    z = np.arange(nz)[:, None, None]
    y = np.arange(ny)[None, :, None]
    x = np.arange(nx)[None, None, :]
    rho = np.empty((2, nz, ny, nx))
    rho[0] = 0.515 + 0.485 * np.tanh(3.0 * (np.sin(2 * np.pi * x / 37) + np.sin(2 * np.pi * y / 29)
                                             + np.sin(2 * np.pi * z / 23)))
    rho[0] += np.random.default_rng(4242).uniform(-1e-4, 1e-4, size=(nz, ny, nx))
    rho[1] = 1.03 - rho[0]
    mat = np.zeros((nz, ny, nx), np.uint8)
    lp = LatticeParams(shape=(nz, ny, nx), periodic=(True, True, True), prec="f32", G=3.6, psi_solid=cases.PSI_SOLID,
                       tile_y=8, rows_per_thread=1)
    c = lp.to_c()
    assert 19 * _lib.load().lb_pop_stride(ct.byref(c)) * 4 > 0xFFFFFFFF - 16 * 2 ** 20  # within 16 MiB of the limit
    lat = Lattice(lp, rho, mat)
    lat.step(2)
    obs = lat.observables()
    f = torch.empty((2, 19, n), dtype=torch.float64, device=lat.device)
    _lib.check(lat.lib.lb_export(lat._ctx, None, ct.c_void_p(f.data_ptr()), _stream_ptr(lat.stream)))
    rng = np.random.default_rng(77)
    pts = [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (nz - 1, 0, nx - 1)]
    pts += [tuple(int(v) for v in (rng.integers(nz), rng.integers(ny), rng.integers(nx))) for _ in range(5)]
    idx = torch.tensor([(pz * ny + py) * nx + px for pz, py, px in pts], device=lat.device)
    got = f[:, :, idx].cpu().numpy()
    lat.close()
    del f
    assert obs["status"] == 0
    p = lbm.Params(shape=(13, 13, 13), periodic=(True, True, True), G=3.6, psi_solid=cases.PSI_SOLID)
    worst = 0.0
    for s, (pz, py, px) in enumerate(pts):
        sub = rho[:, np.arange(pz - 6, pz + 7) % nz][:, :, np.arange(py - 6, py + 7) % ny][:, :, :, np.arange(px - 6, px + 7) % nx]
        run = lbm.Run(sub, np.zeros((13, 13, 13), np.uint8), p).step(2)
        want = run.f[:, :, 6, 6, 6]
        err = float(np.abs(got[:, :, s] - want).max() / np.abs(want).max())
        worst = max(worst, err)
    say(f"[gpu] largest lattice: worst sampled rel err {worst:.3e} over {len(pts)} nodes")
    assert worst <= 1e-5


@pytest.mark.parametrize("kind", ["no_fluid", "one_fluid_node", "smallest_periodic"])
def test_degenerate_lattices(kind):
    # a lattice without fluid, a single fluid node boxed in by walls, and the
    # smallest lattice the library takes (3 x 3 x 3, periodic): 4 FP64 steps
    # against the oracle, mass kept, status clear
    from paper_2607_06794_amd.sim import Lattice, LatticeParams

    say(f"[gpu] degenerate lattice {kind}")
    if kind == "smallest_periodic":
        shape, per = (3, 3, 3), (True, True, True)
        mat = np.zeros(shape, np.uint8)
        rho = np.empty((2,) + shape)
        rho[0] = 0.5 + 0.1 * np.random.default_rng(3).uniform(-1, 1, size=shape)
        rho[1] = 0.5 + 0.1 * np.random.default_rng(4).uniform(-1, 1, size=shape)
    else:
        shape, per = (5, 6, 7), (False, False, False)
        mat = np.full(shape, 2, np.uint8)
        rho = np.zeros((2,) + shape)
        if kind == "one_fluid_node":
            mat[2, 3, 3] = 0
            rho[:, 2, 3, 3] = (0.8, 0.2)
    lp = LatticeParams(shape=shape, periodic=per, prec="f64", G=3.6, psi_solid=cases.PSI_SOLID)
    lat = Lattice(lp, rho, mat)
    m0 = lat.observables()["mass"].copy()
    lat.step(4)
    obs = lat.observables()
    _, f = lat.export()
    lat.close()
    run = lbm.Run(rho, mat, lbm.Params(shape=shape, periodic=per, G=3.6, psi_solid=cases.PSI_SOLID)).step(4)
    fl = (mat == 0)[None, None]
    assert np.abs(np.where(fl, f - run.f, 0)).max() <= 1e-13 * max(1.0, np.abs(run.f).max())
    assert np.allclose(obs["mass"], m0, rtol=1e-13, atol=1e-300) and obs["status"] == 0
    assert obs["fluid_nodes"] == int((mat == 0).sum())


def test_failed_lattice_raises_status_without_slowing_down():
    # a lattice whose state is NaN everywhere raises ST_NAN and then steps as
    # fast as a healthy one: the status word takes each bit once per
    # wavefront and only while it is not yet set (an atomic per node and step
    # into the one word made such a lattice several times slower, and a
    # batch with one failed lattice slowed down with it); a single NaN node
    # raises the bit too
    import torch

    from paper_2607_06794_amd.sim import Lattice, LatticeParams

    shape = (64, 128, 128)
    mat = np.zeros(shape, np.uint8)
    rng = np.random.default_rng(11)
    # the A-rich bulk phase of the droplet cases (stable at G = 3.6)
    ok = np.stack([1.0 + 1e-3 * rng.uniform(-1, 1, size=shape), 0.03 + 1e-4 * rng.uniform(-1, 1, size=shape)])
    one = ok.copy()
    one[0, 30, 60, 70] = np.nan
    bad = np.full_like(ok, np.nan)
    lp = LatticeParams(shape=shape, periodic=(True, True, True), prec="f32", G=3.6)
    times, status = {}, {}
    for name, rho in (("healthy", ok), ("one_nan", one), ("all_nan", bad)):
        say(f"[gpu] failed-lattice status: {name} {shape}")
        lat = Lattice(lp, rho, mat)
        lat.step(5)
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        lat.step(40)
        e1.record(s)
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1) / 40
        status[name] = int(lat.observables(allow_unstable=True)["status"])
        lat.close()
    say(f"[gpu] ms per step {times}, status {status}")
    assert status["healthy"] == 0
    assert status["one_nan"] & 1 and status["all_nan"] & 1
    assert times["all_nan"] <= 1.5 * times["healthy"] + 0.02
