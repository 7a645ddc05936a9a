"""Thin Python front end over liblbm: device memory from PyTorch, work in HIP.

``Lattice`` owns the caller-side buffers (torch tensors on the GPU) and a
library context.  Every computation happens inside liblbm's kernels; this
module only allocates memory, passes pointers and converts results.
"""
from __future__ import annotations

import ctypes as ct
import json
import os
from dataclasses import dataclass, field

import numpy as np

from . import _lib

PREC = {"f64": _lib.LB_F64, "f32": _lib.LB_F32, "f16dev": _lib.LB_F16DEV, "bf16dev": _lib.LB_BF16DEV}


@dataclass
class LatticeParams:
    """Python mirror of lb_params (see include/lbm.h)."""

    shape: tuple  # (nz, ny, nx)
    periodic: tuple = (True, True, True)  # x, y, z
    prec: str = "f64"
    tau: tuple = (1.0, 1.0)
    G: float = 3.6
    body_force: tuple = (0.0, 0.0, 0.0)
    psi_solid: np.ndarray = field(default_factory=lambda: np.zeros((9, 2)))
    evaporation: bool = False
    rho_top: tuple = (0.0, 1.0)
    rho_ref: tuple = (0.0, 0.0)  # storage reference: 0 stores f_i, else f_i - w_i rho_ref
    # rigid rods
    n_sub: int = 5
    rod_length: float = 24.0
    rod_radius: float = 2.0
    rod_rho: float = 1.0
    eps_att: float = 1e-4
    eps_rep: float = 0.03
    rod_d0: float = 5.0
    rod_rcut: float = 7.5
    eps_wall: float = 0.03
    rod_d0_wall: float = 3.0
    wall_z: float | None = None  # wall plane repelling rods (None: no wall force)
    tile_y: int = 0
    rows_per_thread: int = 0
    zchunk: int = 0
    # interfacial evaporation sink of Eq. 8: (J0, K, h0), None: off
    sink: tuple | None = None
    # fluid model: "sc" (Shan-Chen) or "cg" (the paper's colour gradient)
    model: str = "sc"
    cg_sigma: float = 0.01
    cg_beta: float = 0.7
    cg_grad_eps: float = 1e-2
    cg_theta: np.ndarray = field(default_factory=lambda: np.full(9, np.pi / 2))  # radians per wall material
    # 16-bit storage: "nearest" (round to nearest even) or "stochastic"
    rounding: str = "nearest"
    sr_seed: int = 0
    # bead-spring filaments: n_fil chains of fil_beads beads (see lb_params)
    n_fil: int = 0
    fil_beads: int = 6
    fil_k_s: float = 0.3
    fil_R_m: float = 2.4
    fil_eps: float = 0.03
    fil_d0: float = 2.0
    fil_k_b: float = 8.0
    fil_eps_coh: float = 0.0
    fil_r_cut: float = 3.0
    fil_eps_s: float = 0.006
    fil_sigma_s: float = 1.0
    fil_r_cut_s: float = 2.5
    fil_mu: float = 0.5
    fil_gamma: float = 1.0
    fil_kappa_s: float = 0.05
    fil_skin: float = 1.0

    def to_c(self) -> _lib.LbParams:
        p = _lib.LbParams()
        p.nz, p.ny, p.nx = (int(v) for v in self.shape)
        for d in range(3):
            p.periodic[d] = int(bool(self.periodic[d]))
            p.body_force[d] = float(self.body_force[d])
        p.prec = PREC[self.prec]
        for k in range(2):
            p.tau[k] = float(self.tau[k])
            p.rho_top[k] = float(self.rho_top[k])
            p.rho_ref[k] = float(self.rho_ref[k])
        p.G = float(self.G)
        ps = np.asarray(self.psi_solid, dtype=np.float64)
        for m in range(_lib.LB_NMAT):
            for k in range(2):
                p.psi_solid[m][k] = float(ps[m, k]) if m < ps.shape[0] else 0.0
        p.evap_on = int(bool(self.evaporation))
        p.n_sub = int(self.n_sub)
        p.rod_length = float(self.rod_length)
        p.rod_radius = float(self.rod_radius)
        p.rod_rho = float(self.rod_rho)
        p.eps_att = float(self.eps_att)
        p.eps_rep = float(self.eps_rep)
        p.rod_d0 = float(self.rod_d0)
        p.rod_rcut = float(self.rod_rcut)
        p.eps_wall = float(self.eps_wall)
        p.rod_d0_wall = float(self.rod_d0_wall)
        p.wall_on = int(self.wall_z is not None)
        p.wall_z = float(self.wall_z) if self.wall_z is not None else 0.0
        p.tile_y = int(self.tile_y)
        p.rows_per_thread = int(self.rows_per_thread)
        p.zchunk = int(self.zchunk)
        p.model = {"sc": _lib.LB_MODEL_SC, "cg": _lib.LB_MODEL_CG}[self.model]
        p.cg_sigma, p.cg_beta, p.cg_grad_eps = float(self.cg_sigma), float(self.cg_beta), float(self.cg_grad_eps)
        th = np.asarray(self.cg_theta, dtype=np.float64)
        for m in range(_lib.LB_NMAT):
            p.cg_theta[m] = float(th[m]) if m < th.shape[0] else np.pi / 2
        p.round_stochastic = {"nearest": 0, "stochastic": 1}[self.rounding]
        p.sr_seed = int(self.sr_seed) & 0xFFFFFFFF
        p.n_fil, p.fil_beads = int(self.n_fil), int(self.fil_beads)
        for name in ("k_s", "R_m", "eps", "d0", "k_b", "eps_coh", "r_cut", "eps_s", "sigma_s", "r_cut_s", "mu", "gamma",
                     "kappa_s", "skin"):
            setattr(p, "fil_" + name, float(getattr(self, "fil_" + name)))
        p.sink_on = int(self.sink is not None)
        if self.sink is not None:
            p.sink_J0, p.sink_K, p.sink_h0 = (float(v) for v in self.sink)
        return p


def _stream_ptr(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


class Lattice:
    """One lattice on one GPU: caller-owned buffers plus a liblbm context."""

    def __init__(self, params: LatticeParams, rho0: np.ndarray, material: np.ndarray, device="cuda:0", stream=None,
                 rods: np.ndarray | None = None, beads: np.ndarray | None = None):
        """rods: optional FP64 [n][13] array (X, q (w,x,y,z), V, L) per rod;
        beads: FP64 [n_fil * fil_beads][6] positions and velocities of the
        filaments' beads (params.n_fil > 0)."""
        import torch

        self.lib = _lib.load()
        self.params = params
        self.device = torch.device(device)
        self.stream = stream
        self._cp = params.to_c()
        self.rods_in = None if rods is None else np.ascontiguousarray(rods, dtype=np.float64).reshape(-1, 13)
        self._cp.n_rods = 0 if self.rods_in is None else self.rods_in.shape[0]
        nz, ny, nx = params.shape
        self.n = nx * ny * nz
        pop_bytes = self.lib.lb_pop_bytes(ct.byref(self._cp))
        ws_bytes = self.lib.lb_workspace_bytes(ct.byref(self._cp))
        self.pop_stride = self.lib.lb_pop_stride(ct.byref(self._cp))
        with torch.cuda.device(self.device):
            self.f = [torch.empty(pop_bytes, dtype=torch.uint8, device=self.device) for _ in range(2)]
            self.ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=self.device)
        ws_ptr = self.ws.data_ptr()
        ws_ptr = (ws_ptr + 255) & ~255
        self._buf = _lib.LbBuffers()
        self._buf.f[0] = self.f[0].data_ptr()
        self._buf.f[1] = self.f[1].data_ptr()
        self._buf.workspace = ws_ptr
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        material = np.ascontiguousarray(material, dtype=np.uint8)
        assert rho0.shape == (2,) + tuple(params.shape), rho0.shape
        assert material.shape == tuple(params.shape), material.shape
        self._ctx = ct.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.lb_init(
                ct.byref(self._cp),
                ct.byref(self._buf),
                rho0.ctypes.data_as(ct.c_void_p),
                material.ctypes.data_as(ct.c_void_p),
                self.rods_in.ctypes.data_as(ct.c_void_p) if self.rods_in is not None and len(self.rods_in) else None,
                _stream_ptr(self.stream),
                ct.byref(self._ctx),
            )
        _lib.check(rc)
        self.n_beads = int(params.n_fil) * int(params.fil_beads) if params.n_fil > 0 else 0
        if self.n_beads:
            b = np.ascontiguousarray(beads, dtype=np.float64).reshape(self.n_beads, 6)
            with torch.cuda.device(self.device):
                _lib.check(self.lib.lb_fil_set(self._ctx, b.ctypes.data_as(ct.c_void_p), _stream_ptr(self.stream)))

    # ------------------------------------------------------------------
    def step(self, n: int = 1):
        _lib.check(self.lib.lb_step(self._ctx, int(n), _stream_ptr(self.stream)))
        return self

    @property
    def n_rods(self) -> int:
        return int(self._cp.n_rods)

    def rods_step(self):
        _lib.check(self.lib.lb_rods_step(self._ctx, _stream_ptr(self.stream)))
        return self

    def filament_step(self):
        _lib.check(self.lib.lb_fil_step(self._ctx, _stream_ptr(self.stream)))
        return self

    def coupled_step(self, n: int = 1):
        """n coupled steps: one fluid step then one rod or filament update each."""
        for _ in range(int(n)):
            self.step(1)
            if self.n_beads:
                self.filament_step()
            else:
                self.rods_step()
        return self

    def beads(self) -> np.ndarray:
        """[n_beads][12]: position, velocity, interpolated fluid velocity and
        the impulse handed to the fluid in the last filament update."""
        out = np.zeros((self.n_beads, 12))
        _lib.check(self.lib.lb_fil_get(self._ctx, out.ctypes.data_as(ct.c_void_p), _stream_ptr(self.stream)))
        return out

    def rods(self) -> np.ndarray:
        out = np.zeros((self.n_rods, 13))
        _lib.check(self.lib.lb_rods_get(self._ctx, out.ctypes.data_as(ct.c_void_p), _stream_ptr(self.stream)))
        return out

    def observables(self, allow_unstable=False) -> dict:
        o = _lib.LbObs()
        allow = (_lib.LB_OK, _lib.LB_EUNSTABLE) if allow_unstable else (_lib.LB_OK,)
        _lib.check(self.lib.lb_observables(self._ctx, ct.byref(o), _stream_ptr(self.stream)), allow=allow)
        return {
            "step": o.step,
            "mass": np.array(o.mass[:]),
            "ledger": np.array(o.ledger[:]),
            "momentum": np.array(o.momentum[:]),
            "max_speed": o.max_speed,
            "kinetic": o.kinetic,
            "fluid_nodes": o.fluid_nodes,
            "status": o.status,
            "solid": np.array(o.solid[:]),
            "rod_momentum": np.array(o.rod_momentum[:]),
        }

    def export(self, populations: bool = True):
        """Decoded FP64 state: (rho[2, nz, ny, nx], f[2, 19, nz, ny, nx] or None) as numpy."""
        import torch

        nz, ny, nx = self.params.shape
        rho = torch.empty((2, nz, ny, nx), dtype=torch.float64, device=self.device)
        f = torch.empty((2, 19, nz, ny, nx), dtype=torch.float64, device=self.device) if populations else None
        _lib.check(
            self.lib.lb_export(
                self._ctx,
                ct.c_void_p(rho.data_ptr()),
                ct.c_void_p(f.data_ptr()) if f is not None else None,
                _stream_ptr(self.stream),
            )
        )
        return rho.cpu().numpy(), (f.cpu().numpy() if f is not None else None)

    def droplet_shape(self, xc: float, yc: float) -> dict:
        """Height, footprint half-lengths and contact angles (radians) of the droplet."""
        d = _lib.LbDroplet()
        _lib.check(self.lib.lb_droplet_shape(self._ctx, float(xc), float(yc), ct.byref(d), _stream_ptr(self.stream)))
        return {"height": d.height, "r_x": d.r_x, "r_y": d.r_y, "theta_x": d.theta_x, "theta_y": d.theta_y,
                "wet_nodes": d.wet_nodes}

    def deposit(self, n_bins_x: int, n_bins_y: int, xc: float, yc: float, strip_x: float, strip_y: float,
                bead_spacing: float = 2.0, r_contact: float = 5.25, x_src: float = 0.0, x_snk: float = 0.0) -> dict:
        """Deposit profiles g^b (Eq. 14) and S_x^b (Eq. 13) and the rod contact graph."""
        spec = _lib.LbDepositSpec(int(n_bins_x), int(n_bins_y), xc, yc, strip_x, strip_y, bead_spacing, r_contact,
                                  x_src, x_snk)
        gx, sx = np.zeros(n_bins_x), np.zeros(n_bins_x)
        gy, sy = np.zeros(n_bins_y), np.zeros(n_bins_y)
        nx_, ny_ = np.zeros(n_bins_x, np.int32), np.zeros(n_bins_y, np.int32)
        labels = np.zeros(max(self.n_rods, 1), np.int32)
        g = _lib.LbGraph()
        ptr = lambda a: a.ctypes.data_as(ct.c_void_p)
        _lib.check(self.lib.lb_deposit(self._ctx, ct.byref(spec), ptr(gx), ptr(sx), ptr(nx_), ptr(gy), ptr(sy),
                                       ptr(ny_), ptr(labels), ct.byref(g), _stream_ptr(self.stream)))
        return {"g_x": gx, "s_x": sx, "n_x": nx_, "g_y": gy, "s_y": sy, "n_y": ny_,
                "labels": labels[: self.n_rods], "edges": g.edges, "largest": g.largest,
                "spanning": bool(g.spanning)}

    def rod_beads(self, spacing: float = 1.0):
        """Beads of the rods (lb_rod_beads) as a CUDA FP64 tensor [n, 3]."""
        import torch

        n = ct.c_int32()
        # first call with no buffer: only the count (and LB_EINVAL if any)
        _lib.check(self.lib.lb_rod_beads(self._ctx, float(spacing), None, 0, ct.byref(n), _stream_ptr(self.stream)),
                   allow=(_lib.LB_OK, _lib.LB_EINVAL))
        pos = torch.empty((max(n.value, 1), 3), dtype=torch.float64, device=self.device)
        _lib.check(self.lib.lb_rod_beads(self._ctx, float(spacing), ct.c_void_p(pos.data_ptr()), int(pos.shape[0]),
                                         ct.byref(n), _stream_ptr(self.stream)))
        return pos[: n.value]

    def snapshot(self):
        """Device copy of the lattice's state for restore(): the current
        populations and the workspace (material map, rods, ledgers, status).
        The workspace holds device addresses of this lattice's own buffers,
        so a snapshot goes back only into the lattice that took it."""
        import torch

        torch.cuda.synchronize(self.device)
        cur = self.lib.lb_current_buffer(self._ctx)
        snap = (self.f[cur].clone(), self.ws.clone(), self.ws.data_ptr())
        torch.cuda.synchronize(self.device)
        return snap

    def restore(self, snap):
        """Return to a snapshot() of this lattice.  Between steps the other
        population buffer carries no state (a step writes everything the next
        one reads from it), so the saved populations go to whichever buffer is
        current now."""
        import torch

        f, ws, owner = snap
        if owner != self.ws.data_ptr():
            raise ValueError("snapshot of another lattice (its workspace points at that lattice's buffers)")
        torch.cuda.synchronize(self.device)
        cur = self.lib.lb_current_buffer(self._ctx)
        self.f[cur].copy_(f)
        self.ws.copy_(ws)
        torch.cuda.synchronize(self.device)

    def pressure(self, probes) -> np.ndarray:
        """Shan-Chen pressure at probe nodes [(x, y, z), ...] (NaN off the fluid)."""
        xyz = np.ascontiguousarray(np.asarray(probes, np.int32).reshape(-1, 3))
        out = np.zeros(len(xyz))
        _lib.check(self.lib.lb_pressure(self._ctx, xyz.ctypes.data_as(ct.c_void_p), len(xyz),
                                        out.ctypes.data_as(ct.c_void_p), _stream_ptr(self.stream)))
        return out

    def rod_map(self) -> np.ndarray:
        """Rod nodes per (y, x) column (z-projected occupancy)."""
        nz, ny, nx = self.params.shape
        m = np.zeros((ny, nx), np.int32)
        _lib.check(self.lib.lb_rod_map(self._ctx, m.ctypes.data_as(ct.c_void_p), _stream_ptr(self.stream)))
        return m

    def set_tiles(self, tile_y: int, rows_per_thread: int, zchunk: int = 0):
        t = _lib.LbTile(int(tile_y), int(rows_per_thread), int(zchunk), 0.0)
        _lib.check(self.lib.lb_set_tiles(self._ctx, ct.byref(t), _stream_ptr(self.stream)))
        return self

    def _tile_key(self):
        import torch

        p = self.params
        arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        return f"{arch}|{p.prec}|{'x'.join(str(v) for v in p.shape)}|tau1={p.tau == (1.0, 1.0)}"

    def autotune(self, trial_steps: int = 20, cache: str | None = None) -> dict:
        """Pick the fastest tile shape with lb_autotune (real steps), caching by lattice class.

        The cache is a JSON file keyed by (gfx arch, precision, lattice shape,
        tau = 1); a hit applies the stored shape without running trials.
        """
        path = cache or os.path.join(
            os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "paper_2607_06794_amd", "tiles.json")
        key = self._tile_key()
        table = {}
        try:
            with open(path) as fh:
                table = json.load(fh)
        except (OSError, ValueError):
            table = {}
        if key in table:
            t = table[key]
            self.set_tiles(t["tile_y"], t["rows_per_thread"], t["zchunk"])
            return dict(t, cached=True)
        best = _lib.LbTile()
        _lib.check(self.lib.lb_autotune(self._ctx, int(trial_steps), _stream_ptr(self.stream), ct.byref(best)))
        t = {"tile_y": best.tile_y, "rows_per_thread": best.rows_per_thread, "zchunk": best.zchunk,
             "us_per_step": best.us_per_step}
        table[key] = t
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path + ".tmp", "w") as fh:
                json.dump(table, fh, indent=1)
            os.replace(path + ".tmp", path)
        except OSError:
            pass
        return dict(t, cached=False)

    def close(self):
        if self._ctx:
            self.lib.lb_destroy(self._ctx)
            self._ctx = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def deposit_ensemble(lattices, n_bins_x: int, n_bins_y: int, xc: float, yc: float, strip_x: float, strip_y: float,
                     bead_spacing: float = 2.0, mirror: bool = True, stream=None) -> dict:
    """Deposit profiles g^b and S_x^b averaged over the rods of several
    lattices (independent runs) and, with mirror, their mirror images at
    (xc, yc) (lb_deposit_ensemble)."""
    lib = _lib.load()
    ctxs = (ct.c_void_p * len(lattices))(*[lat._ctx for lat in lattices])
    spec = _lib.LbDepositSpec(int(n_bins_x), int(n_bins_y), xc, yc, strip_x, strip_y, bead_spacing, 0.0, 0.0, 0.0)
    gx, sx, gy, sy = np.zeros(n_bins_x), np.zeros(n_bins_x), np.zeros(n_bins_y), np.zeros(n_bins_y)
    nx_, ny_ = np.zeros(n_bins_x, np.int32), np.zeros(n_bins_y, np.int32)
    ptr = lambda a: a.ctypes.data_as(ct.c_void_p)
    st = stream if stream is not None else lattices[0].stream
    _lib.check(lib.lb_deposit_ensemble(ctxs, len(lattices), ct.byref(spec), int(bool(mirror)), ptr(gx), ptr(sx),
                                       ptr(nx_), ptr(gy), ptr(sy), ptr(ny_), _stream_ptr(st)))
    return {"g_x": gx, "s_x": sx, "n_x": nx_, "g_y": gy, "s_y": sy, "n_y": ny_}


def kirchhoff(pos, r_c: float, x_src: float, x_snk: float, dV: float = 1.0, tol: float = 1e-12,
              max_iter: int = 20000, stream=None, noalloc: bool = False) -> dict:
    """Resistor network of a deposit (lb_kirchhoff, Eqs. 15-18) for bead
    positions `pos`, a CUDA FP64 tensor [n, 3]: potentials V and node
    currents I (CUDA tensors), I_tot, I_ref, kappa and the solve's counts.
    The solve's workspace is a torch tensor sized by
    lb_kirchhoff_workspace_bytes; noalloc=True calls lb_kirchhoff_noalloc,
    which uses the library's fixed device scratch instead."""
    import torch

    lib = _lib.load()
    pos = pos.to(torch.float64).contiguous()
    n = int(pos.shape[0])
    V = torch.empty(max(n, 1), dtype=torch.float64, device=pos.device)
    I = torch.empty_like(V)
    spec = _lib.LbKirchhoffSpec(float(r_c), float(x_src), float(x_snk), float(dV), float(tol), int(max_iter))
    out = _lib.LbKirchhoffOut()
    st = torch.cuda.current_stream(pos.device) if stream is None else stream
    if noalloc:
        _lib.check(lib.lb_kirchhoff_noalloc(ct.c_void_p(pos.data_ptr()), n, ct.byref(spec), ct.c_void_p(V.data_ptr()),
                                            ct.c_void_p(I.data_ptr()), ct.byref(out), _stream_ptr(st)))
    else:
        nb = int(lib.lb_kirchhoff_workspace_bytes(n))
        ws = torch.empty(nb + 256, dtype=torch.uint8, device=pos.device)
        wp = (ws.data_ptr() + 255) & ~255
        _lib.check(lib.lb_kirchhoff(ct.c_void_p(pos.data_ptr()), n, ct.byref(spec), ct.c_void_p(V.data_ptr()),
                                    ct.c_void_p(I.data_ptr()), ct.c_void_p(wp if n else None), nb, ct.byref(out),
                                    _stream_ptr(st)))
    return {"V": V[:n], "I": I[:n], "I_tot": out.I_tot, "I_ref": out.I_ref, "kappa": out.kappa,
            "rel_residual": out.rel_residual, "iterations": out.iterations, "edges": out.edges,
            "n_source": out.n_source, "n_sink": out.n_sink, "max_degree": out.max_degree}


class Batch:
    """Many lattices advanced by shared launches (the library's lb_batch).

    The lattices keep their own state; while the batch exists, step them only
    through it.  Results equal stepping each lattice alone.
    """

    def __init__(self, lattices, stream=None):
        import torch

        self.lattices = list(lattices)
        self.lib = _lib.load()
        self.device = self.lattices[0].device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        n = len(self.lattices)
        arr = (ct.c_void_p * n)(*[lat._ctx for lat in self.lattices])
        nbytes = self.lib.lb_batch_workspace_bytes(arr, n)
        if nbytes == 0:
            _lib.check(_lib.LB_EINVAL)
        self._ws = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self._b = ct.c_void_p()
        _lib.check(self.lib.lb_batch_create(arr, n, ct.c_void_p(self._ws.data_ptr()), _stream_ptr(self.stream),
                                            ct.byref(self._b)))

    def step(self, n: int = 1, rods: bool = True, graph: bool = True):
        _lib.check(self.lib.lb_batch_step(self._b, int(n), int(bool(rods)), int(bool(graph)), _stream_ptr(self.stream)))
        return self

    def close(self):
        if getattr(self, "_b", None):
            self.lib.lb_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
