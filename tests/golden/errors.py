"""Error measures of the 16-bit storage forms against the oracle's fields
(plain NumPy on exported states; no lattice Boltzmann arithmetic).  Shared
by the script that writes the expected values, the GPU tests and the
benchmark's error report."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CONFIG3_ORACLE = os.path.join(HERE, "config3_oracle_1e4.npz")
CONFIG3_MODEL = os.path.join(HERE, "config3_rounding_model.json")


def velocity(rho, f):
    """Post-collision barycentric velocity sum_k sum_i f_i^k c_i / sum_k rho_k
    of an exported state (f[2][19][z][y][x], D3Q19 in the library's order)."""
    c = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 0], [-1, -1, 0],
                  [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1],
                  [0, 1, -1], [0, -1, 1]], dtype=float)
    j = np.einsum("kiabc,id->dabc", f, c)
    tot = rho[0] + rho[1]
    return j / np.where(tot > 0, tot, 1.0)


def field_errors(rho, u, rho_o, u_o, mass=None, mass_o=None):
    """Errors of (rho, u) against the oracle's (rho_o, u_o): per field the
    relative max and RMS (over max |oracle|; the velocity over max |u_o|),
    and per phase (liquid C > 0.5, gas C < -0.5, interface, C from the
    oracle) the absolute max and RMS of each density."""
    out = {}
    for k, name in ((0, "rho_A"), (1, "rho_B")):
        d = rho[k] - rho_o[k]
        s = np.abs(rho_o[k]).max()
        out[name] = {"max": float(np.abs(d).max() / s), "rms": float(np.sqrt((d * d).mean()) / s)}
    du = np.sqrt(((u - u_o) ** 2).sum(axis=0))
    su = np.sqrt((u_o ** 2).sum(axis=0)).max()
    out["u"] = {"max": float(du.max() / su), "rms": float(np.sqrt((du * du).mean()) / su)}
    C = (rho_o[0] - rho_o[1]) / (rho_o[0] + rho_o[1])
    for ph, sel in (("liquid", C > 0.5), ("gas", C < -0.5), ("interface", np.abs(C) <= 0.5)):
        for k, name in ((0, "rho_A"), (1, "rho_B")):
            d = (rho[k] - rho_o[k])[sel]
            out[f"{ph}_{name}"] = {"max": float(np.abs(d).max()), "rms": float(np.sqrt((d * d).mean()))}
    if mass is not None:
        out["mass_rel"] = [float(abs(mass[k] - mass_o[k]) / mass_o[k]) for k in range(2)]
    return out


def liquid_centre(rho):
    """Centre (x, y, z) of the liquid (C > 0 weight (1 + C) / 2) in a periodic
    box: per axis the argument of the circular mean of the weight."""
    C = (rho[0] - rho[1]) / np.where(rho[0] + rho[1] > 0, rho[0] + rho[1], 1.0)
    wgt = 0.5 * (1.0 + C)
    out = []
    for ax, a in ((2, 0), (1, 1), (0, 2)):  # array axes z, y, x -> x, y, z
        n = rho.shape[1 + ax]
        prof = wgt.sum(axis=tuple(b for b in range(3) if b != ax))
        ang = 2 * np.pi * np.arange(n) / n
        out.append(np.angle((prof * np.exp(1j * ang)).sum()) * n / (2 * np.pi))
    return np.array(out)


def periodic_shift(field, d):
    """field (..., nz, ny, nx) translated by d = (dx, dy, dz) (band-limited
    interpolation on the periodic box)."""
    nz, ny, nx = field.shape[-3:]
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.fftfreq(nx)[None, None, :]
    ph = np.exp(-2j * np.pi * (kx * d[0] + ky * d[1] + kz * d[2]))
    return np.real(np.fft.ifftn(np.fft.fftn(field, axes=(-3, -2, -1)) * ph, axes=(-3, -2, -1)))


def aligned_errors(rho, u, rho_o, u_o):
    """The liquid centre displacement of (rho, u) against the oracle's
    (minimum image), and the field errors after translating (rho, u) back by
    it: what is left once the rigid drift is taken out."""
    d = liquid_centre(rho) - liquid_centre(rho_o)
    n = np.array(rho.shape[1:][::-1], dtype=float)
    d -= n * np.round(d / n)
    out = field_errors(periodic_shift(rho, -d), periodic_shift(u, -d), rho_o, u_o)
    out["displacement"] = [float(v) for v in d]
    return out


UNIT_ROUNDOFF = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def rounding_walk(rho_o, rho_ref, fmt, steps):
    """Random-walk model of the conserved totals under stochastic rounding:
    a stored value d_i = f_i - w_i rho_ref that lies a fraction p of the
    spacing h above its lower neighbour moves by -p h or (1 - p) h, mean
    zero, variance p (1 - p) h^2 <= h^2 / 4 with h <= 2 u |d_i| (u the
    format's unit roundoff), independent between populations and steps; with
    d_i taken at rest, d_i = w_i (rho_k - rho_ref), the mass of component k
    walks with
      sigma_M = u sqrt(steps sum_i w_i^2 sum_x (rho_k - rho_ref)^2).
    Returns sigma_M / M_k for k = 0, 1."""
    u = UNIT_ROUNDOFF[fmt]
    s2 = 1.0 / 9.0 + 6.0 / 18.0 ** 2 + 12.0 / 36.0 ** 2  # sum_i w_i^2
    dev2 = [float(((rho_o[k] - rho_ref) ** 2).sum()) for k in range(2)]
    mk = [float(rho_o[k].sum()) for k in range(2)]
    return [u * np.sqrt(steps * s2 * dev2[k]) / mk[k] for k in range(2)]
