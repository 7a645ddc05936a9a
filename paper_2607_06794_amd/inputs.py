"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module builds initial density fields, material maps and rod lists.  It
holds geometry and random numbers only -- none of the lattice Boltzmann
arithmetic -- so that the HIP path and the oracle can both start from the
same data without sharing any of the method's code.

Random numbers come from ``numpy.random.Generator(PCG64(seed))``; the order
of every draw is fixed and documented per function.

Material codes: 0 fluid, 1 top reservoir plane, 2 hydrophilic stripe,
3 hydrophobic surround, 8 rod.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

FLUID, GHOST, STRIPE, SURROUND, ROD = 0, 1, 2, 3, 8


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def add_noise(rho, amplitude, seed):
    """Independent U[-a, a] on every rho_k at every node, drawn in [k][z][y][x] order."""
    if amplitude == 0:
        return rho
    return rho + _rng(seed).uniform(-amplitude, amplitude, size=rho.shape)


def sphere_droplet(shape, radius, rho_in=1.0, rho_out=0.03, noise=1e-4, seed=1000):
    """Static spherical droplet in a periodic box.

    Node (x, y, z) is inside iff |x - c| <= R with c = (n/2 - 1/2) per axis.
    Component A: rho_in inside, rho_out outside; component B mirrored.
    Returns (rho[2, nz, ny, nx] float64, material[nz, ny, nx] uint8).
    """
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d2 = (x - (nx / 2 - 0.5)) ** 2 + (y - (ny / 2 - 0.5)) ** 2 + (z - (nz / 2 - 0.5)) ** 2
    ins = d2 <= radius * radius
    rho = np.empty((2,) + tuple(shape))
    rho[0] = np.where(ins, rho_in, rho_out)
    rho[1] = np.where(ins, rho_out, rho_in)
    rho = add_noise(rho, noise, seed)
    return rho, np.zeros(shape, np.uint8)


@dataclass
class CapSpec:
    """Ellipsoidal sessile cap on a wall with a wettable stripe and a reservoir top."""

    shape: tuple = (64, 128, 256)  # (nz, ny, nx)
    footprint: tuple = (150.0, 36.0)  # full lengths along x, y
    height: float = 24.0
    stripe: tuple = (160, 40)  # full lengths along x, y
    rho_in: float = 1.0
    rho_out: float = 0.03
    noise: float = 1e-4
    seed: int = 2000
    reservoir: bool = True


def sessile_cap(spec: CapSpec):
    """Elongated droplet on a patterned wall.

    Wall plane z = 0 (surround material, stripe of full size stripe[0] x
    stripe[1] centred at ((nx-1)/2, (ny-1)/2)); reservoir plane z = nz-1 when
    ``spec.reservoir``; x and y periodic.  Cap: ((x-cx)/a)^2 + ((y-cy)/b)^2 +
    ((z-1/2)/h)^2 <= 1 for z >= 1 with a, b the footprint half-lengths and h
    the height (the wall surface sits at z = 1/2).
    """
    nz, ny, nx = spec.shape
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a, b = spec.footprint[0] / 2.0, spec.footprint[1] / 2.0
    ins = ((x - cx) / a) ** 2 + ((y - cy) / b) ** 2 + ((z - 0.5) / spec.height) ** 2 <= 1.0
    ins &= z >= 1
    mat = np.zeros(spec.shape, np.uint8)
    mat[0] = SURROUND
    sx, sy = spec.stripe
    in_stripe = (np.abs(x[0] - cx) <= sx / 2.0) & (np.abs(y[0] - cy) <= sy / 2.0)
    mat[0][in_stripe] = STRIPE
    if spec.reservoir:
        mat[-1] = GHOST
    rho = np.empty((2,) + tuple(spec.shape))
    rho[0] = np.where(ins, spec.rho_in, spec.rho_out)
    rho[1] = np.where(ins, spec.rho_out, spec.rho_in)
    rho = add_noise(rho, spec.noise, spec.seed)
    solid = mat != FLUID
    rho[:, solid] = 0.0
    return rho, mat


def channel(shape, rho=1.0):
    """Single-component channel between walls at z = 0 and z = nz-1 (Poiseuille)."""
    nz, ny, nx = shape
    mat = np.zeros(shape, np.uint8)
    mat[0] = SURROUND
    mat[-1] = SURROUND
    r = np.zeros((2,) + tuple(shape))
    r[0] = rho
    r[:, mat != FLUID] = 0.0
    return r, mat
