"""Seeded synthetic Eulerian fields: velocity on the staggered (MAC) lattices of each box, and the
conformation tensor at the cell centres.

The finite-volume fluid solve is not part of the coupling step; these fields
stand in for its output.  Component ``d`` of box ``b`` is sampled at
``origin + (i + s_d) h`` with ``s_d = 1/2`` on the two axes other than ``d``
and ``0`` on axis ``d`` (u_x at (i, j+1/2, k+1/2) h, and so on), stored in a
``[3][total_cells]`` array with x fastest.

Each field is a sum of divergence-free Fourier modes
``a_m cos(kappa_m . (x - origin) + theta_m)`` with ``a_m . kappa_m = 0``,
periodic on the box.  Evaluation uses torch so that large grids can be
synthesised on the device; the CPU and GPU consumers are always handed the
same array.
"""
from __future__ import annotations

import math

import numpy as np
import torch

# lattice offsets in cells: the three velocity components, then the cell centres (comp 3)
STAGGER = np.array([[0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0], [0.5, 0.5, 0.5]])
CONFORMATION = ("xx", "yy", "zz", "xy", "xz", "yz")


def draw_modes(rng: np.random.Generator, n_modes: int = 8, kmax: int = 4, amp: float = 1.0):
    """Integer wave numbers in [-kmax, kmax]^3 \\ 0, unit-free amplitudes and phases."""
    ks, amps, phases = [], [], []
    while len(ks) < n_modes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if not np.any(k):
            continue
        ks.append(k)
        amps.append(amp * rng.uniform(0.0, 1.0))
        phases.append(rng.uniform(0.0, 2 * np.pi))
    dirs = rng.normal(size=(n_modes, 3))
    return np.asarray(ks, dtype=np.float64), np.asarray(amps), np.asarray(phases), dirs


def _mode_vectors(box, ks, amps, dirs):
    L = np.array(box.length)
    kap = 2 * np.pi * ks / L[None, :]
    a = dirs - (np.einsum("ij,ij->i", dirs, kap) / np.einsum("ij,ij->i", kap, kap))[:, None] * kap
    a = a / np.linalg.norm(a, axis=1, keepdims=True) * amps[:, None]
    return kap, a


def _plane_wave(kap, phase, coords):
    """cos(kx x + ky y + kz z + phase) on the (nz, ny, nx) lattice, separably:
    cos(a + b) = cos a cos b - sin a sin b with a on x and b on the (z, y) plane."""
    a = kap[0] * coords[0]
    b = kap[2] * coords[2][:, None] + kap[1] * coords[1][None, :] + phase
    return torch.cos(b)[:, :, None] * torch.cos(a)[None, None, :] - torch.sin(b)[:, :, None] * torch.sin(a)[None, None, :]


def fourier_field(box, modes, comp: int, device="cpu", dtype=torch.float64, shear_rate: float = 0.0):
    """Sample component ``comp`` of the mode sum on its staggered lattice, shape (nz, ny, nx)."""
    ks, amps, phases, dirs = modes
    kap, a = _mode_vectors(box, ks, amps, dirs)
    nx, ny, nz = box.n
    s = STAGGER[comp]
    coords = [(torch.arange(n, dtype=torch.float64, device=device) + s[i]) * box.h for i, n in enumerate((nx, ny, nz))]
    out = torch.zeros((nz, ny, nx), dtype=torch.float64, device=device)
    for m in range(kap.shape[0]):
        if a[m, comp] == 0.0:
            continue
        out += a[m, comp] * _plane_wave(kap[m], phases[m], coords)
    if shear_rate and comp == 0:
        Ly = box.length[1]
        out += shear_rate * Ly / (2 * math.pi) * torch.sin(2 * math.pi * coords[1] / Ly)[None, :, None]
    return out.to(dtype)


def scene_velocity(scene, seed: int | None = None, device="cpu", dtype=torch.float64, n_modes: int = 8,
                   shear_rate: float = 0.0, mode_amp: float = 1.0):
    """[3][total_cells] velocity for every box of ``scene`` (one mode set per box)."""
    rng = np.random.default_rng(scene.seed + 77 if seed is None else seed)
    total = scene.total_cells
    u = torch.empty((3, total), dtype=dtype, device=device)
    off = scene.cell_offset
    for b, box in enumerate(scene.boxes):
        modes = draw_modes(rng, n_modes, amp=mode_amp)
        for d in range(3):
            u[d, off[b]:off[b + 1]] = fourier_field(box, modes, d, device, dtype, shear_rate).reshape(-1)
    return u


def lattice_positions(box, comp: int) -> np.ndarray:
    """Node coordinates of lattice ``comp`` as (nz, ny, nx, 3) float64 (tests only)."""
    nx, ny, nz = box.n
    s = STAGGER[comp]
    g = [box.origin[i] + (np.arange(n) + s[i]) * box.h for i, n in enumerate((nx, ny, nz))]
    Z, Y, X = np.meshgrid(g[2], g[1], g[0], indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def random_forces(scene, seed: int = 5, scale: float = 1.0) -> np.ndarray:
    """[3][n_nodes] float64 nodal force field for transfer tests that do not need element forces."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=(3, scene.n_nodes))


def conformation_field(scene, seed: int | None = None, amp: float = 0.2, n_modes: int = 6, device="cpu",
                       dtype=torch.float64):
    """[6][total_cells] conformation tensor C = I + perturbation at the cell centres of every box
    (components xx, yy, zz, xy, xz, yz).  Each component's perturbation is a sum of periodic Fourier
    modes scaled so that its magnitude stays below ``amp``; with amp <= 1/3 every C is symmetric
    positive definite (diagonal >= 1 - amp, off-diagonal row sums <= 2 amp)."""
    rng = np.random.default_rng(scene.seed + 91 if seed is None else seed)
    out = torch.empty((6, scene.total_cells), dtype=dtype, device=device)
    off = scene.cell_offset
    for b, box in enumerate(scene.boxes):
        L = np.array(box.length)
        nx, ny, nz = box.n
        coords = [(torch.arange(n, dtype=torch.float64, device=device) + 0.5) * box.h for n in (nx, ny, nz)]
        for c in range(6):
            ks, amps, phases, _ = draw_modes(rng, n_modes)
            amps = amps / max(amps.sum(), 1e-300) * amp * rng.uniform(0.5, 1.0)
            kap = 2 * np.pi * ks / L[None, :]
            f = torch.full((nz, ny, nx), 1.0 if c < 3 else 0.0, dtype=torch.float64, device=device)
            for m in range(n_modes):
                f += amps[m] * _plane_wave(kap[m], phases[m], coords)
            out[c, off[b]:off[b + 1]] = f.reshape(-1).to(dtype)
    return out
