"""Initial states and fine-region masks for the synthetic workloads.

* Linear inertia-gravity wave on an f-plane (periodic hexagonal mesh): the
  height perturbation A cos(phi), phi = k x + l y - omega t, with the velocity
  of the linearised rotating shallow water equations,
  omega^2 = f^2 + g H (k^2 + l^2).
* Gaussian height bump at rest (variable-resolution planar meshes).
* Seeded random states for operator parity tests.

Velocities are sampled as point values u_e = u(x_e) . n_e at the edge points;
heights as point values at cell centres.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .mesh import Mesh


@dataclass
class IGWParams:
    g: float
    H: float
    f: float
    amp: float
    k: float
    l: float
    omega: float

    @property
    def period(self) -> float:
        return 2.0 * math.pi / self.omega


def igw_parameters(mesh: Mesh, g=9.81, H=1000.0, f=1.0e-4, amp=1.0,
                   mode=(2, 1)) -> IGWParams:
    k = 2.0 * math.pi * mode[0] / mesh.Lx
    l = 2.0 * math.pi * mode[1] / mesh.Ly
    omega = math.sqrt(f * f + g * H * (k * k + l * l))
    return IGWParams(g, H, f, amp, k, l, omega)


def igw_state(mesh: Mesh, p: IGWParams, t: float = 0.0):
    """Height at cells and normal velocity at edges of the linear wave at time t."""
    phi_c = p.k * mesh.xCell + p.l * mesh.yCell - p.omega * t
    h = p.H + p.amp * np.cos(phi_c)
    phi_e = p.k * mesh.xEdge + p.l * mesh.yEdge - p.omega * t
    kap2 = p.k * p.k + p.l * p.l
    s = p.amp / (p.H * kap2)
    uu = s * (p.omega * p.k * np.cos(phi_e) - p.f * p.l * np.sin(phi_e))
    vv = s * (p.omega * p.l * np.cos(phi_e) + p.f * p.k * np.sin(phi_e))
    u = uu * mesh.normalEdge[:, 0] + vv * mesh.normalEdge[:, 1]
    return h, u


def strip_fine_mask(mesh: Mesh, row_lo: int, row_hi: int, dc: float) -> np.ndarray:
    """Fine mask for hex rows row_lo..row_hi inclusive (a horizontal strip)."""
    row = np.rint(mesh.yCell / (dc * math.sqrt(3.0) / 2.0)).astype(np.int64)
    return ((row >= row_lo) & (row <= row_hi)).astype(np.uint8)


def periodic_distance(mesh: Mesh, x, y, cx: float, cy: float):
    dx = np.abs(x - cx)
    dy = np.abs(y - cy)
    if mesh.Lx > 0:
        dx = np.minimum(dx, mesh.Lx - dx)
        dy = np.minimum(dy, mesh.Ly - dy)
    return np.hypot(dx, dy)


def disk_fine_mask(mesh: Mesh, cx: float, cy: float, radius: float) -> np.ndarray:
    d = periodic_distance(mesh, mesh.xCell, mesh.yCell, cx, cy)
    return (d < radius).astype(np.uint8)


def gaussian_bump_state(mesh: Mesh, H: float, amp: float, sigma: float,
                        cx: float, cy: float):
    d = periodic_distance(mesh, mesh.xCell, mesh.yCell, cx, cy)
    h = H + amp * np.exp(-0.5 * (d / sigma) ** 2)
    u = np.zeros(mesh.nEdges)
    return h, u


def random_state(mesh: Mesh, seed: int, H=1000.0, amp_h=1.0, amp_u=0.5):
    rng = np.random.default_rng(seed)
    h = H + amp_h * rng.standard_normal(mesh.nCells)
    u = amp_u * rng.standard_normal(mesh.nEdges)
    return h, u
