"""The synthetic workloads: meshes, fine masks, initial states and time steps.

* ``igw_hex``: 64 x 64 doubly periodic hexagonal mesh, dc = 10 km, f-plane
  f = 1e-4, g = 9.81, flat bottom H = 1000 m; linear inertia-gravity wave of
  amplitude 1 m and wavenumber (2, 1); fine strip of hex rows 28-35 with two
  interface rings each side; M = 4, coarse dt = 30 s.
* ``vr_planar``: doubly periodic 2000 x 2000 km Voronoi mesh of 200,000 seeded
  points Lloyd-relaxed 50 times under density rho ~ s^-4, where the target
  spacing s is 1 inside a 150 km disk and 8 outside with a 50 km tanh
  transition (the 2 km / 16 km shape; at 200k cells the actual spacing is
  about 0.6 km inside and 6.8 km outside).  Gaussian bump 5 m, sigma 40 km,
  over H = 500 m at rest, f = 1e-4.  Fine region: target spacing below 0.9 of
  the outer one; interface 2 + 2 rings; M = 8.  The fine step is 0.3 of the
  gravity-wave crossing time of the smallest cell.

The relaxed points of ``vr_planar`` are cached as uint32 fixed-point
coordinates in ``data/`` (written by ``make_vr_points.py``, which re-runs the
seeded relaxation); the mesh is rebuilt from them on every run.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

from .cases import gaussian_bump_state, igw_parameters, igw_state, strip_fine_mask
from .hexmesh import periodic_hex_mesh
from .mesh import Mesh
from . import voronoi_planar as vp

DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
VR_SEED = 2106071540
VR_N = 200_000
VR_ITERS = 50


@dataclass
class Workload:
    name: str
    mesh: Mesh
    fine_mask: np.ndarray
    h0: np.ndarray
    u0: np.ndarray
    dt_coarse: float
    M: int
    n_if1: int = 2
    n_if2: int = 2
    gravity: float = 9.81
    extra: dict = field(default_factory=dict)


def igw_hex() -> Workload:
    m = periodic_hex_mesh(64, 64, 1.0e4, f0=1.0e-4, name="hex64x64_dc10km")
    p = igw_parameters(m, g=9.81, H=1000.0, f=1.0e-4, amp=1.0, mode=(2, 1))
    h0, u0 = igw_state(m, p, 0.0)
    fm = strip_fine_mask(m, 28, 35, 1.0e4)
    return Workload("igw-hex64", m, fm, h0, u0, 30.0, 4, extra=dict(igw=p))


def _vr_cache_path(n, seed, iters):
    return os.path.join(DATA, f"vr{n}_s{seed}_i{iters}_u32.npy")


def vr_points_cached(n=VR_N, seed=VR_SEED, iters=VR_ITERS, progress=None):
    path = _vr_cache_path(n, seed, iters)
    L = vp.VR_DOMAIN
    if os.path.exists(path):
        q = np.load(path, allow_pickle=False)
        return q.astype(np.float64) * (L / 2.0 ** 32)
    p = vp.morton_sort(vp.vr_points(n, seed, iters, progress), L)
    return quantize(p, L).astype(np.float64) * (L / 2.0 ** 32)


def quantize(p, L):
    return np.minimum(np.floor(p / L * 2.0 ** 32), 2.0 ** 32 - 1).astype(np.uint32)


def vr_planar(n=VR_N, seed=VR_SEED, iters=VR_ITERS, H=500.0, amp=5.0, sigma=4.0e4,
              M=8, progress=None) -> Workload:
    L = vp.VR_DOMAIN
    pts = vr_points_cached(n, seed, iters, progress)
    m = vp.periodic_voronoi_mesh(pts, L, L, f0=1.0e-4, name=f"vr{n}")
    fm = (vp.vr_spacing_shape(m.xCell, m.yCell) < 0.9 * vp.VR_RATIO).astype(np.uint8)
    h0, u0 = gaussian_bump_state(m, H, amp, sigma, L / 2, L / 2)
    c = math.sqrt(9.81 * H)
    spacing = np.sqrt(m.areaCell / (math.sqrt(3.0) / 2.0))
    dt_fine = 0.3 * spacing.min() / c
    return Workload(f"vr-planar-{n // 1000}k", m, fm, h0, u0, dt_fine * M, M,
                    extra=dict(dt_fine=dt_fine, spacing_min=float(spacing.min()),
                               spacing_max=float(spacing.max()), H=H))


# ---------------------------------------------------------------------------
# The batched ensemble: 64 members of 10k-400k cells (log-uniform, seeded)

ENS_SEED = 7000


def ensemble_sizes(n_members=64, lo=1.0e4, hi=4.0e5, seed=ENS_SEED):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n_members)).astype(np.int64)


def ensemble_member(j, n_cells, iters=10, seed=ENS_SEED) -> Workload:
    """Member j: the variable-resolution planar family scaled to n_cells,
    Lloyd-relaxed at least `iters` times and then two at a time until every
    kite area is positive and no cell has more than 8 edges (at most 40
    iterations); bump 5(1 + 0.2 z) m, sigma 40(1 + 0.1 z) km, centre jittered
    by up to 50 km; M drawn from {2, 4, 8}."""
    rng = np.random.default_rng(seed + j)
    L = vp.VR_DOMAIN
    p = vp.sample_points(int(n_cells), L, L, vp.vr_spacing_shape, seed + j)
    dens = lambda x, y: vp.vr_spacing_shape(x, y) ** -4.0
    done = 0
    m = None
    while m is None:
        for _ in range(iters if done == 0 else 2):
            p = vp.lloyd_step(p, L, L, dens)
            done += 1
        try:
            m = vp.periodic_voronoi_mesh(vp.morton_sort(p, L), L, L, f0=1.0e-4, name=f"member{j}")
            if m.maxEdges > 8 and done < 40:
                m = None
        except ValueError:
            if done >= 40:
                raise
    fm = (vp.vr_spacing_shape(m.xCell, m.yCell) < 0.9 * vp.VR_RATIO).astype(np.uint8)
    z = rng.standard_normal(2)
    cx, cy = L / 2 + rng.uniform(-5.0e4, 5.0e4, 2)
    H = 500.0
    h0, u0 = gaussian_bump_state(m, H, 5.0 * (1 + 0.2 * z[0]), 4.0e4 * (1 + 0.1 * z[1]), cx, cy)
    M = int(rng.choice([2, 4, 8]))
    spacing = np.sqrt(m.areaCell / (math.sqrt(3.0) / 2.0))
    dt_fine = 0.3 * spacing.min() / math.sqrt(9.81 * H)
    return Workload(f"member{j}", m, fm, h0, u0, dt_fine * M, M,
                    extra=dict(dt_fine=dt_fine, H=H, lloyd_iterations=done))


def _member_job(args):
    return ensemble_member(*args)


def ensemble_members(n_members=64, iters=10, workers=None, seed=ENS_SEED):
    """Generate the members in a pool of spawned processes (call before any GPU
    initialisation in the calling process)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    sizes = ensemble_sizes(n_members, seed=seed)
    jobs = [(j, int(sizes[j]), iters, seed) for j in range(n_members)]
    workers = workers or min(16, os.cpu_count() or 1)
    order = sorted(range(n_members), key=lambda j: -sizes[j])  # big ones first
    out = [None] * n_members
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        futs = {ex.submit(_member_job, jobs[j]): j for j in order}
        for f in cf.as_completed(futs):
            out[futs[f]] = f.result()
    return out


# ---------------------------------------------------------------------------
# Training trajectories of the fine-region surrogate (on the vr_planar mesh)

SUR_SEED = 8000


def surrogate_initial_state(mesh, i, H=500.0, seed=SUR_SEED):
    """Initial state of trajectory i: a Gaussian bump of 5(1 + 0.2 z) m,
    sigma 40(1 + 0.1 z) km, centre jittered by up to 50 km around the
    domain centre, at rest over H = 500 m."""
    rng = np.random.default_rng(seed + i)
    z = rng.standard_normal(2)
    L = vp.VR_DOMAIN
    cx, cy = L / 2 + rng.uniform(-5.0e4, 5.0e4, 2)
    return gaussian_bump_state(mesh, H, 5.0 * (1 + 0.2 * z[0]), 4.0e4 * (1 + 0.1 * z[1]), cx, cy)
