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
# Three resolutions (800k cells): the multi-level LTS3 workload

VR3_SEED = 2106071542
VR3_N = 800_000
VR3_ITERS = 30


def _vr3_cache_path(n, seed, iters):
    return os.path.join(DATA, f"vr3_{n}_s{seed}_i{iters}_u32.npy")


def vr3_points_cached(n=VR3_N, seed=VR3_SEED, iters=VR3_ITERS, progress=None):
    path = _vr3_cache_path(n, seed, iters)
    L = vp.VR_DOMAIN
    if os.path.exists(path):
        q = np.load(path, allow_pickle=False)
        return q.astype(np.float64) * (L / 2.0 ** 32)
    p = vp.morton_sort(vp.vr3_points(n, seed, iters, progress), L)
    return quantize(p, L).astype(np.float64) * (L / 2.0 ** 32)


def vr3_planar(n=VR3_N, seed=VR3_SEED, iters=VR3_ITERS, H=500.0, amp=5.0, sigma=4.0e4,
               M=8, progress=None) -> Workload:
    """Three resolutions in the 2000 km periodic domain: target spacing 1
    inside a 60 km disk, 2 in a ring to 300 km, 8 outside (tanh blends of 15
    and 50 km); Gaussian bump over H = 500 m at rest; fine region (level 0):
    target spacing below 0.9 of the outer one; `extra["level1_mask"]`: target
    spacing below 1.5 (the disk, for an inner level with ratio 2); fine step
    0.3 of the gravity-wave crossing time of the smallest cell."""
    L = vp.VR_DOMAIN
    pts = vr3_points_cached(n, seed, iters, progress)
    m = vp.periodic_voronoi_mesh(pts, L, L, f0=1.0e-4, name=f"vr3-{n}")
    shape = vp.vr3_spacing_shape(m.xCell, m.yCell)
    fm = (shape < 0.9 * vp.VR_RATIO).astype(np.uint8)
    h0, u0 = gaussian_bump_state(m, H, amp, sigma, L / 2, L / 2)
    c = math.sqrt(9.81 * H)
    spacing = np.sqrt(m.areaCell / (math.sqrt(3.0) / 2.0))
    dt_fine = 0.3 * spacing.min() / c
    return Workload(f"vr3-planar-{n // 1000}k", m, fm, h0, u0, dt_fine * M, M,
                    extra=dict(dt_fine=dt_fine, spacing_min=float(spacing.min()),
                               spacing_max=float(spacing.max()), H=H,
                               level1_mask=(shape < 1.5).astype(np.uint8)))


# ---------------------------------------------------------------------------
# The batched ensemble: 64 members of 10k-400k cells (log-uniform, seeded)

ENS_SEED = 7000


def ensemble_sizes(n_members=64, lo=1.0e4, hi=4.0e5, seed=ENS_SEED):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n_members)).astype(np.int64)


# Members whose relaxed points are cached in data/ (written by
# make_ensemble_points.py): two of each size class, one above 300k cells, M
# covering {2, 4, 8}; the oracle-checked ensemble test uses them.
ENS_CACHED = (20, 40, 24, 33, 62, 23)


def _member_cache_path(j, n_cells, iters, seed):
    return os.path.join(DATA, f"ens{j}_n{int(n_cells)}_s{seed}_i{iters}_u32.npy")


def member_points(j, n_cells, iters=10, seed=ENS_SEED):
    """Relaxed generator points of member j (Morton-sorted) and the Lloyd
    iterations taken: n_cells seeded points of the variable-resolution
    planar family, Lloyd-relaxed at least `iters` times and then two at a
    time until every kite area is positive and no cell has more than 8 edges
    (at most 40 iterations)."""
    L = vp.VR_DOMAIN
    p = vp.sample_points(int(n_cells), L, L, vp.vr_spacing_shape, seed + j)
    dens = lambda x, y: vp.vr_spacing_shape(x, y) ** -4.0
    done = 0
    while True:
        for _ in range(iters if done == 0 else 2):
            p = vp.lloyd_step(p, L, L, dens)
            done += 1
        ps = vp.morton_sort(p, L)
        try:
            m = vp.periodic_voronoi_mesh(ps, L, L, f0=1.0e-4, name=f"member{j}")
            if m.maxEdges <= 8 or done >= 40:
                return ps, done
        except ValueError:
            if done >= 40:
                raise


def ensemble_member(j, n_cells, iters=10, seed=ENS_SEED) -> Workload:
    """Member j: the variable-resolution planar family scaled to n_cells
    (member_points; read from data/ when cached there as uint32 fixed-point
    coordinates); bump 5(1 + 0.2 z) m, sigma 40(1 + 0.1 z) km, centre jittered
    by up to 50 km; M drawn from {2, 4, 8}."""
    rng = np.random.default_rng(seed + j)
    L = vp.VR_DOMAIN
    path = _member_cache_path(j, n_cells, iters, seed)
    if os.path.exists(path):
        q = np.load(path, allow_pickle=False)
        p, done = q[:-1].astype(np.float64) * (L / 2.0 ** 32), int(q[-1, 0])
    else:
        p, done = member_points(j, n_cells, iters, seed)
    m = vp.periodic_voronoi_mesh(p, L, L, f0=1.0e-4, name=f"member{j}")
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


# ---------------------------------------------------------------------------
# The variable-resolution sphere (1.6M cells)

SPH_SEED = 2106071541
SPH_N = 1_600_000
SPH_ITERS = 30


def _sphere_cache_path(n, seed, iters):
    return os.path.join(DATA, f"sphere{n}_s{seed}_i{iters}_deg8_u32.npy")


def sphere_points(n=SPH_N, seed=SPH_SEED, iters=SPH_ITERS, progress=None):
    """The relaxation recipe: `iters` Lloyd iterations from the seeded sample,
    Morton order, uint32 fixed point, then further iterations (each followed
    by the same ordering and fixed point) until no cell has more than 8
    edges.  Returns the fixed-point (longitude, latitude) array."""
    from . import voronoi_sphere as vs
    q = vs.quantize_lonlat(vs.morton_sort_sphere(vs.cap_points(n, seed, iters, progress)))
    dens = lambda x: vs.cap_spacing_shape(x) ** -4.0
    extra = 0
    while vs.max_cell_degree(vs.dequantize_lonlat(q)) > 8:
        if extra >= 20:
            raise ValueError("cells with more than 8 edges remain")
        p = vs.lloyd_step_sphere(vs.dequantize_lonlat(q), dens)
        q = vs.quantize_lonlat(vs.morton_sort_sphere(p))
        extra += 1
        if progress:
            progress(iters + extra - 1)
    return q


def sphere_points_cached(n=SPH_N, seed=SPH_SEED, iters=SPH_ITERS, progress=None):
    from . import voronoi_sphere as vs
    path = _sphere_cache_path(n, seed, iters)
    if os.path.exists(path):
        return vs.dequantize_lonlat(np.load(path, allow_pickle=False))
    return vs.dequantize_lonlat(sphere_points(n, seed, iters, progress))


def _plane_wave_field(x, kmax, n_waves, rng):
    """Random-phase superposition of n_waves plane waves exp(i R k.x) with
    random directions and |k| R uniform in [1, kmax], restricted to the unit
    vectors x: a smooth random field whose spectrum ends near degree kmax.
    Returned with zero mean and unit RMS over the points."""
    d = rng.standard_normal((n_waves, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    k = rng.uniform(1.0, kmax, n_waves)
    ph = rng.uniform(0.0, 2 * math.pi, n_waves)
    amp = 1.0 / k
    f = np.zeros(len(x))
    for j in range(n_waves):
        f += amp[j] * np.cos(k[j] * (x @ d[j]) + ph[j])
    f -= f.mean()
    return f / math.sqrt(np.mean(f * f))


def sphere_state(m, u0=20.0, depth=5000.0, noise_rms=10.0, topo_rms=500.0, seed=SPH_SEED,
                 g=9.81):
    """Zonal flow u = u0 cos(lat) in gradient-wind balance (the surface height
    of the steady zonal-flow solution on the rotating sphere), random
    topography (plane-wave spectrum up to degree 16, 500 m RMS), random height
    noise (up to degree 32, 10 m RMS), mean depth 5000 m.  Sets m.bottom;
    returns (h, u)."""
    from . import voronoi_sphere as vs
    R, Om = vs.EARTH_RADIUS, vs.OMEGA
    rng = np.random.default_rng(seed + 3)
    xc = np.stack([m.xCell, m.yCell, m.zCell], 1) / R
    lat = np.arcsin(np.clip(xc[:, 2], -1, 1))
    b = topo_rms * _plane_wave_field(xc, 16.0, 256, np.random.default_rng(seed + 4))
    m.bottom = b
    surf = -(R * Om * u0 + 0.5 * u0 * u0) * np.sin(lat) ** 2 / g
    h = surf - b + noise_rms * _plane_wave_field(xc, 32.0, 256, rng)
    h += depth - np.sum(m.areaCell * h) / np.sum(m.areaCell)
    xe = np.stack([m.xEdge, m.yEdge, m.zEdge], 1) / R
    late = np.arcsin(np.clip(xe[:, 2], -1, 1))
    lone = np.arctan2(xe[:, 1], xe[:, 0])
    east = np.stack([-np.sin(lone), np.cos(lone), np.zeros_like(lone)], 1)
    u = u0 * np.cos(late) * np.einsum("ij,ij->i", east, m.normalEdge)
    return h, u


def tc5_state(m, u0=20.0, h0=5960.0, hs0=2000.0, g=9.81):
    """Zonal flow over an isolated mountain (the standard shallow-water test
    case 5): u = u0 cos(lat), surface h + b = h0 - (R Omega u0 + u0^2/2)
    sin^2(lat) / g, conical mountain b = hs0 (1 - r / (pi/9)) with r the
    (lon, lat) distance from (3 pi/2, pi/6), capped at pi/9.  Sets m.bottom;
    returns (h, u)."""
    from . import voronoi_sphere as vs
    R, Om = vs.EARTH_RADIUS, vs.OMEGA
    xc = np.stack([m.xCell, m.yCell, m.zCell], 1) / R
    lat = np.arcsin(np.clip(xc[:, 2], -1, 1))
    lon = np.mod(np.arctan2(xc[:, 1], xc[:, 0]), 2 * math.pi)
    rm = math.pi / 9.0
    r = np.minimum(rm, np.sqrt((lon - vs.CAP_LON) ** 2 + (lat - vs.CAP_LAT) ** 2))
    b = hs0 * (1.0 - r / rm)
    m.bottom = b
    h = h0 - (R * Om * u0 + 0.5 * u0 * u0) * np.sin(lat) ** 2 / g - b
    xe = np.stack([m.xEdge, m.yEdge, m.zEdge], 1) / R
    late = np.arcsin(np.clip(xe[:, 2], -1, 1))
    lone = np.arctan2(xe[:, 1], xe[:, 0])
    east = np.stack([-np.sin(lone), np.cos(lone), np.zeros_like(lone)], 1)
    u = u0 * np.cos(late) * np.einsum("ij,ij->i", east, m.normalEdge)
    return h, u


def sphere_cap(n=SPH_N, seed=SPH_SEED, iters=SPH_ITERS, M=4, progress=None,
               case="jet") -> Workload:
    """The variable-resolution sphere: n points Lloyd-relaxed `iters` times
    under rho ~ s^-4 with s 1 inside a 20-degree cap at (3 pi/2, pi/6) and 4
    outside (3-degree tanh transition), radius 6371 km, f = 2 Omega sin(lat);
    balanced zonal jet over random topography; fine region: target spacing
    below 0.9 of the outer one; interface 2 + 2 rings; the fine step is 0.3 of
    the crossing time of the smallest cell at the fastest gravity-wave speed
    plus the jet speed."""
    from . import voronoi_sphere as vs
    P = sphere_points_cached(n, seed, iters, progress)
    m = vs.sphere_voronoi_mesh(P, name=f"sphere{n}")
    xc = np.stack([m.xCell, m.yCell, m.zCell], 1) / vs.EARTH_RADIUS
    fm = (vs.cap_spacing_shape(xc) < 0.9 * vs.CAP_RATIO).astype(np.uint8)
    h0, u0 = tc5_state(m) if case == "tc5" else sphere_state(m, seed=seed)
    spacing = np.sqrt(m.areaCell / (math.sqrt(3.0) / 2.0))
    c = math.sqrt(9.81 * float((h0 + m.bottom).max())) + 20.0
    dt_fine = 0.3 * spacing.min() / c
    name = f"sphere-{n // 1000}k" + ("-tc5" if case == "tc5" else "")
    return Workload(name, m, fm, h0, u0, dt_fine * M, M,
                    extra=dict(dt_fine=dt_fine, spacing_min=float(spacing.min()),
                               spacing_max=float(spacing.max())))
