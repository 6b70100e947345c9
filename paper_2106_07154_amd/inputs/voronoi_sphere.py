"""Spherical centroidal Voronoi meshes and the variable-resolution sphere
workload.

The mesh is the Voronoi diagram of a point set on the unit sphere, built from
its Delaunay triangulation (the convex hull of the points,
scipy.spatial.ConvexHull), scaled to radius R.  Voronoi vertices are the
circumcentres of the Delaunay triangles on the sphere; edge points x_e are the
midpoints of the great-circle arcs between neighbouring cells (where primal
and dual edges cross).  Kite areas are the spherical quadrilaterals
(x_i, x_e1, x_v, x_e2); cell and triangle areas are the sums of their kites,
so the kites tile both meshes and the sphere exactly.  Distances are
great-circle arc lengths.  Orientation conventions are those of mesh.py with
k the outward normal of the sphere.

Lloyd relaxation moves every point to the density-weighted centroid of its
Voronoi cell (kite by kite, a degree-2 triangle rule on the chordal
triangles, projected back onto the sphere).
"""
from __future__ import annotations

import math
import os

import numpy as np

from .mesh import Mesh

EARTH_RADIUS = 6.371e6
OMEGA = 7.292e-5

# The variable-resolution sphere: fine cap of 20 degrees around
# (lon, lat) = (3 pi / 2, pi / 6), spacing ratio 4 (60 -> 15 km), tanh
# transition of 3 degrees.
CAP_LON = 1.5 * math.pi
CAP_LAT = math.pi / 6.0
CAP_RADIUS = math.radians(20.0)
CAP_WIDTH = math.radians(3.0)
CAP_RATIO = 4.0


def _unit(v):
    return v / np.linalg.norm(v, axis=1)[:, None]


def _sph_tri_area(a, b, c):
    """Signed area of the spherical triangle (a, b, c) on the unit sphere
    (positive counter-clockwise seen from outside)."""
    num = np.einsum("ij,ij->i", a, np.cross(b, c))
    den = 1.0 + np.einsum("ij,ij->i", a, b) + np.einsum("ij,ij->i", b, c) + \
        np.einsum("ij,ij->i", c, a)
    return 2.0 * np.arctan2(num, den)


def _arc(a, b):
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.einsum("ij,ij->i", a, b))


def _delaunay(P):
    """Triangles of the convex hull, counter-clockwise seen from outside, and
    their circumcentres on the unit sphere."""
    from scipy.spatial import ConvexHull
    S = ConvexHull(P).simplices.astype(np.int64)
    a, b, c = P[S[:, 0]], P[S[:, 1]], P[S[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, a) < 0
    S[flip] = S[flip][:, [0, 2, 1]]
    n[flip] = -n[flip]
    return S, _unit(n)


def _star(P, S, cc):
    """(point, triangle, corner) incidences sorted counter-clockwise around
    each point by the direction of the circumcentre in the tangent plane."""
    N = len(P)
    t_idx = np.repeat(np.arange(len(S)), 3)
    corner = np.tile(np.arange(3), len(S))
    p_idx = S[t_idx, corner]
    p = P[p_idx]
    ref = np.where(np.abs(p[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    e1 = _unit(np.cross(ref, p))
    e2 = np.cross(p, e1)
    d = cc[t_idx]
    ang = np.arctan2(np.einsum("ij,ij->i", d, e2), np.einsum("ij,ij->i", d, e1))
    srt = np.lexsort((ang, p_idx))
    return p_idx[srt], t_idx[srt], corner[srt], N


def lloyd_step_sphere(P, density):
    """One density-weighted Lloyd iteration on the unit sphere."""
    N = len(P)
    S, cc = _delaunay(P)
    t_idx = np.repeat(np.arange(len(S)), 3)
    corner = np.tile(np.arange(3), len(S))
    p_idx = S[t_idx, corner]
    xp = P[p_idx]
    ma = _unit(xp + P[S[t_idx, (corner + 1) % 3]])
    mb = _unit(xp + P[S[t_idx, (corner + 2) % 3]])
    o = cc[t_idx]
    mass = np.zeros(N)
    acc = np.zeros((N, 3))
    for (p, q, r) in ((xp, ma, o), (xp, o, mb)):
        A = _sph_tri_area(p, q, r)
        for (s, t) in ((p, q), (q, r), (r, p)):
            m = _unit(s + t)
            w = A / 3.0 * density(m)
            mass += np.bincount(p_idx, w, N)
            for k in range(3):
                acc[:, k] += np.bincount(p_idx, w * m[:, k], N)
    return _unit(acc / mass[:, None])


def sphere_voronoi_mesh(P, radius=EARTH_RADIUS, omega=OMEGA, name="sphere") -> Mesh:
    """MPAS-style Voronoi mesh of the unit vectors P on a sphere of `radius`;
    f = 2 omega sin(latitude) at vertices."""
    P = _unit(np.asarray(P, np.float64))
    S, cc = _delaunay(P)
    nV = len(S)
    p_s, t_s, c_s, N = _star(P, S, cc)
    nEoC = np.bincount(p_s, minlength=N)
    maxE = int(nEoC.max())
    start = np.concatenate([[0], np.cumsum(nEoC)[:-1]])
    slot = np.arange(len(p_s)) - np.repeat(start, nEoC)
    prev = np.arange(len(p_s)) - 1
    prev[start] = start + nEoC - 1
    t_prev = t_s[prev]
    # neighbour across edge j: the common point of t_prev and t_s other than p
    Sp, Sc = S[t_prev], S[t_s]
    nb = np.full(len(p_s), -1, np.int64)
    for a in range(3):
        cand = Sc[:, a]
        shared = (Sp == cand[:, None]).any(1) & (cand != p_s)
        nb = np.where(shared, cand, nb)
    if (nb < 0).any():
        raise ValueError("broken Delaunay star")
    va, vb = t_prev, t_s
    ekey = np.minimum(va, vb) * nV + np.maximum(va, vb)
    ukeys, first, einv = np.unique(ekey, return_index=True, return_inverse=True)
    nE = len(ukeys)
    if not (np.bincount(einv, minlength=nE) == 2).all():
        raise ValueError("edge not shared by exactly two cells")
    edgesOnCell = np.full((N, maxE), -1, np.int64)
    cellsOnCell = np.full((N, maxE), -1, np.int64)
    verticesOnCell = np.full((N, maxE), -1, np.int64)
    edgesOnCell[p_s, slot] = einv
    cellsOnCell[p_s, slot] = nb
    verticesOnCell[p_s, slot] = vb

    f = first
    c0, c1 = p_s[f], nb[f]
    x0, x1 = P[c0], P[c1]
    xe = _unit(x0 + x1)
    d = x1 - x0
    normal = _unit(d - np.einsum("ij,ij->i", d, xe)[:, None] * xe)
    dcE = radius * _arc(x0, x1)
    dvE = radius * _arc(cc[va[f]], cc[vb[f]])
    cellsOnEdge = np.stack([c0, c1], 1)
    verticesOnEdge = np.stack([va[f], vb[f]], 1)

    # kites: cell p_s, vertex v_j, quad (x_p, m_j, cc_j, m_{j+1})
    nxt = np.arange(len(p_s)) + 1
    last = start + nEoC - 1
    nxt[last] = start
    xp = P[p_s]
    m_j = _unit(xp + P[nb])
    m_n = m_j[nxt]
    o = cc[t_s]
    kite = (_sph_tri_area(xp, m_j, o) + _sph_tri_area(xp, o, m_n)) * radius ** 2
    if (kite <= 0).any():
        raise ValueError("non-positive kite area (circumcentre outside its kite)")
    areaCell = np.bincount(p_s, kite, N)

    cellsOnVertex = S
    kites_v = np.zeros((nV, 3))
    for k in range(3):
        m = cellsOnVertex[t_s, k] == p_s
        kites_v[t_s[m], k] = kite[m]
    if (kites_v <= 0).any():
        raise ValueError("vertex kite lookup failed")
    eov = np.full((nV, 3), -1, np.int64)
    cnt = np.zeros(nV, np.int64)
    for side in range(2):
        vv = verticesOnEdge[:, side]
        o2 = np.argsort(vv, kind="stable")
        vv_s = vv[o2]
        st = np.searchsorted(vv_s, vv_s, side="left")
        rank = np.arange(len(vv_s)) - st
        eov[vv_s, cnt[vv_s] + rank] = o2
        cnt += np.bincount(vv, minlength=nV)
    if (cnt != 3).any():
        raise ValueError("vertex degree is not 3")

    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    xc, xee, xv = radius * P, radius * xe, radius * cc
    return Mesh(
        nCells=N, nEdges=nE, nVertices=nV, maxEdges=maxE,
        nEdgesOnCell=i32(nEoC), edgesOnCell=i32(edgesOnCell),
        cellsOnCell=i32(cellsOnCell), verticesOnCell=i32(verticesOnCell),
        cellsOnEdge=i32(cellsOnEdge), verticesOnEdge=i32(verticesOnEdge),
        edgesOnVertex=i32(eov), cellsOnVertex=i32(cellsOnVertex),
        kiteAreasOnVertex=kites_v, areaCell=areaCell,
        areaTriangle=kites_v.sum(1), dcEdge=dcE, dvEdge=dvE,
        fVertex=2.0 * omega * cc[:, 2], bottom=np.zeros(N),
        xCell=xc[:, 0].copy(), yCell=xc[:, 1].copy(),
        xEdge=xee[:, 0].copy(), yEdge=xee[:, 1].copy(),
        xVertex=xv[:, 0].copy(), yVertex=xv[:, 1].copy(), normalEdge=normal,
        zCell=xc[:, 2].copy(), zEdge=xee[:, 2].copy(), zVertex=xv[:, 2].copy(),
        Lx=0.0, Ly=0.0, name=name)


# ---------------------------------------------------------------------------
# Variable-resolution point sets on the sphere

def lonlat_to_xyz(lon, lat):
    return np.stack([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)], -1)


CAP_CENTRE = lonlat_to_xyz(np.array(CAP_LON), np.array(CAP_LAT))


def cap_spacing_shape(x):
    """Relative target spacing at unit vectors x: 1 in the cap, CAP_RATIO
    outside, tanh blend in the angular distance from the cap centre."""
    d = np.arccos(np.clip(x @ CAP_CENTRE, -1.0, 1.0))
    return 1.0 + (CAP_RATIO - 1.0) * 0.5 * (1.0 + np.tanh((d - CAP_RADIUS) / CAP_WIDTH))


def sample_sphere(n, spacing_fn, seed):
    """n seeded unit vectors with areal density proportional to spacing^-2."""
    rng = np.random.default_rng(seed)
    out, got = [], 0
    while got < n:
        m = max(4 * (n - got), 1024)
        p = _unit(rng.standard_normal((m, 3)))
        acc = rng.random(m) < (1.0 / spacing_fn(p)) ** 2
        out.append(p[acc])
        got += int(acc.sum())
    return np.concatenate(out)[:n]


def cap_points(n, seed, iters, progress=None):
    """Seeded points Lloyd-relaxed on the sphere under rho ~ spacing^-4."""
    p = sample_sphere(n, cap_spacing_shape, seed)
    dens = lambda x: cap_spacing_shape(x) ** -4.0
    for it in range(iters):
        p = lloyd_step_sphere(p, dens)
        if progress:
            progress(it)
    return p


def max_cell_degree(P):
    """Largest number of Voronoi edges of a cell (Delaunay degree)."""
    from scipy.spatial import ConvexHull
    return int(np.bincount(ConvexHull(P).simplices.ravel(), minlength=len(P)).max())


def relax_to_degree(P, max_degree=8, max_extra=20, progress=None):
    """Further Lloyd iterations until no cell has more than max_degree edges;
    returns (points, iterations done)."""
    dens = lambda x: cap_spacing_shape(x) ** -4.0
    done = 0
    while max_cell_degree(P) > max_degree:
        if done >= max_extra:
            raise ValueError("cells with too many edges remain")
        P = lloyd_step_sphere(P, dens)
        done += 1
        if progress:
            progress(done)
    return P, done


def morton_sort_sphere(P):
    """Order unit vectors along a 3-D Morton curve (locality of cell ids)."""
    q = np.clip(((P + 1.0) * 0.5 * 1023.0).astype(np.int64), 0, 1023)

    def spread(v):
        v = (v | (v << 16)) & 0x030000FF
        v = (v | (v << 8)) & 0x0300F00F
        v = (v | (v << 4)) & 0x030C30C3
        v = (v | (v << 2)) & 0x09249249
        return v
    key = spread(q[:, 0]) | (spread(q[:, 1]) << 1) | (spread(q[:, 2]) << 2)
    return P[np.argsort(key, kind="stable")]


def quantize_lonlat(P):
    lon = np.mod(np.arctan2(P[:, 1], P[:, 0]), 2 * math.pi)
    lat = np.arcsin(np.clip(P[:, 2], -1.0, 1.0))
    qlon = np.minimum(np.floor(lon / (2 * math.pi) * 2.0 ** 32), 2.0 ** 32 - 1)
    qlat = np.minimum(np.floor((lat / math.pi + 0.5) * 2.0 ** 32), 2.0 ** 32 - 1)
    return np.stack([qlon, qlat], 1).astype(np.uint32)


def dequantize_lonlat(Q):
    lon = (Q[:, 0].astype(np.float64) + 0.5) / 2.0 ** 32 * 2 * math.pi
    lat = ((Q[:, 1].astype(np.float64) + 0.5) / 2.0 ** 32 - 0.5) * math.pi
    return lonlat_to_xyz(lon, lat)
