"""Doubly periodic planar Voronoi meshes and density-weighted Lloyd relaxation.

The mesh is the Voronoi diagram of a periodic point set, built from the
Delaunay triangulation of the points plus their periodic images within a
margin band (scipy.spatial.Delaunay).  Each Voronoi vertex is the circumcentre
of one periodic Delaunay triangle: of all images of a triangle, the one whose
circumcentre lies in [0, Lx) x [0, Ly) is kept.  Edge points x_e are the
midpoints of the cell-to-cell segments (where primal and dual edges cross).
Kite areas are the quadrilaterals (x_i, x_e1, x_v, x_e2); cell and triangle
areas are the sums of their kites, so the kites tile both meshes exactly.

Lloyd relaxation moves every point to the density-weighted centroid of its
Voronoi cell, integrated kite by kite with a degree-2 triangle rule.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import Delaunay

from .mesh import Mesh


def _extend(points, Lx, Ly, margin):
    N = len(points)
    P = [points]
    ids = [np.arange(N)]
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            if sx == 0 and sy == 0:
                continue
            p = points + np.array([sx * Lx, sy * Ly])
            keep = ((p[:, 0] > -margin) & (p[:, 0] < Lx + margin) &
                    (p[:, 1] > -margin) & (p[:, 1] < Ly + margin))
            P.append(p[keep])
            ids.append(np.nonzero(keep)[0])
    return np.concatenate(P), np.concatenate(ids)


def _circumcentres(X, S):
    a = X[S[:, 0]]
    b = X[S[:, 1]]
    c = X[S[:, 2]]
    bx, by = b[:, 0] - a[:, 0], b[:, 1] - a[:, 1]
    cx, cy = c[:, 0] - a[:, 0], c[:, 1] - a[:, 1]
    d = 2.0 * (bx * cy - by * cx)
    b2 = bx * bx + by * by
    c2 = cx * cx + cy * cy
    ux = (cy * b2 - by * c2) / d
    uy = (bx * c2 - cx * b2) / d
    return np.stack([a[:, 0] + ux, a[:, 1] + uy], 1)


def _tri_area(p, q, r):
    return 0.5 * ((q[:, 0] - p[:, 0]) * (r[:, 1] - p[:, 1]) -
                  (q[:, 1] - p[:, 1]) * (r[:, 0] - p[:, 0]))


def _star(points, Lx, Ly, margin):
    """Delaunay of the extended set; returns ext coords, orig ids, simplices,
    circumcentres and the (point, triangle, corner) star of original points."""
    N = len(points)
    X, oid = _extend(points, Lx, Ly, margin)
    tri = Delaunay(X)
    S = tri.simplices.astype(np.int64)
    cc = _circumcentres(X, S)
    t_idx, corner = np.nonzero(S < N)
    p_idx = S[t_idx, corner]
    return X, oid, S, cc, p_idx, t_idx, corner


def _margin(points, Lx, Ly):
    N = len(points)
    return 6.0 * math.sqrt(Lx * Ly / N) if N < 1000 else 0.06 * max(Lx, Ly) + 6.0 * math.sqrt(Lx * Ly / N)


def lloyd_step(points, Lx, Ly, density, margin=None):
    """One density-weighted Lloyd iteration; returns the new (wrapped) points."""
    N = len(points)
    if margin is None:
        margin = _margin(points, Lx, Ly)
    X, oid, S, cc, p_idx, t_idx, corner = _star(points, Lx, Ly, margin)
    xp = X[p_idx]
    xa = X[S[t_idx, (corner + 1) % 3]]
    xb = X[S[t_idx, (corner + 2) % 3]]
    ma = 0.5 * (xp + xa)
    mb = 0.5 * (xp + xb)
    o = cc[t_idx]
    mass = np.zeros(N)
    mx = np.zeros(N)
    my = np.zeros(N)
    for (p, q, r) in ((xp, ma, o), (xp, o, mb)):
        A = _tri_area(p, q, r)
        # degree-2 rule: edge midpoints with weight 1/3 each
        for (s, t) in ((p, q), (q, r), (r, p)):
            m = 0.5 * (s + t)
            w = A / 3.0 * density(m[:, 0] % Lx, m[:, 1] % Ly)
            mass += np.bincount(p_idx, w, N)
            mx += np.bincount(p_idx, w * m[:, 0], N)
            my += np.bincount(p_idx, w * m[:, 1], N)
    new = np.stack([mx / mass, my / mass], 1)
    new[:, 0] %= Lx
    new[:, 1] %= Ly
    return new


def periodic_voronoi_mesh(points, Lx, Ly, f0=0.0, name="voronoi",
                          margin=None) -> Mesh:
    points = np.asarray(points, np.float64)
    N = len(points)
    if margin is None:
        margin = _margin(points, Lx, Ly)
    X, oid, S, cc, p_idx, t_idx, corner = _star(points, Lx, Ly, margin)

    # canonical Voronoi vertex per periodic triangle: key = sorted original ids
    ko = np.sort(oid[S], axis=1)
    key = (ko[:, 0] * N + ko[:, 1]) * N + ko[:, 2]
    kept = (cc[:, 0] >= 0) & (cc[:, 0] < Lx) & (cc[:, 1] >= 0) & (cc[:, 1] < Ly)
    kkeys = key[kept]
    order = np.argsort(kkeys)
    kkeys_sorted = kkeys[order]
    if len(kkeys_sorted) > 1 and (np.diff(kkeys_sorted) == 0).any():
        raise ValueError("periodic triangle images are not unique; mesh too small")
    kept_tri = np.nonzero(kept)[0][order]
    nV = len(kept_tri)

    # star of each original point, counter-clockwise by circumcentre angle
    xp = X[p_idx]
    ang = np.arctan2(cc[t_idx, 1] - xp[:, 1], cc[t_idx, 0] - xp[:, 0])
    srt = np.lexsort((ang, p_idx))
    p_s, t_s, c_s = p_idx[srt], t_idx[srt], corner[srt]
    nEoC = np.bincount(p_s, minlength=N)
    maxE = int(nEoC.max())
    start = np.concatenate([[0], np.cumsum(nEoC)[:-1]])
    slot = np.arange(len(p_s)) - np.repeat(start, nEoC)
    vid = np.searchsorted(kkeys_sorted, key[t_s])
    if not (kkeys_sorted[np.minimum(vid, nV - 1)] == key[t_s]).all():
        raise ValueError("star triangle without a canonical vertex; margin too small")

    # previous triangle in the ring (cyclic): edge j lies between v_{j-1} and v_j
    prev = np.arange(len(p_s)) - 1
    prev[start] = start + nEoC - 1
    t_prev = t_s[prev]
    # neighbour point across edge j: common point of t_prev and t_s other than p
    Sp = S[t_prev]
    Sc = S[t_s]
    nb = np.full(len(p_s), -1, np.int64)
    for a in range(3):
        cand = Sc[:, a]
        shared = (Sp == cand[:, None]).any(1) & (cand != p_s)
        nb = np.where(shared, cand, nb)
    if (nb < 0).any():
        raise ValueError("broken Delaunay star")

    va = vid[prev]
    vb = vid
    ekey = np.minimum(va, vb).astype(np.int64) * nV + np.maximum(va, vb)
    ukeys, first, einv = np.unique(ekey, return_index=True, return_inverse=True)
    nE = len(ukeys)
    # each edge must appear exactly twice (once from each cell)
    if not (np.bincount(einv, minlength=nE) == 2).all():
        raise ValueError("edge not shared by exactly two cells")

    edgesOnCell = np.full((N, maxE), -1, np.int64)
    cellsOnCell = np.full((N, maxE), -1, np.int64)
    verticesOnCell = np.full((N, maxE), -1, np.int64)
    edgesOnCell[p_s, slot] = einv
    cellsOnCell[p_s, slot] = oid[nb]
    # vertex between edge j and edge j+1 is v_j
    verticesOnCell[p_s, slot] = vid

    # per-edge data from its first occurrence: n_e from that cell to the other
    f = first
    c0 = p_s[f]
    c1 = oid[nb[f]]
    x0 = X[p_s[f]]
    x1 = X[nb[f]]
    dvec = x1 - x0
    dcE = np.hypot(dvec[:, 0], dvec[:, 1])
    normal = dvec / dcE[:, None]
    xe = 0.5 * (x0 + x1)
    ccA = cc[t_prev[f]]
    ccB = cc[t_s[f]]
    dvE = np.hypot(*(ccB - ccA).T)
    cellsOnEdge = np.stack([c0, c1], 1)
    # traversing the cell counter-clockwise goes from v_{j-1} to v_j along +t_e
    verticesOnEdge = np.stack([va[f], vb[f]], 1)

    # kites: cell p_s, vertex v_j, quad (x_p, m_j, cc_j, m_{j+1})
    nxt = np.arange(len(p_s)) + 1
    last = start + nEoC - 1
    nxt[last] = start
    m_j = 0.5 * (xp[srt] + X[nb])
    m_n = m_j[nxt]
    o = cc[t_s]
    kite = _tri_area(xp[srt], m_j, o) + _tri_area(xp[srt], o, m_n)
    if (kite <= 0).any():
        raise ValueError("non-positive kite area (circumcentre outside its kite)")
    areaCell = np.bincount(p_s, kite, N)

    # vertex-based arrays
    cellsOnVertex = oid[S[kept_tri]]
    kites_v = np.zeros((nV, 3))
    for k in range(3):
        m = cellsOnVertex[vid, k] == p_s
        kites_v[vid[m], k] = kite[m]
    if (kites_v <= 0).any():
        raise ValueError("vertex kite lookup failed")
    # edges on vertex: each edge contributes to its two vertices
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

    xv = cc[kept_tri]
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    return Mesh(
        nCells=N, nEdges=nE, nVertices=nV, maxEdges=maxE,
        nEdgesOnCell=i32(nEoC), edgesOnCell=i32(edgesOnCell),
        cellsOnCell=i32(cellsOnCell), verticesOnCell=i32(verticesOnCell),
        cellsOnEdge=i32(cellsOnEdge), verticesOnEdge=i32(verticesOnEdge),
        edgesOnVertex=i32(eov), cellsOnVertex=i32(cellsOnVertex),
        kiteAreasOnVertex=kites_v, areaCell=areaCell,
        areaTriangle=kites_v.sum(1), dcEdge=dcE, dvEdge=dvE,
        fVertex=np.full(nV, float(f0)), bottom=np.zeros(N),
        xCell=points[:, 0].copy(), yCell=points[:, 1].copy(),
        xEdge=xe[:, 0] % Lx, yEdge=xe[:, 1] % Ly,
        xVertex=xv[:, 0], yVertex=xv[:, 1], normalEdge=normal,
        Lx=float(Lx), Ly=float(Ly), name=name)


# ---------------------------------------------------------------------------
# Variable-resolution point sets

def tanh_spacing(d, dc_in, dc_out, r0, width):
    """Target cell spacing: dc_in inside radius r0, dc_out outside, tanh blend."""
    return dc_in + (dc_out - dc_in) * 0.5 * (1.0 + np.tanh((d - r0) / width))


def sample_points(n, Lx, Ly, spacing_fn, seed):
    """n seeded points with density proportional to spacing^-2 (rejection)."""
    rng = np.random.default_rng(seed)
    out = []
    got = 0
    smin = None
    while got < n:
        m = max(4 * (n - got), 1024)
        p = rng.random((m, 2)) * np.array([Lx, Ly])
        s = spacing_fn(p[:, 0], p[:, 1])
        if smin is None:
            smin = float(s.min())
        acc = rng.random(m) < (smin / s) ** 2
        out.append(p[acc])
        got += int(acc.sum())
    return np.concatenate(out)[:n]


def jittered_hex_points(nx, ny, dc, jitter, seed):
    """Regular hex lattice points moved by a seeded uniform jitter (fraction of dc)."""
    rng = np.random.default_rng(seed)
    r = np.repeat(np.arange(ny), nx)
    c = np.tile(np.arange(nx), ny)
    x = (c + 0.5 * (r % 2)) * dc
    y = r * dc * math.sqrt(3.0) / 2.0
    p = np.stack([x, y], 1) + jitter * dc * (rng.random((nx * ny, 2)) - 0.5)
    Lx = nx * dc
    Ly = ny * dc * math.sqrt(3.0) / 2.0
    p[:, 0] %= Lx
    p[:, 1] %= Ly
    return p, Lx, Ly


def ring_hex_points(nx, ny, dc, n_ring, r_ring, iters):
    """A hex lattice whose points within 1.9 dc of the domain centre are
    replaced by the centre and a regular ring of n_ring points at radius
    r_ring dc, both held in place while the other points take `iters`
    uniform Lloyd steps: the Voronoi mesh has one n_ring-sided cell (up to
    11 with n_ring = 11, r_ring = 1.2, iters = 20) among mostly hexagons."""
    p, Lx, Ly = jittered_hex_points(nx, ny, dc, 0.0, seed=0)
    c = np.array([Lx / 2, Ly / 2])
    keep = np.hypot(*(p - c).T) > 1.9 * dc
    ang = 2.0 * math.pi * np.arange(n_ring) / n_ring
    ring = c + r_ring * dc * np.stack([np.cos(ang), np.sin(ang)], 1)
    pts = np.concatenate([c[None], ring, p[keep]])
    pinned = pts[:1 + n_ring].copy()
    for _ in range(iters):
        pts = lloyd_step(pts, Lx, Ly, lambda x, y: np.ones_like(x))
        pts[:1 + n_ring] = pinned
    return pts, Lx, Ly


# ---------------------------------------------------------------------------
# The variable-resolution planar workload

VR_DOMAIN = 2.0e6          # doubly periodic 2000 km x 2000 km
VR_RADIUS = 1.5e5          # fine disk radius 150 km
VR_WIDTH = 5.0e4           # tanh transition width 50 km
VR_RATIO = 8.0             # dc_out / dc_in (2 km inside, 16 km outside)


def vr_spacing_shape(x, y):
    """Relative target spacing (1 inside the disk, 8 outside, tanh blend)."""
    d = np.hypot(x - VR_DOMAIN / 2, y - VR_DOMAIN / 2)
    return tanh_spacing(d, 1.0, VR_RATIO, VR_RADIUS, VR_WIDTH)


def vr_points(n: int, seed: int, iters: int, progress=None):
    """Seeded points Lloyd-relaxed under density rho ~ spacing^-4."""
    L = VR_DOMAIN
    p = sample_points(n, L, L, vr_spacing_shape, seed)
    dens = lambda x, y: vr_spacing_shape(x, y) ** -4.0
    for it in range(iters):
        p = lloyd_step(p, L, L, dens)
        if progress:
            progress(it)
    return p


# A three-resolution variant (more than two LTS levels, Remark 3.1): spacing 1
# inside a 60 km disk, 2 in a ring out to 300 km, 8 outside.
VR3_R1, VR3_W1 = 6.0e4, 1.5e4
VR3_R2, VR3_W2 = 3.0e5, 5.0e4
VR3_MID = 2.0


def vr3_spacing_shape(x, y):
    """Relative target spacing of the three-resolution workload (1, 2, 8 with
    tanh blends of 15 and 50 km)."""
    d = np.hypot(x - VR_DOMAIN / 2, y - VR_DOMAIN / 2)
    return (1.0 + (VR3_MID - 1.0) * 0.5 * (1.0 + np.tanh((d - VR3_R1) / VR3_W1)) +
            (VR_RATIO - VR3_MID) * 0.5 * (1.0 + np.tanh((d - VR3_R2) / VR3_W2)))


def vr3_points(n: int, seed: int, iters: int, progress=None):
    """Seeded points Lloyd-relaxed under rho ~ spacing^-4 (three resolutions)."""
    L = VR_DOMAIN
    p = sample_points(n, L, L, vr3_spacing_shape, seed)
    dens = lambda x, y: vr3_spacing_shape(x, y) ** -4.0
    for it in range(iters):
        p = lloyd_step(p, L, L, dens)
        if progress:
            progress(it)
    return p


def morton_sort(points, L):
    q = np.clip((points / L * 65535.0).astype(np.int64), 0, 65535)

    def spread(v):
        v = (v | (v << 8)) & 0x00FF00FF
        v = (v | (v << 4)) & 0x0F0F0F0F
        v = (v | (v << 2)) & 0x33333333
        v = (v | (v << 1)) & 0x55555555
        return v
    key = spread(q[:, 0]) | (spread(q[:, 1]) << 1)
    return points[np.argsort(key, kind="stable")]
