"""Doubly periodic regular hexagonal Voronoi mesh, built in closed form.

Cell (r, c) sits at x = (c + (r mod 2)/2) dc, y = r dc sqrt(3)/2; the number of
rows must be even so the staggered rows close periodically.  Neighbours in
counter-clockwise order from the east are E, NE, NW, W, SW, SE; each cell owns
its E, NE and NW edges and its vertices at 30 and 90 degrees, so the mesh has
3N edges and 2N vertices.  Geometry is exact: d_e = dc, l_e = dc/sqrt(3),
A_i = (sqrt(3)/2) dc^2, every kite = A_i/6.
"""
from __future__ import annotations

import numpy as np

from .mesh import Mesh


def periodic_hex_mesh(nx: int, ny: int, dc: float, f0: float = 0.0,
                      name: str | None = None) -> Mesh:
    if ny % 2 != 0 or nx < 3 or ny < 4:
        raise ValueError("need nx >= 3 and an even ny >= 4")
    N = nx * ny
    r = np.repeat(np.arange(ny), nx)
    c = np.tile(np.arange(nx), ny)
    odd = (r % 2) == 1

    def cid(rr, cc):
        return (rr % ny) * nx + (cc % nx)

    E = cid(r, c + 1)
    W = cid(r, c - 1)
    NE = np.where(odd, cid(r + 1, c + 1), cid(r + 1, c))
    NW = np.where(odd, cid(r + 1, c), cid(r + 1, c - 1))
    SW = np.where(odd, cid(r - 1, c), cid(r - 1, c - 1))
    SE = np.where(odd, cid(r - 1, c + 1), cid(r - 1, c))
    i = np.arange(N)

    edgesOnCell = np.stack([3 * i, 3 * i + 1, 3 * i + 2, 3 * W, 3 * SW + 1, 3 * SE + 2], 1)
    cellsOnCell = np.stack([E, NE, NW, W, SW, SE], 1)
    verticesOnCell = np.stack([2 * i, 2 * i + 1, 2 * W, 2 * SW + 1, 2 * SW, 2 * SE + 1], 1)

    nE = 3 * N
    cellsOnEdge = np.empty((nE, 2), np.int64)
    verticesOnEdge = np.empty((nE, 2), np.int64)
    cellsOnEdge[0::3] = np.stack([i, E], 1)
    cellsOnEdge[1::3] = np.stack([i, NE], 1)
    cellsOnEdge[2::3] = np.stack([i, NW], 1)
    verticesOnEdge[0::3] = np.stack([2 * SE + 1, 2 * i], 1)
    verticesOnEdge[1::3] = np.stack([2 * i, 2 * i + 1], 1)
    verticesOnEdge[2::3] = np.stack([2 * i + 1, 2 * W], 1)

    nV = 2 * N
    cellsOnVertex = np.empty((nV, 3), np.int64)
    edgesOnVertex = np.empty((nV, 3), np.int64)
    cellsOnVertex[0::2] = np.stack([i, E, NE], 1)
    cellsOnVertex[1::2] = np.stack([i, NE, NW], 1)
    edgesOnVertex[0::2] = np.stack([3 * i, 3 * E + 2, 3 * i + 1], 1)
    edgesOnVertex[1::2] = np.stack([3 * i + 1, 3 * NW, 3 * i + 2], 1)

    s3 = np.sqrt(3.0)
    Lx = nx * dc
    Ly = ny * dc * s3 / 2.0
    R = dc / s3
    xc = (c + 0.5 * odd) * dc
    yc = r * dc * s3 / 2.0
    ang = np.deg2rad(np.array([0.0, 60.0, 120.0]))
    xe = (xc[:, None] + 0.5 * dc * np.cos(ang)[None, :]).reshape(-1) % Lx
    ye = (yc[:, None] + 0.5 * dc * np.sin(ang)[None, :]).reshape(-1) % Ly
    normal = np.tile(np.stack([np.cos(ang), np.sin(ang)], 1), (N, 1))
    vang = np.deg2rad(np.array([30.0, 90.0]))
    xv = (xc[:, None] + R * np.cos(vang)[None, :]).reshape(-1) % Lx
    yv = (yc[:, None] + R * np.sin(vang)[None, :]).reshape(-1) % Ly

    areaCell = np.full(N, s3 / 2.0 * dc * dc)
    kites = np.full((nV, 3), s3 / 12.0 * dc * dc)
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    return Mesh(
        nCells=N, nEdges=nE, nVertices=nV, maxEdges=6,
        nEdgesOnCell=np.full(N, 6, np.int32),
        edgesOnCell=i32(edgesOnCell), cellsOnCell=i32(cellsOnCell),
        verticesOnCell=i32(verticesOnCell),
        cellsOnEdge=i32(cellsOnEdge), verticesOnEdge=i32(verticesOnEdge),
        edgesOnVertex=i32(edgesOnVertex), cellsOnVertex=i32(cellsOnVertex),
        kiteAreasOnVertex=kites, areaCell=areaCell,
        areaTriangle=np.full(nV, s3 / 4.0 * dc * dc),
        dcEdge=np.full(nE, dc), dvEdge=np.full(nE, R),
        fVertex=np.full(nV, float(f0)), bottom=np.zeros(N),
        xCell=xc, yCell=yc, xEdge=xe, yEdge=ye, xVertex=xv, yVertex=yv,
        normalEdge=normal, Lx=Lx, Ly=Ly,
        name=name or f"hex{nx}x{ny}_dc{dc:g}")
