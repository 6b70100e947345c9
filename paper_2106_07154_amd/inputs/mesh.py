"""MPAS-style mesh container for Voronoi C-grid meshes (planar periodic or spherical).

Connectivity follows the sets of the TRiSK appendix of the paper (EC, EV, CE,
VE, EE) with these orientation conventions, which the library and the oracle
both document and rely on:

* ``cellsOnEdge[e] = (c0, c1)``: the edge normal n_e points from c0 to c1, so
  n_{e,c0} = +1 (outward for c0) and n_{e,c1} = -1.
* ``verticesOnEdge[e] = (v0, v1)``: the tangent t_e = k x n_e points from v0 to
  v1, so t_{e,v1} = +1 (v1 is the left end of e) and t_{e,v0} = -1.
* ``edgesOnCell[i, :nEdgesOnCell[i]]`` runs counter-clockwise around cell i;
  ``verticesOnCell[i, j]`` is the vertex shared by ``edgesOnCell[i, j]`` and
  ``edgesOnCell[i, j+1]``; ``cellsOnCell[i, j]`` is the cell across
  ``edgesOnCell[i, j]``.  Unused slots hold -1.
* ``kiteAreasOnVertex[v, k]`` is the area of the part of cell
  ``cellsOnVertex[v, k]`` cut by the kite (x_i, x_e1, x_v, x_e2).

All index arrays are int32, 0-based; geometry is float64 in metres.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Mesh:
    nCells: int
    nEdges: int
    nVertices: int
    maxEdges: int
    nEdgesOnCell: np.ndarray
    edgesOnCell: np.ndarray
    cellsOnCell: np.ndarray
    verticesOnCell: np.ndarray
    cellsOnEdge: np.ndarray
    verticesOnEdge: np.ndarray
    edgesOnVertex: np.ndarray
    cellsOnVertex: np.ndarray
    kiteAreasOnVertex: np.ndarray
    areaCell: np.ndarray
    areaTriangle: np.ndarray
    dcEdge: np.ndarray
    dvEdge: np.ndarray
    fVertex: np.ndarray
    bottom: np.ndarray
    # positions: planar meshes use (x, y); spherical meshes (x, y, z) on the sphere
    xCell: np.ndarray
    yCell: np.ndarray
    xEdge: np.ndarray
    yEdge: np.ndarray
    xVertex: np.ndarray
    yVertex: np.ndarray
    # unit normal n_e at each edge point (planar: 2 components, sphere: 3)
    normalEdge: np.ndarray
    zCell: Optional[np.ndarray] = None
    zEdge: Optional[np.ndarray] = None
    zVertex: Optional[np.ndarray] = None
    Lx: float = 0.0
    Ly: float = 0.0
    radius: float = 0.0
    name: str = "mesh"

    @property
    def spherical(self) -> bool:
        return self.radius > 0.0

    def copy(self) -> "Mesh":
        kw = {}
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            kw[f.name] = v.copy() if isinstance(v, np.ndarray) else v
        return Mesh(**kw)

    # ------------------------------------------------------------------
    def check(self) -> None:
        """Raise ValueError when connectivity is inconsistent."""
        nC, nE, nV = self.nCells, self.nEdges, self.nVertices
        nEoC = self.nEdgesOnCell
        if nEoC.min() < 3 or nEoC.max() > self.maxEdges:
            raise ValueError("nEdgesOnCell out of range")
        for i in range(nC):
            n = int(nEoC[i])
            eoc = self.edgesOnCell[i, :n]
            if (eoc < 0).any() or (eoc >= nE).any():
                raise ValueError(f"cell {i}: bad edge index")
            for j in range(n):
                e = int(eoc[j])
                c0, c1 = self.cellsOnEdge[e]
                if i not in (c0, c1):
                    raise ValueError(f"cell {i}: edge {e} does not list it")
                other = c1 if c0 == i else c0
                if self.cellsOnCell[i, j] != other:
                    raise ValueError(f"cell {i}: cellsOnCell slot {j} mismatch")
                v = int(self.verticesOnCell[i, j])
                en = int(eoc[(j + 1) % n])
                if v not in self.verticesOnEdge[e] or v not in self.verticesOnEdge[en]:
                    raise ValueError(f"cell {i}: vertex slot {j} not shared by its edges")
        for v in range(nV):
            for k in range(3):
                e = int(self.edgesOnVertex[v, k])
                if v not in self.verticesOnEdge[e]:
                    raise ValueError(f"vertex {v}: edge {e} does not list it")
                c = int(self.cellsOnVertex[v, k])
                if v not in self.verticesOnCell[c, :nEoC[c]]:
                    raise ValueError(f"vertex {v}: cell {c} does not list it")
        if (self.kiteAreasOnVertex <= 0).any() or (self.areaCell <= 0).any():
            raise ValueError("non-positive areas")
        if (self.dcEdge <= 0).any() or (self.dvEdge <= 0).any():
            raise ValueError("non-positive lengths")
