"""Python handle on the FP64 C oracle (oracle.c).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The GPU library never does.

The shared object is compiled in place with gcc on first use (and again when
oracle.c or oracle.h is newer than it), with contraction of multiply-adds
turned off so every operation rounds as written.  A second build,
liboracle_omp.so (-O3 -march=native -fopenmp, contraction still off), splits
the per-element loops over host threads; it computes bitwise the same
results and serves only to time the oracle on all host cores
(Oracle(..., threads=n)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "oracle.h")]
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_FLAGS = {_LIB: ["-O2", "-Wno-unknown-pragmas"],
          _LIB_OMP: ["-O3", "-march=native", "-fopenmp"]}
_libs = {}


def build(force: bool = False, omp: bool = False) -> str:
    """Compile liboracle.so (or the threaded timing build liboracle_omp.so)
    next to its source; returns its path."""
    path = _LIB_OMP if omp else _LIB
    stale = (not os.path.exists(path)) or any(
        os.path.getmtime(s) > os.path.getmtime(path) for s in _SRC)
    if force or stale:
        tmp = path + f".tmp{os.getpid()}"
        cmd = ["gcc", *_FLAGS[path], "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-o", tmp, _SRC[0], "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return path


def _load(omp: bool = False):
    if omp in _libs:
        return _libs[omp]
    lib = ctypes.CDLL(build(omp=omp))
    P = ctypes.c_void_p
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
    u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    ci = ctypes.c_int
    cd = ctypes.c_double
    lib.om_create.restype = P
    lib.om_create.argtypes = [ci, ci, ci, ci] + [i32p] * 8 + [f64p] * 7 + [cd]
    lib.om_destroy.argtypes = [P]
    lib.om_n_edges_on_edge.argtypes = [P, ci]
    lib.om_n_edges_on_edge.restype = ci
    lib.om_weights_on_edge.argtypes = [P, ci, i32p, f64p]
    lib.om_weights_on_edge.restype = ci
    lib.om_rhs.argtypes = [P, f64p, f64p, f64p, f64p]
    lib.om_diag_fields.argtypes = [P, f64p, f64p, f64p, f64p, f64p, f64p]
    lib.om_regions.argtypes = [P, u8p, ci, ci, i8p, i8p, u8p, u8p]
    lib.om_regions.restype = ci
    lib.om_ssprk_step.argtypes = [P, ci, f64p, f64p, cd]
    lib.om_rk4_step.argtypes = [P, f64p, f64p, cd]
    lib.om_lts_step.argtypes = [P, ci, i8p, i8p, u8p, u8p, f64p, f64p, cd, ci]
    lib.om_lts_predict_coeffs.argtypes = [ci, ci, ci, ci, f64p]
    lib.om_mlts_regions.argtypes = [P, ci, u8p, ci, ci, i8p, i8p, u8p, u8p]
    lib.om_mlts_regions.restype = ci
    lib.om_mlts_step.argtypes = [P, ci, i8p, i8p, u8p, u8p, i32p, f64p, f64p, cd]
    lib.om_set_reading.argtypes = [ci]
    lib.om_get_reading.restype = ci
    lib.om_diagnostics.argtypes = [P, f64p, f64p, ctypes.POINTER(cd), ctypes.POINTER(cd)]
    lib.om_set_threads.argtypes = [ci]
    lib.om_get_threads.restype = ci
    _libs[omp] = lib
    return lib


C, I2, I1, F = 0, 1, 2, 3


@dataclass
class Regions:
    cell: np.ndarray       # int8 labels C=0, I2=1, I1=2, F=3
    edge: np.ndarray
    cell_fbar: np.ndarray  # uint8, underlined F (two fine rings nearest I1)
    edge_fbar: np.ndarray


class reading:
    """Context manager selecting a literal reading of a garbled passage
    (1: Step 3.3.3 with dt, 2: 2/3 x^{1st} in Steps 3.3.3/4, 3: clockwise
    weights).  Only for tests that show the pins reject those readings."""

    def __init__(self, r: int):
        self.r = r

    def __enter__(self):
        _load().om_set_reading(self.r)
        return self

    def __exit__(self, *exc):
        _load().om_set_reading(0)
        return False


def predict_coeffs(order: int, stage: int, k: int, M: int) -> np.ndarray:
    out = np.zeros(3)
    _load().om_lts_predict_coeffs(order, stage, k, M, out)
    return out


class Oracle:
    """FP64 reference for the TRiSK right-hand side and the time integrators."""

    def __init__(self, mesh, gravity: float = 9.81, threads: int | None = None):
        """threads: None for the single-threaded build; n > 0 for the threaded
        timing build with n threads (bitwise the same results)."""
        lib = _load(omp=threads is not None)
        if threads is not None:
            lib.om_set_threads(int(threads))
        self.threads = lib.om_get_threads()
        self.mesh = mesh
        self.gravity = float(gravity)
        m = mesh
        i32 = lambda a: np.ascontiguousarray(a, np.int32).reshape(-1)
        f64 = lambda a: np.ascontiguousarray(a, np.float64).reshape(-1)
        self._keep = [i32(m.nEdgesOnCell), i32(m.edgesOnCell), i32(m.cellsOnCell),
                      i32(m.verticesOnCell), i32(m.cellsOnEdge), i32(m.verticesOnEdge),
                      i32(m.edgesOnVertex), i32(m.cellsOnVertex),
                      f64(m.kiteAreasOnVertex), f64(m.areaCell), f64(m.areaTriangle),
                      f64(m.dcEdge), f64(m.dvEdge), f64(m.fVertex), f64(m.bottom)]
        self._h = lib.om_create(m.nCells, m.nEdges, m.nVertices, m.maxEdges,
                                *self._keep, self.gravity)
        if not self._h:
            raise MemoryError("om_create failed")
        self._lib = lib

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.om_destroy(self._h)
            self._h = None

    # -- operators -------------------------------------------------------
    def rhs(self, h, u):
        h = np.ascontiguousarray(h, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        dh = np.empty_like(h)
        du = np.empty_like(u)
        self._lib.om_rhs(self._h, h, u, dh, du)
        return dh, du

    def diag_fields(self, h, u):
        m = self.mesh
        h = np.ascontiguousarray(h, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        K = np.empty(m.nCells)
        q = np.empty(m.nVertices)
        z = np.empty(m.nVertices)
        fp = np.empty(m.nEdges)
        self._lib.om_diag_fields(self._h, h, u, K, q, z, fp)
        return K, q, z, fp

    def weights(self, e: int):
        n = self._lib.om_n_edges_on_edge(self._h, int(e))
        ee = np.empty(n, np.int32)
        w = np.empty(n)
        self._lib.om_weights_on_edge(self._h, int(e), ee, w)
        return ee, w

    def regions(self, fine_mask, n1: int = 2, n2: int = 2) -> Regions:
        m = self.mesh
        fm = np.ascontiguousarray(fine_mask, np.uint8)
        cr = np.empty(m.nCells, np.int8)
        er = np.empty(m.nEdges, np.int8)
        cf = np.empty(m.nCells, np.uint8)
        ef = np.empty(m.nEdges, np.uint8)
        rc = self._lib.om_regions(self._h, fm, int(n1), int(n2), cr, er, cf, ef)
        if rc != 0:
            raise ValueError("unusable LTS region labels")
        return Regions(cr, er, cf, ef)

    # -- integrators (copies in, copies out) -------------------------------
    def ssprk(self, h, u, dt: float, n: int = 1, order: int = 3):
        h = np.array(h, np.float64)
        u = np.array(u, np.float64)
        for _ in range(n):
            self._lib.om_ssprk_step(self._h, order, h, u, float(dt))
        return h, u

    def rk4(self, h, u, dt: float, n: int = 1):
        h = np.array(h, np.float64)
        u = np.array(u, np.float64)
        for _ in range(n):
            self._lib.om_rk4_step(self._h, h, u, float(dt))
        return h, u

    def lts(self, h, u, dt: float, M: int, regions: Regions, n: int = 1,
            order: int = 3):
        h = np.array(h, np.float64)
        u = np.array(u, np.float64)
        r = regions
        for _ in range(n):
            self._lib.om_lts_step(self._h, order, r.cell, r.edge, r.cell_fbar,
                                  r.edge_fbar, h, u, float(dt), int(M))
        return h, u

    def ml_regions(self, masks, n1: int = 2, n2: int = 2) -> Regions:
        """Labels of every level of a multi-level LTS3 (Remark 3.1): masks is
        a list of nested fine masks, outermost first; the Regions arrays hold
        one row per level.  Raises when a level is unusable or not nested at
        least three cell rings inside the previous one."""
        m = self.mesh
        fm = np.ascontiguousarray(np.stack([np.asarray(x, np.uint8) for x in masks]))
        nl = fm.shape[0]
        cr = np.empty((nl, m.nCells), np.int8)
        er = np.empty((nl, m.nEdges), np.int8)
        cf = np.empty((nl, m.nCells), np.uint8)
        ef = np.empty((nl, m.nEdges), np.uint8)
        rc = self._lib.om_mlts_regions(self._h, nl + 1, fm.reshape(-1), int(n1), int(n2),
                                       cr.reshape(-1), er.reshape(-1), cf.reshape(-1),
                                       ef.reshape(-1))
        if rc != 0:
            raise ValueError("unusable or insufficiently nested LTS levels")
        return Regions(cr, er, cf, ef)

    def mlts(self, h, u, dt: float, Ms, regions: Regions, n: int = 1):
        """n coarse steps of multi-level LTS3: Ms[l] is the step ratio of level
        l to level l+1 (len(Ms) = number of fine regions)."""
        h = np.array(h, np.float64)
        u = np.array(u, np.float64)
        r = regions
        Ma = np.ascontiguousarray(Ms, np.int32)
        assert r.cell.ndim == 2 and Ma.shape[0] == r.cell.shape[0]
        for _ in range(n):
            self._lib.om_mlts_step(self._h, Ma.shape[0] + 1, r.cell.reshape(-1),
                                   r.edge.reshape(-1), r.cell_fbar.reshape(-1),
                                   r.edge_fbar.reshape(-1), Ma, h, u, float(dt))
        return h, u

    def diagnostics(self, h, u):
        mass = ctypes.c_double()
        energy = ctypes.c_double()
        self._lib.om_diagnostics(self._h, np.ascontiguousarray(h, np.float64),
                                 np.ascontiguousarray(u, np.float64),
                                 ctypes.byref(mass), ctypes.byref(energy))
        return mass.value, energy.value
