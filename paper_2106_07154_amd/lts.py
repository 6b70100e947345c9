"""ctypes binding of liblts (include/lts.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts numpy
arrays and torch device tensors to pointers and status codes to exceptions.
Loading fails loudly when liblts.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblts.so")

LTS_OK, LTS_EINVAL, LTS_EMESH, LTS_ELABEL, LTS_ENONFINITE, LTS_EDEVICE, LTS_ESTATE, LTS_ENOMEM = \
    0, -1, -2, -3, -4, -5, -6, -7
LTS_FP64, LTS_FP32 = 0, 1
LTS_C, LTS_I2, LTS_I1, LTS_F = 0, 1, 2, 3
KERNEL_CLASSES = ["vertex_pv", "cell_tendency", "edge_tendency"]

EXPORTED = ["lts_create", "lts_set_layers", "lts_upload_mesh", "lts_upload_mesh_levels",
            "lts_get_level_regions", "lts_step_levels", "lts_plan_levels", "lts_get_regions", "lts_init_state",
            "lts_init_state_device", "lts_step", "lts_step_rk3", "lts_step_scheme", "lts_eval_rhs",
            "lts_diagnostics", "lts_get_state", "lts_get_state_device", "lts_set_timing",
            "lts_kernel_stats", "lts_region_counts", "lts_plan", "lts_last_error", "lts_destroy",
            "lts_ens_create", "lts_ens_add_member", "lts_ens_add_member_levels",
            "lts_ens_init_member", "lts_ens_build",
            "lts_ens_step", "lts_ens_set_scheme", "lts_ens_set_fused", "lts_ens_kernel_stats",
            "lts_ens_get_member",
            "lts_ens_diagnostics", "lts_ens_info",
            "lts_ens_last_error", "lts_ens_destroy",
            "lts_sur_create", "lts_sur_info", "lts_sur_node_map", "lts_sur_record",
            "lts_sur_normalize", "lts_sur_set_norm", "lts_sur_get_norm", "lts_sur_get_params",
            "lts_sur_set_params", "lts_sur_save", "lts_sur_load", "lts_sur_train",
            "lts_sur_grad", "lts_sur_features",
            "lts_sur_predict", "lts_sur_step", "lts_sur_last_error", "lts_sur_destroy",
            "lts_nn_gemm_bf16", "lts_nn_gemm_tn_bf16", "lts_nn_gemm_bf16_device",
            "lts_nn_gemm_tn_bf16_device_noalloc", "lts_nn_gemm_tn_noalloc_max_rows"]


class LTSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"liblts status {status}: {msg}")
        self.status = status


class _Mesh(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("n_vertices", ctypes.c_int32), ("max_edges", ctypes.c_int32)] + [
        (name, ctypes.c_void_p) for name in (
            "n_edges_on_cell", "edges_on_cell", "cells_on_cell", "vertices_on_cell",
            "cells_on_edge", "vertices_on_edge", "edges_on_vertex", "cells_on_vertex",
            "kite_areas_on_vertex", "area_cell", "area_triangle", "dc_edge", "dv_edge",
            "f_vertex", "bottom", "cell_xyz")] + [
        ("max_edges2", ctypes.c_int32), ("n_edges_on_edge", ctypes.c_void_p),
        ("edges_on_edge", ctypes.c_void_p), ("weights_on_edge", ctypes.c_void_p),
        ("edge_sign_on_cell", ctypes.c_void_p), ("edge_sign_on_vertex", ctypes.c_void_p)]


class _Diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("mass", ctypes.c_double),
                ("energy", ctypes.c_double), ("h_min", ctypes.c_double),
                ("h_max", ctypes.c_double), ("u_absmax", ctypes.c_double),
                ("n_nonfinite", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("gate_fallbacks", ctypes.c_int64)]


@dataclass
class Diag:
    t: float
    mass: float
    energy: float
    h_min: float
    h_max: float
    u_absmax: float
    n_nonfinite: int
    steps: int
    gate_fallbacks: int = 0


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblts.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"liblts.so not built at {path}; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    PP = ctypes.POINTER(ctypes.c_void_p)
    ci, cd = ctypes.c_int, ctypes.c_double
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "lts_create": ([PP, ci, ci, P], ci),
        "lts_set_layers": ([P, ci], ci),
        "lts_upload_mesh": ([P, ctypes.POINTER(_Mesh), P, ci, ci, cd], ci),
        "lts_get_regions": ([P, P, P, P, P], ci),
        "lts_upload_mesh_levels": ([P, ctypes.POINTER(_Mesh), ci, P, ci, ci, cd], ci),
        "lts_get_level_regions": ([P, ci, P, P, P, P], ci),
        "lts_step_levels": ([P, cd, P, ci], ci),
        "lts_init_state": ([P, P, P, cd], ci),
        "lts_init_state_device": ([P, P, P, cd], ci),
        "lts_step": ([P, cd, ci, ci], ci),
        "lts_step_rk3": ([P, cd, ci], ci),
        "lts_step_scheme": ([P, ci, cd, ci, ci], ci),
        "lts_eval_rhs": ([P, P, P, P, P], ci),
        "lts_diagnostics": ([P, ctypes.POINTER(_Diag)], ci),
        "lts_get_state": ([P, P, P], ci),
        "lts_get_state_device": ([P, P, P], ci),
        "lts_set_timing": ([P, ci], ci),
        "lts_kernel_stats": ([P, ci, i64p, dp, dp], ci),
        "lts_region_counts": ([P, i64p, i64p, i64p], ci),
        "lts_last_error": ([P], ctypes.c_char_p),
        "lts_destroy": ([P], None),
        "lts_ens_create": ([PP, ci, ci, P], ci),
        "lts_ens_add_member": ([P, ctypes.POINTER(_Mesh), P, ci, ci, cd, cd, ci,
                               ctypes.POINTER(ctypes.c_int)], ci),
        "lts_ens_add_member_levels": ([P, ctypes.POINTER(_Mesh), ci, P, ci, ci, cd, cd, P,
                                      ctypes.POINTER(ctypes.c_int)], ci),
        "lts_ens_init_member": ([P, ci, P, P], ci),
        "lts_ens_build": ([P, ci], ci),
        "lts_ens_step": ([P, ci], ci),
        "lts_ens_set_scheme": ([P, ci, P], ci),
        "lts_ens_set_fused": ([P, ci, ci], ci),
        "lts_ens_kernel_stats": ([P, ci, P, P, P], ci),
        "lts_ens_get_member": ([P, ci, P, P], ci),
        "lts_ens_diagnostics": ([P, ci, ctypes.POINTER(_Diag)], ci),
        "lts_ens_info": ([P, P, P, P, P, P], ci),
        "lts_ens_last_error": ([P], ctypes.c_char_p),
        "lts_ens_destroy": ([P], None),
        "lts_sur_create": ([PP, P, ci, ci, ctypes.c_uint64, ci], ci),
        "lts_sur_info": ([P, P, P, P, P, P], ci),
        "lts_sur_node_map": ([P, P, P], ci),
        "lts_sur_record": ([P, cd, ci, ci], ci),
        "lts_sur_normalize": ([P, ci], ci),
        "lts_sur_set_norm": ([P, P], ci),
        "lts_sur_get_norm": ([P, P], ci),
        "lts_sur_get_params": ([P, P], ci),
        "lts_sur_set_params": ([P, P], ci),
        "lts_sur_save": ([P, ctypes.c_char_p], ci),
        "lts_sur_load": ([P, ctypes.c_char_p], ci),
        "lts_sur_train": ([P, P, ci, ctypes.c_float, P], ci),
        "lts_sur_grad": ([P, ci, P, P], ci),
        "lts_sur_features": ([P, P], ci),
        "lts_sur_predict": ([P, P, P], ci),
        "lts_sur_step": ([P, cd, ci, ci, cd, ci, P, P], ci),
        "lts_sur_last_error": ([P], ctypes.c_char_p),
        "lts_sur_destroy": ([P], None),
        "lts_nn_gemm_bf16": ([ci, P, ci, ci, P, P, P], ci),
        "lts_nn_gemm_tn_bf16": ([ci, P, ci, ci, P, P], ci),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class LTSContext:
    """One liblts context: a mesh, its LTS regions and a state on one GPU."""

    def __init__(self, device: int = 0, precision: str = "fp64", stream=None, layers: int = 1):
        self._lib = load_library()
        self.precision = precision
        self.layers = int(layers)
        prec = {"fp64": LTS_FP64, "fp32": LTS_FP32}[precision]
        if stream is not None and not isinstance(stream, int):
            stream = stream.cuda_stream  # a torch.cuda.Stream
        if stream == 0:
            raise ValueError("pass a non-default stream (handle 0 is the legacy null stream); "
                             "None makes the context create its own")
        h = ctypes.c_void_p()
        st = self._lib.lts_create(ctypes.byref(h), int(device), prec,
                                  ctypes.c_void_p(stream) if stream else None)
        if st != LTS_OK:
            raise LTSError(st, "lts_create failed")
        self._h = h
        self._keep = []
        self.mesh = None
        if self.layers != 1:
            self._check(self._lib.lts_set_layers(self._h, self.layers))

    def _check(self, st: int):
        if st != LTS_OK:
            msg = self._lib.lts_last_error(self._h)
            raise LTSError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lts_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # ---------------------------------------------------------------- mesh
    def upload_mesh(self, mesh, fine_mask, n_if1: int = 2, n_if2: int = 2,
                    gravity: float = 9.81, use_positions: bool = True, edge_weights=None,
                    edge_signs=None):
        m, keep = _mesh_struct(mesh, use_positions, edge_weights, edge_signs)
        fm = np.ascontiguousarray(fine_mask, np.uint8)
        self._check(self._lib.lts_upload_mesh(self._h, ctypes.byref(m), _ptr(fm), int(n_if1),
                                              int(n_if2), float(gravity)))
        self.mesh = mesh

    def upload_mesh_levels(self, mesh, fine_masks, n_if1: int = 2, n_if2: int = 2,
                           gravity: float = 9.81, use_positions: bool = True):
        """Multi-level LTS3 mesh: fine_masks is a list of nested fine masks,
        outermost first (Remark 3.1)."""
        m, keep = _mesh_struct(mesh, use_positions)
        fm = np.ascontiguousarray(np.stack([np.asarray(x, np.uint8) for x in fine_masks]))
        self._check(self._lib.lts_upload_mesh_levels(self._h, ctypes.byref(m), fm.shape[0],
                                                     _ptr(fm), int(n_if1), int(n_if2),
                                                     float(gravity)))
        self.mesh = mesh
        self.n_fine_levels = fm.shape[0]

    def level_regions(self, level: int):
        m = self.mesh
        cr = np.empty(m.nCells, np.int8)
        er = np.empty(m.nEdges, np.int8)
        cf = np.empty(m.nCells, np.uint8)
        ef = np.empty(m.nEdges, np.uint8)
        self._check(self._lib.lts_get_level_regions(self._h, int(level), _ptr(cr), _ptr(er),
                                                    _ptr(cf), _ptr(ef)))
        return cr, er, cf, ef

    def regions(self):
        m = self.mesh
        cr = np.empty(m.nCells, np.int8)
        er = np.empty(m.nEdges, np.int8)
        cf = np.empty(m.nCells, np.uint8)
        ef = np.empty(m.nEdges, np.uint8)
        self._check(self._lib.lts_get_regions(self._h, _ptr(cr), _ptr(er), _ptr(cf), _ptr(ef)))
        return cr, er, cf, ef

    def region_counts(self):
        c = np.zeros(4, np.int64)
        e = np.zeros(4, np.int64)
        f = np.zeros(2, np.int64)
        P = ctypes.POINTER(ctypes.c_int64)
        self._check(self._lib.lts_region_counts(self._h, c.ctypes.data_as(P),
                                                e.ctypes.data_as(P), f.ctypes.data_as(P)))
        return c, e, f

    # ---------------------------------------------------------------- state
    def init_state(self, h, u, t0: float = 0.0):
        h = np.ascontiguousarray(h, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        self._check(self._lib.lts_init_state(self._h, _ptr(h), _ptr(u), float(t0)))

    def init_state_device(self, h_tensor, u_tensor, t0: float = 0.0):
        self._check(self._lib.lts_init_state_device(self._h, h_tensor.data_ptr(),
                                                    u_tensor.data_ptr(), float(t0)))

    def get_state(self):
        """(h, u); with several layers, arrays of shape (layers, n)."""
        L = self.layers
        h = np.empty(self.mesh.nCells * L)
        u = np.empty(self.mesh.nEdges * L)
        self._check(self._lib.lts_get_state(self._h, _ptr(h), _ptr(u)))
        if L > 1:
            return h.reshape(L, -1), u.reshape(L, -1)
        return h, u

    def get_state_device(self, h_tensor, u_tensor):
        self._check(self._lib.lts_get_state_device(self._h, h_tensor.data_ptr(),
                                                   u_tensor.data_ptr()))

    # ---------------------------------------------------------------- stepping
    def step(self, dt_coarse: float, M: int, n_steps: int = 1):
        self._check(self._lib.lts_step(self._h, float(dt_coarse), int(M), int(n_steps)))

    def step_levels(self, dt_coarse: float, Ms, n_steps: int = 1):
        """Multi-level LTS3: Ms[l] is the step ratio of level l to level l+1."""
        Ma = np.ascontiguousarray(Ms, np.int32)
        self._check(self._lib.lts_step_levels(self._h, float(dt_coarse), _ptr(Ma),
                                              int(n_steps)))

    def step_rk3(self, dt: float, n_steps: int = 1):
        self._check(self._lib.lts_step_rk3(self._h, float(dt), int(n_steps)))

    SCHEMES = {"lts3": 0, "lts2": 1, "ssprk3": 2, "ssprk2": 3, "rk4": 4}

    def step_scheme(self, scheme: str, dt: float, M: int = 1, n_steps: int = 1):
        self._check(self._lib.lts_step_scheme(self._h, self.SCHEMES[scheme], float(dt), int(M),
                                              int(n_steps)))

    def eval_rhs(self, h, u):
        h = np.ascontiguousarray(h, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        dh = np.empty_like(h)
        du = np.empty_like(u)
        self._check(self._lib.lts_eval_rhs(self._h, _ptr(h), _ptr(u), _ptr(dh), _ptr(du)))
        return dh, du

    def diagnostics(self) -> Diag:
        d = _Diag()
        self._check(self._lib.lts_diagnostics(self._h, ctypes.byref(d)))
        return Diag(d.t, d.mass, d.energy, d.h_min, d.h_max, d.u_absmax, d.n_nonfinite, d.steps,
                    d.gate_fallbacks)

    def diagnostics_status(self):
        d = _Diag()
        st = self._lib.lts_diagnostics(self._h, ctypes.byref(d))
        return st, Diag(d.t, d.mass, d.energy, d.h_min, d.h_max, d.u_absmax, d.n_nonfinite,
                        d.steps, d.gate_fallbacks)

    # ---------------------------------------------------------------- timing
    def set_timing(self, enable: bool):
        self._check(self._lib.lts_set_timing(self._h, 1 if enable else 0))

    def kernel_stats(self):
        n = len(KERNEL_CLASSES)
        la = np.zeros(n, np.int64)
        ms = np.zeros(n)
        by = np.zeros(n)
        k = self._lib.lts_kernel_stats(self._h, n, la.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       by.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return {KERNEL_CLASSES[i]: dict(launches=int(la[i]), ms=float(ms[i]), bytes=float(by[i]))
                for i in range(k)}


def _mesh_struct(mesh, use_positions=True, edge_weights=None, edge_signs=None):
    """ctypes lts_mesh of a mesh object (MPAS field names).  edge_weights:
    optional (n_edges_on_edge [nE], edges_on_edge [nE][maxE2],
    weights_on_edge [nE][maxE2]) tables for the library to check;
    edge_signs: optional (edge_sign_on_cell [nC][maxE] or None,
    edge_sign_on_vertex [nV][3] or None), int8, checked likewise."""
    i32 = lambda a: np.ascontiguousarray(a, np.int32)
    f64 = lambda a: np.ascontiguousarray(a, np.float64)
    arrs = dict(
        n_edges_on_cell=i32(mesh.nEdgesOnCell), edges_on_cell=i32(mesh.edgesOnCell),
        cells_on_cell=i32(mesh.cellsOnCell), vertices_on_cell=i32(mesh.verticesOnCell),
        cells_on_edge=i32(mesh.cellsOnEdge), vertices_on_edge=i32(mesh.verticesOnEdge),
        edges_on_vertex=i32(mesh.edgesOnVertex), cells_on_vertex=i32(mesh.cellsOnVertex),
        kite_areas_on_vertex=f64(mesh.kiteAreasOnVertex), area_cell=f64(mesh.areaCell),
        area_triangle=f64(mesh.areaTriangle), dc_edge=f64(mesh.dcEdge),
        dv_edge=f64(mesh.dvEdge), f_vertex=f64(mesh.fVertex), bottom=f64(mesh.bottom))
    if use_positions:
        z = mesh.zCell if getattr(mesh, "zCell", None) is not None else np.zeros(mesh.nCells)
        arrs["cell_xyz"] = f64(np.stack([mesh.xCell, mesh.yCell, z], 1))
    m = _Mesh(mesh.nCells, mesh.nEdges, mesh.nVertices, mesh.maxEdges)
    if edge_weights is not None:
        ne, ee, we = edge_weights
        ee, we = i32(ee), f64(we)
        assert ee.ndim == 2 and ee.shape == we.shape and ee.shape[0] == mesh.nEdges
        arrs.update(n_edges_on_edge=i32(ne), edges_on_edge=ee, weights_on_edge=we)
        m.max_edges2 = ee.shape[1]
    if edge_signs is not None:
        sc, sv = edge_signs
        if sc is not None:
            sc = np.ascontiguousarray(sc, np.int8)
            assert sc.shape == (mesh.nCells, mesh.maxEdges)
            arrs["edge_sign_on_cell"] = sc
        if sv is not None:
            sv = np.ascontiguousarray(sv, np.int8)
            assert sv.shape == (mesh.nVertices, 3)
            arrs["edge_sign_on_vertex"] = sv
    for k, v in arrs.items():
        setattr(m, k, _ptr(v))
    return m, arrs


PASS_NAMES = ["full", "step1", "step2", "step3", "step4"]


def plan(mesh, fine_mask, n_if1: int = 2, n_if2: int = 2, use_positions: bool = True,
         edge_weights=None, edge_signs=None):
    """Host-only lts_plan: labels, device ordering and pass ranges (no GPU)."""
    lib = load_library()
    if not hasattr(lib, "_plan_typed"):
        P = ctypes.c_void_p
        lib.lts_plan.argtypes = [ctypes.POINTER(_Mesh), P, ctypes.c_int, ctypes.c_int] + [P] * 8 + \
            [ctypes.c_char_p, ctypes.c_int]
        lib.lts_plan.restype = ctypes.c_int
        lib._plan_typed = True
    m, keep = _mesh_struct(mesh, use_positions, edge_weights, edge_signs)
    fm = np.ascontiguousarray(fine_mask, np.uint8)
    out = dict(cell_region=np.empty(mesh.nCells, np.int8), edge_region=np.empty(mesh.nEdges, np.int8),
               cell_fbar=np.empty(mesh.nCells, np.uint8), edge_fbar=np.empty(mesh.nEdges, np.uint8),
               cell_order=np.empty(mesh.nCells, np.int32), edge_order=np.empty(mesh.nEdges, np.int32),
               vertex_order=np.empty(mesh.nVertices, np.int32), ranges=np.empty(54, np.int32))
    err = ctypes.create_string_buffer(512)
    st = lib.lts_plan(ctypes.byref(m), _ptr(fm), int(n_if1), int(n_if2),
                      *[_ptr(out[k]) for k in ("cell_region", "edge_region", "cell_fbar",
                                              "edge_fbar", "cell_order", "edge_order",
                                              "vertex_order", "ranges")],
                      err, len(err))
    if st != LTS_OK:
        raise LTSError(st, err.value.decode())
    r = out.pop("ranges")
    out["cell_class_start"] = r[:8].copy()
    out["edge_class_start"] = r[8:14].copy()
    out["passes"] = {name: dict(zip(["c_lo", "c_hi", "v_lo", "v_hi", "ct_lo", "ct_hi",
                                     "et_lo", "et_hi"], r[14 + 8 * k: 22 + 8 * k].tolist()))
                     for k, name in enumerate(PASS_NAMES)}
    return out


def plan_levels(mesh, fine_masks, n_if1: int = 2, n_if2: int = 2, use_positions: bool = True):
    """Host-only lts_plan_levels: device ordering and per-level class starts and
    pass ranges of a multi-level mesh (no GPU)."""
    lib = load_library()
    if not hasattr(lib, "_plan_levels_typed"):
        P = ctypes.c_void_p
        lib.lts_plan_levels.argtypes = [ctypes.POINTER(_Mesh), ctypes.c_int, P, ctypes.c_int,
                                        ctypes.c_int] + [P] * 4 + [ctypes.c_char_p, ctypes.c_int]
        lib.lts_plan_levels.restype = ctypes.c_int
        lib._plan_levels_typed = True
    m, keep = _mesh_struct(mesh, use_positions)
    fm = np.ascontiguousarray(np.stack([np.asarray(x, np.uint8) for x in fine_masks]))
    nl = fm.shape[0]
    out = dict(cell_order=np.empty(mesh.nCells, np.int32), edge_order=np.empty(mesh.nEdges, np.int32),
               vertex_order=np.empty(mesh.nVertices, np.int32), ranges=np.empty(46 * nl, np.int32))
    err = ctypes.create_string_buffer(512)
    st = lib.lts_plan_levels(ctypes.byref(m), nl, _ptr(fm), int(n_if1), int(n_if2),
                             *[_ptr(out[k]) for k in ("cell_order", "edge_order", "vertex_order",
                                                      "ranges")], err, len(err))
    if st != LTS_OK:
        raise LTSError(st, err.value.decode())
    r = out.pop("ranges").reshape(nl, 46)
    keys = ["c_lo", "c_hi", "v_lo", "v_hi", "ct_lo", "ct_hi", "et_lo", "et_hi"]
    out["levels"] = [dict(cell_class_start=r[l, :8].copy(), edge_class_start=r[l, 8:14].copy(),
                          passes={name: dict(zip(keys, r[l, 14 + 8 * k: 22 + 8 * k].tolist()))
                                  for k, name in enumerate(["step1", "step2", "step3", "step4"])})
                     for l in range(nl)]
    return out


class Ensemble:
    """Many LTS3 members of uneven size advanced together (lts_ens_* ABI)."""

    def __init__(self, device: int = 0, precision: str = "fp32", stream=None):
        self._lib = load_library()
        if stream is not None and not isinstance(stream, int):
            stream = stream.cuda_stream
        if stream == 0:
            raise ValueError("pass a non-default stream")
        h = ctypes.c_void_p()
        st = self._lib.lts_ens_create(ctypes.byref(h), int(device),
                                      {"fp64": LTS_FP64, "fp32": LTS_FP32}[precision],
                                      ctypes.c_void_p(stream) if stream else None)
        if st != LTS_OK:
            raise LTSError(st, "lts_ens_create failed")
        self._h = h
        self.meshes = []

    def _check(self, st):
        if st != LTS_OK:
            msg = self._lib.lts_ens_last_error(self._h)
            raise LTSError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lts_ens_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def add_member(self, mesh, fine_mask, dt_coarse, M, n_if1=2, n_if2=2, gravity=9.81,
                   use_positions=True) -> int:
        m, keep = _mesh_struct(mesh, use_positions)
        fm = np.ascontiguousarray(fine_mask, np.uint8)
        idx = ctypes.c_int()
        self._check(self._lib.lts_ens_add_member(self._h, ctypes.byref(m), _ptr(fm), int(n_if1),
                                                 int(n_if2), float(gravity), float(dt_coarse),
                                                 int(M), ctypes.byref(idx)))
        self.meshes.append(mesh)
        return idx.value

    def add_member_levels(self, mesh, fine_masks, dt_coarse, Ms, n_if1=2, n_if2=2,
                          gravity=9.81, use_positions=True) -> int:
        """Multi-level member: nested fine masks, outermost first, and the
        step ratio Ms[l] of level l to level l+1 (Remark 3.1)."""
        m, keep = _mesh_struct(mesh, use_positions)
        fm = np.ascontiguousarray(np.stack([np.asarray(x, np.uint8) for x in fine_masks]))
        Ma = np.ascontiguousarray(Ms, np.int32)
        if Ma.shape != (fm.shape[0],):
            raise ValueError("one ratio per fine level")
        idx = ctypes.c_int()
        self._check(self._lib.lts_ens_add_member_levels(self._h, ctypes.byref(m), fm.shape[0],
                                                        _ptr(fm), int(n_if1), int(n_if2),
                                                        float(gravity), float(dt_coarse),
                                                        _ptr(Ma), ctypes.byref(idx)))
        self.meshes.append(mesh)
        return idx.value

    def init_member(self, j, h, u):
        h = np.ascontiguousarray(h, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        self._check(self._lib.lts_ens_init_member(self._h, int(j), _ptr(h), _ptr(u)))

    def build(self, autotune: bool = True):
        self._check(self._lib.lts_ens_build(self._h, 1 if autotune else 0))

    def step(self, n_steps: int = 1):
        self._check(self._lib.lts_ens_step(self._h, int(n_steps)))

    def get_member(self, j):
        m = self.meshes[j]
        h = np.empty(m.nCells)
        u = np.empty(m.nEdges)
        self._check(self._lib.lts_ens_get_member(self._h, int(j), _ptr(h), _ptr(u)))
        return h, u

    def diagnostics(self, j) -> Diag:
        d = _Diag()
        self._check(self._lib.lts_ens_diagnostics(self._h, int(j), ctypes.byref(d)))
        return Diag(d.t, d.mass, d.energy, d.h_min, d.h_max, d.u_absmax, d.n_nonfinite, d.steps,
                    d.gate_fallbacks)

    def set_scheme(self, scheme: str, dt_coarse=None):
        """'lts3' or 'ssprk3' (M_j SSPRK3 steps of dt_j/M_j per ensemble step);
        optional new coarse steps per member.  Rebuild afterwards."""
        code = {"lts3": 0, "ssprk3": 2}[scheme]
        d = None if dt_coarse is None else np.ascontiguousarray(dt_coarse, np.float64)
        self._check(self._lib.lts_ens_set_scheme(self._h, code, None if d is None else _ptr(d)))

    def set_fused(self, enable: bool = True, spin_limit: int = 0):
        """One persistent fused kernel per ensemble step (rebuild afterwards);
        spin_limit bounds every grid-barrier wait (0: the default)."""
        self._check(self._lib.lts_ens_set_fused(self._h, int(bool(enable)), int(spin_limit)))

    def kernel_stats(self, n_steps: int):
        """Event-stamped per-class statistics of n_steps ensemble steps (the
        members advance)."""
        n = np.zeros(3, np.int64)
        ms = np.zeros(3)
        by = np.zeros(3)
        self._check(self._lib.lts_ens_kernel_stats(self._h, int(n_steps), _ptr(n), _ptr(ms),
                                                   _ptr(by)))
        names = ["vertex_pv", "cell_tendency", "edge_tendency"]
        return {names[k]: {"launches": int(n[k]), "ms": float(ms[k]), "bytes": float(by[k])}
                for k in range(3)}

    def info(self):
        tuned = np.zeros(18, np.int32)
        us = np.zeros(9)
        cells = np.zeros(3, np.int64)
        nl = np.zeros(1, np.int32)
        by = np.zeros(3)
        self._check(self._lib.lts_ens_info(self._h, _ptr(tuned), _ptr(us), _ptr(cells), _ptr(nl),
                                           _ptr(by)))
        names = ["vertex_pv", "cell_tendency", "edge_tendency"]
        classes = ["small", "medium", "large"]
        tune = {f"{names[k]}/{classes[s]}": {"block": int(tuned[(k * 3 + s) * 2]),
                                             "grid_factor": int(tuned[(k * 3 + s) * 2 + 1]),
                                             "us": round(float(us[k * 3 + s]), 2)}
                for k in range(3) for s in range(3) if cells[s] > 0}
        return {"tuning": tune, "class_cells": cells.tolist(), "launches_per_step": int(nl[0]),
                "step_bytes": {names[k]: float(by[k]) for k in range(3)}}


# ---------------------------------------------------------------------------
# Learned fine-region surrogate (include/lts_surrogate.h)

N_FEATURES = 16


class Surrogate:
    """A message-passing surrogate attached to an LTSContext (mesh and state
    set).  Arrays are numpy; node order is the library's (see node_map)."""

    def __init__(self, ctx: LTSContext, seed: int = 0, max_samples: int = 0, n_layers: int = 3,
                 hidden: int = 64):
        self._lib = load_library()
        self.ctx = ctx
        h = ctypes.c_void_p()
        st = self._lib.lts_sur_create(ctypes.byref(h), ctx._h, int(n_layers), int(hidden),
                                      ctypes.c_uint64(seed), int(max_samples))
        if st != LTS_OK:
            msg = self._lib.lts_last_error(ctx._h)
            raise LTSError(st, msg.decode() if msg else "")
        self._h = h
        v = np.zeros(5, np.int32)
        self._check(self._lib.lts_sur_info(self._h, *[_ptr(v[i:i + 1]) for i in range(5)]))
        self.n_nodes, self.n_fine_cells, self.n_fine_edges, self.n_params = (int(x) for x in v[:4])

    def _check(self, st):
        if st != LTS_OK:
            msg = self._lib.lts_sur_last_error(self._h)
            raise LTSError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lts_sur_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def n_samples(self) -> int:
        v = np.zeros(1, np.int32)
        self._check(self._lib.lts_sur_info(self._h, None, None, None, None, _ptr(v)))
        return int(v[0])

    def node_map(self):
        nc = np.empty(self.n_nodes, np.int32)
        fe = np.empty(self.n_fine_edges, np.int32)
        self._check(self._lib.lts_sur_node_map(self._h, _ptr(nc), _ptr(fe)))
        return nc, fe

    def record(self, dt: float, M: int, n_steps: int):
        self._check(self._lib.lts_sur_record(self._h, float(dt), int(M), int(n_steps)))

    def normalize(self, n_samples: int | None = None):
        n = self.n_samples if n_samples is None else n_samples
        self._check(self._lib.lts_sur_normalize(self._h, int(n)))

    def set_norm(self, norm):
        a = np.ascontiguousarray(norm, np.float32)
        assert a.size == 16
        self._check(self._lib.lts_sur_set_norm(self._h, _ptr(a)))

    def get_norm(self):
        a = np.empty(16, np.float32)
        self._check(self._lib.lts_sur_get_norm(self._h, _ptr(a)))
        return a

    def get_params(self):
        a = np.empty(self.n_params, np.float32)
        self._check(self._lib.lts_sur_get_params(self._h, _ptr(a)))
        return a

    def set_params(self, p):
        a = np.ascontiguousarray(p, np.float32)
        assert a.size == self.n_params
        self._check(self._lib.lts_sur_set_params(self._h, _ptr(a)))

    def save(self, path):
        """Shape, normalisation vector and parameters to a file (lts_sur_save)."""
        self._check(self._lib.lts_sur_save(self._h, os.fsencode(path)))

    def load(self, path):
        """Parameters (and the normalisation vector) from a file written by
        save; the Adam state restarts."""
        self._check(self._lib.lts_sur_load(self._h, os.fsencode(path)))

    def train(self, idx, lr: float = 1e-3):
        idx = np.ascontiguousarray(idx, np.int32)
        losses = np.empty(idx.size, np.float32)
        self._check(self._lib.lts_sur_train(self._h, _ptr(idx), int(idx.size), ctypes.c_float(lr),
                                            _ptr(losses)))
        return losses

    def grad(self, k: int):
        loss = np.empty(1, np.float32)
        g = np.empty(self.n_params, np.float32)
        self._check(self._lib.lts_sur_grad(self._h, int(k), _ptr(loss), _ptr(g)))
        return float(loss[0]), g

    def features(self):
        a = np.empty((self.n_nodes, N_FEATURES), np.float32)
        self._check(self._lib.lts_sur_features(self._h, _ptr(a)))
        return a

    def predict(self):
        oh = np.empty(self.n_fine_cells, np.float32)
        ou = np.empty(self.n_fine_edges, np.float32)
        self._check(self._lib.lts_sur_predict(self._h, _ptr(oh), _ptr(ou)))
        return oh, ou

    def step(self, dt: float, M: int, n_steps: int = 1, tau: float = 0.0, max_backoff: int = 0):
        acc = np.zeros(1, np.int32)
        res = np.empty(max(n_steps, 1))
        self._check(self._lib.lts_sur_step(self._h, float(dt), int(M), int(n_steps), float(tau),
                                           int(max_backoff), _ptr(acc), _ptr(res)))
        return int(acc[0]), res[:n_steps]


def nn_gemm_bf16(A_bits, W_bits, bias=None, device: int = 0):
    """Y = A W (+ bias) on the matrix cores; A [N x K], W [K x 64] as BF16 bit
    patterns (uint16); returns FP32 [N x 64]."""
    lib = load_library()
    A = np.ascontiguousarray(A_bits, np.uint16)
    W = np.ascontiguousarray(W_bits, np.uint16)
    N, K = A.shape
    assert W.shape == (K, 64)
    Y = np.empty((N, 64), np.float32)
    b = None if bias is None else np.ascontiguousarray(bias, np.float32)
    st = lib.lts_nn_gemm_bf16(int(device), _ptr(A), N, K, _ptr(W), None if b is None else _ptr(b),
                              _ptr(Y))
    if st != LTS_OK:
        raise LTSError(st, "lts_nn_gemm_bf16")
    return Y


def nn_gemm_bf16_device(A, W, Y_f32=None, Y_bf16=None, bias=None, stream=None):
    """The forward product on torch device tensors (no copies, no sync):
    A [N x K] and W [K x 64] int16/uint16 BF16 bit patterns, optional FP32
    bias [64]; fills Y_f32 [N x 64] float32 and/or Y_bf16 [N x 64] (relu,
    BF16 bits) on `stream` (a torch stream or raw handle; None: null stream)."""
    lib = load_library()
    if not hasattr(lib, "_gemm_dev_typed"):
        P = ctypes.c_void_p
        lib.lts_nn_gemm_bf16_device.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, P, P, P]
        lib.lts_nn_gemm_bf16_device.restype = ctypes.c_int
        lib._gemm_dev_typed = True
    N, K = A.shape
    assert tuple(W.shape) == (K, 64) and A.is_contiguous() and W.is_contiguous()
    assert A.element_size() == 2 and W.element_size() == 2
    for Y, size in ((Y_f32, 4), (Y_bf16, 2)):
        assert Y is None or (tuple(Y.shape) == (N, 64) and Y.is_contiguous()
                             and Y.element_size() == size)
    sp = getattr(stream, "cuda_stream", stream)
    dp = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    st = lib.lts_nn_gemm_bf16_device(dp(A), N, K, dp(W), dp(bias), dp(Y_f32), dp(Y_bf16),
                                     None if sp is None else ctypes.c_void_p(sp))
    if st != LTS_OK:
        raise LTSError(st, "lts_nn_gemm_bf16_device")


def nn_gemm_tn_bf16(A_bits, D_bits, device: int = 0):
    """P = A^T D on the matrix cores; A [N x K], D [N x 64] BF16 bit patterns."""
    lib = load_library()
    A = np.ascontiguousarray(A_bits, np.uint16)
    D = np.ascontiguousarray(D_bits, np.uint16)
    N, K = A.shape
    assert D.shape == (N, 64)
    P = np.empty((K, 64), np.float32)
    st = lib.lts_nn_gemm_tn_bf16(int(device), _ptr(A), N, K, _ptr(D), _ptr(P))
    if st != LTS_OK:
        raise LTSError(st, "lts_nn_gemm_tn_bf16")
    return P


def nn_gemm_tn_noalloc_max_rows(K: int) -> int:
    """Largest N the allocation-free weight-gradient product accepts at K."""
    lib = load_library()
    lib.lts_nn_gemm_tn_noalloc_max_rows.argtypes = [ctypes.c_int]
    lib.lts_nn_gemm_tn_noalloc_max_rows.restype = ctypes.c_longlong
    return int(lib.lts_nn_gemm_tn_noalloc_max_rows(int(K)))


def nn_gemm_tn_bf16_device_noalloc(A, D, P, stream=None):
    """P = A^T D on torch device tensors through the entry point that
    allocates nothing: A [N x K] and D [N x 64] int16/uint16 BF16 bit
    patterns, P [K x 64] float32, on `stream` (torch stream or raw handle;
    None: the null stream).  No copies, no synchronisation."""
    lib = load_library()
    if not hasattr(lib, "_gemm_tn_noalloc_typed"):
        Pv = ctypes.c_void_p
        lib.lts_nn_gemm_tn_bf16_device_noalloc.argtypes = [Pv, ctypes.c_int, ctypes.c_int, Pv,
                                                           Pv, Pv]
        lib.lts_nn_gemm_tn_bf16_device_noalloc.restype = ctypes.c_int
        lib._gemm_tn_noalloc_typed = True
    N, K = A.shape
    assert tuple(D.shape) == (N, 64) and tuple(P.shape) == (K, 64)
    assert A.is_contiguous() and D.is_contiguous() and P.is_contiguous()
    assert A.element_size() == 2 and D.element_size() == 2 and P.element_size() == 4
    sp = getattr(stream, "cuda_stream", stream)
    st = lib.lts_nn_gemm_tn_bf16_device_noalloc(
        ctypes.c_void_p(A.data_ptr()) if N else None, N, K,
        ctypes.c_void_p(D.data_ptr()) if N else None, ctypes.c_void_p(P.data_ptr()),
        None if sp is None else ctypes.c_void_p(sp))
    if st != LTS_OK:
        raise LTSError(st, "lts_nn_gemm_tn_bf16_device_noalloc")
