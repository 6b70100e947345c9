"""GPU parity on spherical variable-resolution Voronoi meshes: a small
10,000-cell cap mesh (every scheme against the FP64 oracle) and the full
1.6M-cell workload bench.py times with --workload sphere (FP64 and FP32 LTS3
against the oracle's coarse steps).  Tolerances as in the planar parity tests:
1e-12 relative L2 on h in FP64 (1e-11 on u, whose tendency is a difference of
g(h + b) terms), 1e-5 on total h and u in FP32."""
import math
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2106_07154_amd import lts
from paper_2106_07154_amd.inputs import workloads

pytestmark = pytest.mark.gpu

# FP32 LTS3 on the 1.6M-cell sphere against the FP64 oracle after 2 coarse
# steps, per field: measured values times about 4 (stated in the design doc's
# tolerance section)
FP32_SPHERE_ETA_TOL = 1e-5
FP32_SPHERE_MASS_TOL = 1e-8
FP32_SPHERE_ENERGY_TOL = 1e-6


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b, w=None):
    w = np.ones_like(b) if w is None else w
    return math.sqrt((w * (a - b) ** 2).sum() / max((w * b ** 2).sum(), 1e-300))


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ctx(w, prec):
    c = lts.LTSContext(0, prec)
    c.upload_mesh(w.mesh, w.fine_mask, w.n_if1, w.n_if2, w.gravity)
    return c


@pytest.fixture(scope="module")
def small():
    w = workloads.sphere_cap(n=10_000, iters=25)
    o = Oracle(w.mesh, w.gravity)
    R = o.regions(w.fine_mask, w.n_if1, w.n_if2)
    return w, o, R


def test_small_sphere_lts3_fp64(small):
    w, o, R = small
    m = w.mesh
    say("sphere10k lts3 fp64", m.nCells, "cells, maxE", m.maxEdges)
    c = _ctx(w, "fp64")
    c.init_state(w.h0, w.u0)
    c.step(w.dt_coarse, w.M, 6)
    gh, gu = c.get_state()
    rh, ru = o.lts(w.h0, w.u0, w.dt_coarse, w.M, R, n=6)
    assert rel_l2(gh, rh, m.areaCell) < 1e-12
    assert rel_l2(gu, ru, m.dvEdge * m.dcEdge) < 1e-11
    d = c.diagnostics()
    m0, _ = o.diagnostics(w.h0, w.u0)
    assert abs(d.mass - m0) <= 1e-13 * m0
    c.close()


@pytest.mark.parametrize("scheme", ["ssprk3", "rk4", "lts2"])
def test_small_sphere_schemes_fp64(small, scheme):
    w, o, R = small
    say("sphere10k", scheme)
    c = _ctx(w, "fp64")
    c.init_state(w.h0, w.u0)
    if scheme == "lts2":
        c.step_scheme("lts2", w.dt_coarse, w.M, 4)
        rh, ru = o.lts(w.h0, w.u0, w.dt_coarse, w.M, R, n=4, order=2)
    elif scheme == "rk4":
        c.step_scheme("rk4", w.dt_coarse / w.M, 1, 8)
        rh, ru = o.rk4(w.h0, w.u0, w.dt_coarse / w.M, n=8)
    else:
        c.step_scheme("ssprk3", w.dt_coarse / w.M, 1, 8)
        rh, ru = o.ssprk(w.h0, w.u0, w.dt_coarse / w.M, n=8)
    gh, gu = c.get_state()
    assert rel_l2(gh, rh, w.mesh.areaCell) < 1e-12
    assert rel_l2(gu, ru) < 1e-11
    c.close()


def test_small_sphere_lts3_fp32(small):
    w, o, R = small
    say("sphere10k lts3 fp32")
    c = _ctx(w, "fp32")
    c.init_state(w.h0, w.u0)
    c.step(w.dt_coarse, w.M, 6)
    gh, gu = c.get_state()
    rh, ru = o.lts(w.h0, w.u0, w.dt_coarse, w.M, R, n=6)
    assert rel_l2(gh, rh, w.mesh.areaCell) < 1e-5
    assert rel_l2(gu, ru) < 1e-5
    c.close()


def test_small_sphere_tc5_fp64_and_fp32():
    """Zonal flow over the isolated mountain on the 10k cap mesh: FP64 LTS3
    against the oracle, FP32 within 1e-5, mass to 1e-13 (FP64)."""
    w = workloads.sphere_cap(n=10_000, iters=25, case="tc5")
    say("sphere10k tc5")
    o = Oracle(w.mesh, w.gravity)
    R = o.regions(w.fine_mask, w.n_if1, w.n_if2)
    rh, ru = o.lts(w.h0, w.u0, w.dt_coarse, w.M, R, n=6)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        c = _ctx(w, prec)
        c.init_state(w.h0, w.u0)
        c.step(w.dt_coarse, w.M, 6)
        gh, gu = c.get_state()
        assert rel_l2(gh, rh, w.mesh.areaCell) < tol
        assert rel_l2(gu, ru) < (1e-11 if prec == "fp64" else tol)
        if prec == "fp64":
            m0, _ = o.diagnostics(w.h0, w.u0)
            assert abs(c.diagnostics().mass - m0) <= 1e-13 * m0
        c.close()


@pytest.fixture(scope="module")
def full():
    w = workloads.sphere_cap()
    say("sphere full size", w.mesh.nCells, "cells, maxE", w.mesh.maxEdges)
    o = Oracle(w.mesh, w.gravity)
    R = o.regions(w.fine_mask, w.n_if1, w.n_if2)
    rh, ru = o.lts(w.h0, w.u0, w.dt_coarse, w.M, R, n=2)
    w.extra["oracle_diag"] = o.diagnostics(rh, ru)
    return w, rh, ru


@pytest.mark.parametrize("prec,tol_h,tol_u", [("fp64", 1e-12, 1e-11), ("fp32", 1e-5, 1e-5)])
def test_full_sphere_lts3(full, prec, tol_h, tol_u):
    w, rh, ru = full
    say("sphere full lts3", prec)
    c = _ctx(w, prec)
    c.init_state(w.h0, w.u0)
    c.step(w.dt_coarse, w.M, 2)
    gh, gu = c.get_state()
    m = w.mesh
    eh = rel_l2(gh, rh, m.areaCell)
    eu = rel_l2(gu, ru, m.dvEdge * m.dcEdge)
    # surface anomaly eta = h + b - mean(h + b) (the dynamic part of h)
    Hs = float((m.areaCell * (rh + m.bottom)).sum() / m.areaCell.sum())
    ea = rel_l2(gh + m.bottom - Hs, rh + m.bottom - Hs, m.areaCell)
    d = c.diagnostics()
    m_ref, e_ref = w.extra["oracle_diag"]
    em, ee = abs(d.mass - m_ref) / m_ref, abs(d.energy - e_ref) / abs(e_ref)
    say("rel L2 h", eh, "eta", ea, "u", eu, "mass", em, "energy", ee)
    assert eh < tol_h and eu < tol_u
    if prec == "fp32":
        assert ea < FP32_SPHERE_ETA_TOL and em < FP32_SPHERE_MASS_TOL
        assert ee < FP32_SPHERE_ENERGY_TOL
    else:
        assert ea < 1e-11 and em < 1e-13 and ee < 1e-12
    c.close()
