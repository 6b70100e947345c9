"""GPU parity of multi-level LTS3 (Remark 3.1: nested fine regions, an
integer step ratio between neighbouring levels) against the oracle's
om_mlts_step, through the C ABI.

Tolerances as in the two-level parity tests: FP64 relative L2 1e-12 on h and
1e-11 on u (the u tendency is a difference of g(h + b) ~ gH terms whose
rounding order differs), FP32 1e-5 on total h and u; labels bit-exact; mass
drift 1e-13 over 100 coarse steps.
"""
import math
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2106_07154_amd import lts
from paper_2106_07154_amd.inputs import (gaussian_bump_state, igw_parameters, igw_state,
                                         periodic_hex_mesh, random_state, strip_fine_mask)
from paper_2106_07154_amd.inputs.cases import disk_fine_mask

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b, w=None):
    w = np.ones_like(b) if w is None else w
    return math.sqrt((w * (a - b) ** 2).sum() / max((w * b ** 2).sum(), 1e-300))


@pytest.fixture(scope="module", autouse=True)
def gpu_lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lts.load_library()


@pytest.fixture(scope="module")
def strips():
    """32 x 32 periodic hexagonal mesh (dc = 20 km), 20 m inertia-gravity
    wave; fine strips of rows 6-25 (level 0) and 14-17 (level 1)."""
    n, dc = 32, 20e3
    m = periodic_hex_mesh(n, n, dc, f0=1e-4)
    h0, u0 = igw_state(m, igw_parameters(m, amp=20.0), 0.0)
    masks = [strip_fine_mask(m, 6, 25, dc), strip_fine_mask(m, 14, 17, dc)]
    return m, h0, u0, masks


@pytest.fixture(scope="module")
def strips4():
    """48 x 48 hexagonal mesh with three nested strips (four LTS levels)."""
    n, dc = 48, 20e3
    m = periodic_hex_mesh(n, n, dc, f0=1e-4)
    h0, u0 = igw_state(m, igw_parameters(m, amp=20.0), 0.0)
    masks = [strip_fine_mask(m, 6, 41, dc), strip_fine_mask(m, 14, 33, dc),
             strip_fine_mask(m, 22, 25, dc)]
    return m, h0, u0, masks


@pytest.fixture(scope="module")
def disks():
    """Irregular periodic Voronoi mesh (jittered 32 x 32 lattice, 4- to
    8-gons, random topography and Coriolis), nested disks of 120 and 25 km,
    a Gaussian bump plus random state."""
    from paper_2106_07154_amd.inputs.voronoi_planar import (jittered_hex_points,
                                                            periodic_voronoi_mesh)
    p, Lx, Ly = jittered_hex_points(32, 32, 1.0e4, 0.55, seed=58)
    m = periodic_voronoi_mesh(p, Lx, Ly, f0=1.0e-4, name="irregular32")
    rng = np.random.default_rng(32)
    m.bottom = 20.0 * rng.standard_normal(m.nCells)
    m.fVertex = 1.0e-4 + 2.0e-5 * rng.standard_normal(m.nVertices)
    cx, cy = m.Lx / 2, m.Ly / 2
    masks = [disk_fine_mask(m, cx, cy, 1.2e5), disk_fine_mask(m, cx + 1e4, cy, 2.5e4)]
    h, u = gaussian_bump_state(m, 500.0, 5.0, 3.0e4, cx, cy)
    h2, u2 = random_state(m, 33, H=0.0, amp_h=0.2, amp_u=0.05)
    return m, h + h2, u + u2, masks


def _ctx(m, masks, prec="fp64"):
    c = lts.LTSContext(0, prec)
    c.upload_mesh_levels(m, masks, 2, 2)
    return c


@pytest.mark.parametrize("case", ["strips", "strips4", "disks"])
def test_level_labels_match_oracle(case, request):
    m, h0, u0, masks = request.getfixturevalue(case)
    say("multilevel labels", case)
    c = _ctx(m, masks)
    R = Oracle(m).ml_regions(masks, 2, 2)
    for l in range(len(masks)):
        cr, er, cf, ef = c.level_regions(l)
        assert np.array_equal(cr, R.cell[l]) and np.array_equal(er, R.edge[l])
        assert np.array_equal(cf, R.cell_fbar[l]) and np.array_equal(ef, R.edge_fbar[l])
    c.close()


@pytest.mark.parametrize("case,Ms,dt,n", [("strips", (2, 2), 60.0, 20),
                                          ("strips", (3, 2), 60.0, 10),
                                          ("strips4", (2, 2, 2), 60.0, 6),
                                          ("disks", (2, 3), 40.0, 12)])
def test_multilevel_parity_fp64(case, Ms, dt, n, request):
    m, h0, u0, masks = request.getfixturevalue(case)
    say("multilevel fp64", case, Ms, dt, n)
    c = _ctx(m, masks)
    c.init_state(h0, u0)
    c.step_levels(dt, Ms, n)
    h, u = c.get_state()
    d = c.diagnostics()
    c.close()
    o = Oracle(m)
    rh, ru = o.mlts(h0, u0, dt, list(Ms), o.ml_regions(masks, 2, 2), n=n)
    eh, eu = rel_l2(h, rh, m.areaCell), rel_l2(u, ru, m.dvEdge * m.dcEdge)
    say("rel L2 h u", eh, eu)
    assert eh < 1e-12 and eu < 1e-11
    assert d.steps == n and d.n_nonfinite == 0


@pytest.mark.parametrize("case,Ms", [("strips", (2, 2)), ("disks", (2, 3))])
def test_multilevel_parity_fp32(case, Ms, request):
    m, h0, u0, masks = request.getfixturevalue(case)
    say("multilevel fp32", case, Ms)
    dt, n = (60.0, 10) if case == "strips" else (40.0, 8)
    c = _ctx(m, masks, "fp32")
    c.init_state(h0, u0)
    c.step_levels(dt, Ms, n)
    h, u = c.get_state()
    c.close()
    o = Oracle(m)
    rh, ru = o.mlts(h0, u0, dt, list(Ms), o.ml_regions(masks, 2, 2), n=n)
    eh, eu = rel_l2(h, rh, m.areaCell), rel_l2(u, ru, m.dvEdge * m.dcEdge)
    say("rel L2 h u", eh, eu)
    assert eh < 1e-5 and eu < 1e-5


def test_multilevel_conserves_mass(strips):
    m, h0, u0, masks = strips
    say("multilevel mass")
    rng = np.random.default_rng(5)
    h = h0 + 0.3 * rng.standard_normal(m.nCells)
    c = _ctx(m, masks)
    c.init_state(h, u0)
    m0 = c.diagnostics().mass
    c.step_levels(60.0, (2, 3), 100)
    d = c.diagnostics()
    c.close()
    say("mass drift", abs(d.mass - m0) / m0)
    assert d.n_nonfinite == 0 and abs(d.mass - m0) / m0 < 1e-13


def test_ratio_one_reductions(strips):
    """An inner ratio of 1 gives the two-level LTS3 step; all ratios 1 give
    SSPRK3 (Remark 2.3), both to rounding; and lts_step on a multi-level
    mesh is the two-level scheme on level 0's regions."""
    m, h0, u0, masks = strips
    say("multilevel ratio-one reductions")
    a = _ctx(m, masks)
    a.init_state(h0, u0)
    a.step_levels(60.0, (3, 1), 10)
    ha, ua = a.get_state()
    a.init_state(h0, u0)
    a.step(60.0, 3, 10)
    hb, ub = a.get_state()
    a.init_state(h0, u0)
    a.step_levels(60.0, (1, 1), 10)
    hc, uc = a.get_state()
    a.close()
    b = lts.LTSContext(0, "fp64")
    b.upload_mesh(m, masks[0], 2, 2)
    b.init_state(h0, u0)
    b.step(60.0, 3, 10)
    hd, ud = b.get_state()
    b.init_state(h0, u0)
    b.step_rk3(60.0, 10)
    he, ue = b.get_state()
    b.close()
    w, wu = m.areaCell, m.dvEdge * m.dcEdge
    assert np.array_equal(hb, hd) and np.array_equal(ub, ud)
    assert rel_l2(ha, hd, w) < 1e-13 and rel_l2(ua, ud, wu) < 1e-11
    assert rel_l2(hc, he, w) < 1e-13 and rel_l2(uc, ue, wu) < 1e-11


def test_level_errors(strips):
    m, h0, u0, masks = strips
    say("multilevel errors")
    dc = 20e3
    c = lts.LTSContext(0, "fp64")
    # inner interface rings within three rings of the outer interface
    with pytest.raises(lts.LTSError) as ei:
        c.upload_mesh_levels(m, [masks[0], strip_fine_mask(m, 10, 21, dc)], 2, 2)
    assert ei.value.status == lts.LTS_ELABEL
    # a two-level mesh has no level ratios to step with
    c.upload_mesh(m, masks[0], 2, 2)
    c.init_state(h0, u0)
    with pytest.raises(lts.LTSError) as ei:
        c.step_levels(60.0, (2, 2), 1)
    assert ei.value.status == lts.LTS_EINVAL
    c.upload_mesh_levels(m, masks, 2, 2)
    c.init_state(h0, u0)
    with pytest.raises(lts.LTSError) as ei:
        c.step_levels(60.0, (2, 0), 1)
    assert ei.value.status == lts.LTS_EINVAL
    c.close()


def test_multilevel_parity_vr3_full_size():
    """The benchmark's three-level configuration at full size
    (vr3-planar-800k, ratios (4, 2), level 1 the 61k-cell disk inside the
    410k-cell level-0 region): labels bit-exact, and two coarse steps from a
    state with flow against the oracle's multi-level step at the two-level
    full-size tolerances (h 1e-12, u 1e-11, the perturbation h - H 1e-9)."""
    import os
    from paper_2106_07154_amd.inputs import workloads as wl
    w = wl.vr3_planar()
    m = w.mesh
    masks = [w.fine_mask, (w.extra["level1_mask"] & w.fine_mask).astype(np.uint8)]
    say("multilevel vr3 full size", m.nCells)
    o = Oracle(m, w.gravity, threads=min(16, os.cpu_count() or 1))
    R = o.ml_regions(masks, 2, 2)
    h, u = o.ssprk(w.h0, w.u0, w.dt_coarse / w.M, n=8)
    c = lts.LTSContext(0, "fp64")
    c.upload_mesh_levels(m, masks, 2, 2, w.gravity)
    for l in range(2):
        cr, er, cf, ef = c.level_regions(l)
        assert np.array_equal(cr, R.cell[l]) and np.array_equal(er, R.edge[l])
    c.init_state(h, u)
    c.step_levels(w.dt_coarse, (4, 2), 2)
    gh, gu = c.get_state()
    c.close()
    rh, ru = o.mlts(h, u, w.dt_coarse, [4, 2], R, n=2)
    eh, eu = rel_l2(gh, rh, m.areaCell), rel_l2(gu, ru, m.dvEdge * m.dcEdge)
    ep = rel_l2(gh - 500.0, rh - 500.0, m.areaCell)
    say("rel L2 h u h-H", eh, eu, ep)
    assert eh < 1e-12 and eu < 1e-11 and ep < 1e-9


@pytest.mark.parametrize("L,prec", [(3, "fp64"), (3, "fp32"), (64, "fp64")])
def test_multilevel_layers_parity(disks, L, prec):
    """Multi-level LTS3 on a layered context: L independent layers with
    different states, each against the oracle's multi-level step on that
    layer alone (3 layers: one thread per (element, layer); 64: one wave per
    element), at the single-layer tolerances; the mass of all layers is
    conserved to 1e-13 in FP64."""
    m, h0, u0, masks = disks
    say("multilevel layers", L, prec)
    rng = np.random.default_rng(70 + L)
    hs = np.array([h0 + 0.2 * (l % 5) * rng.standard_normal(m.nCells) for l in range(L)])
    us = np.array([u0 * (1.0 + 0.1 * (l % 7)) for l in range(L)])
    Ms, dt, n = (2, 3), 40.0, 4
    c = lts.LTSContext(0, prec, layers=L)
    c.upload_mesh_levels(m, masks, 2, 2)
    c.init_state(hs, us)
    m0 = c.diagnostics().mass
    c.step_levels(dt, Ms, n)
    gh, gu = c.get_state()
    d = c.diagnostics()
    c.close()
    o = Oracle(m)
    R = o.ml_regions(masks, 2, 2)
    tol_h, tol_u = (1e-12, 1e-11) if prec == "fp64" else (1e-5, 1e-5)
    worst = (0.0, 0.0)
    for l in range(L):
        rh, ru = o.mlts(hs[l], us[l], dt, list(Ms), R, n=n)
        eh, eu = rel_l2(gh[l], rh, m.areaCell), rel_l2(gu[l], ru, m.dvEdge * m.dcEdge)
        worst = (max(worst[0], eh), max(worst[1], eu))
        assert eh < tol_h and eu < tol_u, (l, eh, eu)
    say("worst rel L2 h u over layers", *worst)
    assert d.n_nonfinite == 0
    if prec == "fp64":
        say("mass drift", abs(d.mass - m0) / m0)
        assert abs(d.mass - m0) / m0 < 1e-13
