"""GPU parity on a mesh with one 11-sided cell: cells above 8 edges take the
16-lane slot tables (G = 16), so these cases run the 16-lane instantiations
of the single-range, layered (both thread maps) and batched cell kernels.
The 11-gon sits in the fine region, the first interface ring or the coarse
region.  Tolerances as in the other parity tests: FP64 relative L2 1e-12
on h and one RHS, 1e-11 on u after several steps; FP32 1e-5."""
import math
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2106_07154_amd import lts
from paper_2106_07154_amd.inputs import gaussian_bump_state, random_state
from paper_2106_07154_amd.inputs.cases import disk_fine_mask

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b, w=None):
    w = np.ones_like(b) if w is None else w
    return math.sqrt((w * (a - b) ** 2).sum() / max((w * b ** 2).sum(), 1e-300))


@pytest.fixture(scope="module")
def wide(ring_mesh):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m = ring_mesh
    assert m.nEdgesOnCell.max() == 11
    c11 = int(np.argmax(m.nEdgesOnCell))
    x0, y0 = m.xCell[c11], m.yCell[c11]
    masks = {
        # the 11-gon and its neighbours fine
        "fine11": disk_fine_mask(m, x0, y0, 2.5e4),
        # fine disk 40 km away: the 11-gon is in the first interface ring
        "iface11": disk_fine_mask(m, (x0 + m.Lx / 4) % m.Lx, y0, 2.0e4),
        # fine disk half the domain away: the 11-gon is coarse
        "coarse11": disk_fine_mask(m, (x0 + m.Lx / 2) % m.Lx, (y0 + m.Ly / 2) % m.Ly, 2.0e4),
    }
    o = Oracle(m)
    for name, want in (("fine11", 3), ("iface11", 2), ("coarse11", 0)):
        assert o.regions(masks[name], 2, 2).cell[c11] == want, name
    h, u = gaussian_bump_state(m, 500.0, 5.0, 2.0e4, x0 + 5e3, y0 - 3e3)
    h2, u2 = random_state(m, 21, H=0.0, amp_h=0.2, amp_u=0.05)
    h, u = h + h2, u + u2
    dt = 0.2 * m.dcEdge.min() / math.sqrt(9.81 * 500.0) * 4
    return m, masks, o, h, u, dt


def _ctx(m, fm, prec="fp64", layers=1):
    c = lts.LTSContext(0, prec, layers=layers)
    c.upload_mesh(m, fm, 2, 2)
    return c


def test_wide_cell_rhs(wide):
    m, masks, o, h, u, dt = wide
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        say("wide rhs", prec)
        c = _ctx(m, masks["fine11"], prec)
        hh, uu = random_state(m, 22, H=1000.0, amp_h=3.0, amp_u=1.0)
        dh, du = c.eval_rhs(hh, uu)
        rh, ru = o.rhs(hh, uu)
        say("rhs rel L2", rel_l2(dh, rh), rel_l2(du, ru))
        assert rel_l2(dh, rh) < tol and rel_l2(du, ru) < tol
        c.close()


@pytest.mark.parametrize("mask", ["fine11", "iface11", "coarse11"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wide_cell_lts3(wide, mask, prec):
    m, masks, o, h, u, dt = wide
    fm = masks[mask]
    say("wide lts3", mask, prec)
    R = o.regions(fm, 2, 2)
    c = _ctx(m, fm, prec)
    c.init_state(h, u)
    c.step(dt, 4, 8)
    gh, gu = c.get_state()
    rh, ru = o.lts(h, u, dt, 4, R, n=8)
    eh, eu = rel_l2(gh, rh, m.areaCell), rel_l2(gu, ru)
    say("rel L2 h", eh, "u", eu)
    tol_h, tol_u = (1e-12, 1e-11) if prec == "fp64" else (1e-5, 1e-5)
    assert eh < tol_h and eu < tol_u
    c.close()


@pytest.mark.parametrize("nl", [3, 70])
def test_wide_cell_layers(wide, nl):
    """3 layers: one thread per (cell, layer); 70 layers: one wave per cell
    over 64 layers plus a ragged chunk of 6."""
    m, masks, o, h, u, dt = wide
    fm = masks["fine11"]
    say("wide layers", nl)
    R = o.regions(fm, 2, 2)
    states = [(h, u), (h + 0.5 * (h - h.mean()), 1.5 * u), (h.mean() + 0 * h, 0 * u + 0.01)]
    idx = np.arange(nl) % len(states)
    c = _ctx(m, fm, "fp64", layers=nl)
    c.init_state(np.array([states[k][0] for k in idx]), np.array([states[k][1] for k in idx]))
    c.step(dt, 4, 3)
    gh, gu = c.get_state()
    for k, (hk, uk) in enumerate(states):
        rh, ru = o.lts(hk, uk, dt, 4, R, n=3)
        ls = np.flatnonzero(idx == k)
        for l in ls:
            assert np.array_equal(gh[l], gh[ls[0]]) and np.array_equal(gu[l], gu[ls[0]])
        eh, eu = rel_l2(gh[ls[0]], rh, m.areaCell), rel_l2(gu[ls[0]], ru)
        say("state", k, "rel L2 h", eh, "u", eu)
        assert eh < 1e-12 and eu < 1e-11
    c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wide_cell_ensemble(wide, irregular, prec):
    """A 16-lane member batched with an 8-lane one reproduces each member
    advanced alone."""
    m, masks, o, h, u, dt = wide
    fm2 = disk_fine_mask(irregular, irregular.Lx / 2, irregular.Ly / 2, 3.0e4)
    h2, u2 = gaussian_bump_state(irregular, 500.0, 3.0, 3.0e4, irregular.Lx / 2,
                                 irregular.Ly / 2)
    dt2 = 0.2 * irregular.dcEdge.min() / math.sqrt(9.81 * 500.0) * 2
    members = [(m, masks["fine11"], h, u, dt, 4), (irregular, fm2, h2, u2, dt2, 2)]
    say("wide ensemble", prec)
    ens = lts.Ensemble(0, prec)
    for mm, fm, hh, uu, d, M in members:
        ens.add_member(mm, fm, d, M)
    for j, (mm, fm, hh, uu, d, M) in enumerate(members):
        ens.init_member(j, hh, uu)
    ens.build(autotune=True)
    ens.step(3)
    tol = 1e-14 if prec == "fp64" else 1e-6
    for j, (mm, fm, hh, uu, d, M) in enumerate(members):
        gh, gu = ens.get_member(j)
        c = _ctx(mm, fm, prec)
        c.init_state(hh, uu)
        c.step(d, M, 3)
        rh, ru = c.get_state()
        c.close()
        say("member", j, "rel", rel_l2(gh, rh), rel_l2(gu, ru))
        assert rel_l2(gh, rh) <= tol and rel_l2(gu, ru) <= tol * 10
    gh, gu = ens.get_member(0)
    rh, ru = o.lts(h, u, dt, 4, o.regions(masks["fine11"], 2, 2), n=3)
    assert rel_l2(gh, rh, m.areaCell) < (1e-12 if prec == "fp64" else 1e-5)
    ens.close()


def _restride(m, cap):
    """The same mesh with its per-cell arrays declared at capacity `cap`
    (MPAS meshes declare maxEdges = 10 or more whatever the cells hold);
    unused entries are -1."""
    w = m.copy()
    w.maxEdges = cap
    for name in ("edgesOnCell", "cellsOnCell", "verticesOnCell"):
        a = getattr(m, name)
        b = np.full((m.nCells, cap), -1, dtype=a.dtype)
        b[:, :a.shape[1]] = a
        for i in range(m.nCells):
            b[i, m.nEdgesOnCell[i]:] = -1
        setattr(w, name, b)
    return w


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_declared_capacity_is_not_the_lane_count(hex16, prec):
    """A hexagonal mesh declared with max_edges = 16 runs the same kernels as
    the same mesh declared with 6: the lane count follows the largest cell
    present.  Results are bitwise those of the compact declaration and match
    the oracle (FP64 1e-12 h, 1e-11 u; FP32 1e-5)."""
    import torch
    from paper_2106_07154_amd.inputs import igw_parameters, igw_state, strip_fine_mask
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    say("declared capacity 16", prec)
    m = hex16
    w = _restride(m, 16)
    fm = strip_fine_mask(m, 6, 9, 1.0e4)
    h0, u0 = igw_state(m, igw_parameters(m), 0.0)
    out = []
    for mesh in (m, w):
        c = lts.LTSContext(0, prec)
        c.upload_mesh(mesh, fm, 2, 2)
        c.init_state(h0, u0)
        c.step(30.0, 4, 6)
        out.append(c.get_state())
        c.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    o = Oracle(m)
    rh, ru = o.lts(h0, u0, 30.0, 4, o.regions(fm, 2, 2), n=6)
    tol_h, tol_u = (1e-12, 1e-11) if prec == "fp64" else (1e-5, 1e-5)
    assert rel_l2(out[1][0], rh) < tol_h and rel_l2(out[1][1], ru) < tol_u


@pytest.fixture(scope="module")
def wide_levels():
    """A 32 x 32 ring lattice (10 km, one 11-gon at the centre) with nested
    fine disks placing the 11-gon in the inner fine region, the inner first
    interface ring, the inner coarse region (fine at level 0) or the outer
    first interface ring."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_07154_amd.inputs.voronoi_planar import periodic_voronoi_mesh, ring_hex_points
    p, Lx, Ly = ring_hex_points(32, 32, 1.0e4, 11, 1.2, 30)
    m = periodic_voronoi_mesh(p, Lx, Ly, f0=1.0e-4, name="ring11-32")
    assert m.nEdgesOnCell.max() == 11
    rng = np.random.default_rng(14)
    m.bottom = 20.0 * rng.standard_normal(m.nCells)
    c11 = int(np.argmax(m.nEdgesOnCell))
    x0, y0 = m.xCell[c11], m.yCell[c11]
    d = lambda cx, r: disk_fine_mask(m, cx % Lx, y0, r)
    cases = {"inner_f": ([d(x0, 1.2e5), d(x0, 2.5e4)], (3, 3)),
             "inner_i1": ([d(x0, 1.3e5), d(x0 + 3.5e4, 2.0e4)], (3, 2)),
             "inner_c": ([d(x0 + 5e4, 1.25e5), d(x0 + 8e4, 2.0e4)], (3, 0)),
             "outer_i1": ([d(x0 + 1.05e5, 1.0e5), d(x0 + 1.1e5, 2.0e4)], (2, 0))}
    o = Oracle(m)
    for name, (masks, want) in cases.items():
        R = o.ml_regions(masks, 2, 2)
        assert (R.cell[0][c11], R.cell[1][c11]) == want, name
        lts.plan_levels(m, masks, 2, 2)  # the library's nesting rule (four rings) holds too
    h, u = gaussian_bump_state(m, 500.0, 5.0, 2.0e4, x0 + 5e3, y0 - 3e3)
    h2, u2 = random_state(m, 23, H=0.0, amp_h=0.2, amp_u=0.05)
    dt = 0.2 * m.dcEdge.min() / math.sqrt(9.81 * 500.0) * 6
    return m, cases, o, h + h2, u + u2, dt


@pytest.mark.parametrize("case", ["inner_f", "inner_i1", "inner_c", "outer_i1"])
def test_wide_cell_multilevel(wide_levels, case):
    """Three-level LTS3 (ratios 2 and 3) with the 11-gon in each part of the
    nested regions: FP64 parity with the oracle's multi-level step."""
    m, cases, o, h, u, dt = wide_levels
    masks = cases[case][0]
    say("wide multilevel", case)
    c = lts.LTSContext(0, "fp64")
    c.upload_mesh_levels(m, masks, 2, 2)
    c.init_state(h, u)
    c.step_levels(dt, (2, 3), 4)
    gh, gu = c.get_state()
    c.close()
    rh, ru = o.mlts(h, u, dt, [2, 3], o.ml_regions(masks, 2, 2), n=4)
    eh, eu = rel_l2(gh, rh, m.areaCell), rel_l2(gu, ru, m.dvEdge * m.dcEdge)
    say("rel L2 h u", eh, eu)
    assert eh < 1e-12 and eu < 1e-11
