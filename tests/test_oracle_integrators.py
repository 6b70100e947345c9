"""Pins on the oracle's time integrators: Algorithm 2.1 (SSPRK2/3), RK4 and
Algorithm 2.2 (LTS2/LTS3), plus the LTS index sets.

Independent anchors: stability polynomials on the linearised system (dense
Jacobian by brute-force central differences), the paper's M = 1 identity
(Remark 2.3), exact discrete mass conservation, the Taylor consistency of the
interface-1 predictions derived from the stage polynomials, convergence order
against an RK4 reference, and region counts derived by hand for the strip.
"""
import math

import numpy as np
import pytest

import oracle as om
from oracle import Oracle
from paper_2106_07154_amd.inputs import (igw_parameters, igw_state, periodic_hex_mesh,
                                         strip_fine_mask)


# ---------------------------------------------------------------- helpers
def _rel_l2(a, b, w=None):
    w = np.ones_like(a) if w is None else w
    return math.sqrt((w * (a - b) ** 2).sum() / (w * b ** 2).sum())


@pytest.fixture(scope="module")
def linearised(hex8):
    """Dense Jacobian L of the RHS at the state of rest (h = H, u = 0)."""
    m = hex8
    o = Oracle(m)
    H = 1000.0
    nC, nE = m.nCells, m.nEdges
    n = nC + nE
    L = np.zeros((n, n))
    eps = 1e-2
    h0 = np.full(nC, H)
    u0 = np.zeros(nE)
    for j in range(n):
        hp, up = h0.copy(), u0.copy()
        hm, um = h0.copy(), u0.copy()
        if j < nC:
            hp[j] += eps
            hm[j] -= eps
        else:
            up[j - nC] += eps
            um[j - nC] -= eps
        a = np.concatenate(o.rhs(hp, up))
        b = np.concatenate(o.rhs(hm, um))
        L[:, j] = (a - b) / (2 * eps)
    return m, o, L, H


@pytest.mark.parametrize("scheme,coeffs", [
    ("ssprk2", [1, 1, 1 / 2]),
    ("ssprk3", [1, 1, 1 / 2, 1 / 6]),
    ("rk4", [1, 1, 1 / 2, 1 / 6, 1 / 24]),
])
def test_step_matches_stability_polynomial(linearised, scheme, coeffs):
    """For a small perturbation y of the rest state one step maps y to
    p(dt L) y with p the truncated exponential of the scheme's order."""
    m, o, L, H = linearised
    rng = np.random.default_rng(1)
    n = m.nCells + m.nEdges
    y = 1e-6 * rng.standard_normal(n)
    dt = 40.0
    h = H + y[:m.nCells]
    u = y[m.nCells:]
    if scheme == "rk4":
        h1, u1 = o.rk4(h, u, dt)
    else:
        h1, u1 = o.ssprk(h, u, dt, order=int(scheme[-1]))
    got = np.concatenate([h1 - H, u1])
    Z = dt * L
    want = np.zeros(n)
    term = y.copy()
    for c in coeffs:
        want += c * term
        term = Z @ term
    # a wrong stage coefficient changes the result by ~1e-2 relative
    assert np.abs(got - want).max() < 1e-6 * np.abs(want).max()
    assert np.abs(Z).max() > 0.2


# ---------------------------------------------------------------- regions
def test_region_counts_igw_strip(hex64):
    """Fine strip of hex rows 28-35 with two rings per interface layer:
    F = 512 (underlined F = 256), I1 = 256, I2 = 256, C = 3072 cells; edges
    all-fine 1664 (underlined 768), I1 768, I2 768, C 9088 (counted by hand
    from the row structure: 3 edges per cell)."""
    o = Oracle(hex64)
    R = o.regions(strip_fine_mask(hex64, 28, 35, 1e4), 2, 2)
    assert [int((R.cell == k).sum()) for k in (om.C, om.I2, om.I1, om.F)] == [3072, 256, 256, 512]
    assert [int((R.edge == k).sum()) for k in (om.C, om.I2, om.I1, om.F)] == [9088, 768, 768, 1664]
    assert int(R.cell_fbar.sum()) == 256 and int(R.edge_fbar.sum()) == 768


def test_region_definitions_brute_force(irregular):
    """Check eq:indexSetsCells/eq:index_sets_cells/eq:indexSetsEdges directly."""
    m = irregular
    o = Oracle(m)
    fm = (np.hypot(m.xCell - m.Lx / 2, m.yCell - m.Ly / 2) < 3.5e4).astype(np.uint8)
    R = o.regions(fm, 2, 1)
    nb = [set(m.cellsOnCell[i, :m.nEdgesOnCell[i]]) for i in range(m.nCells)]
    F = set(np.nonzero(fm)[0])
    # breadth-first rings
    ring = {i: 0 for i in F}
    frontier = set(F)
    for r in (1, 2, 3):
        new = {j for i in frontier for j in nb[i] if j not in ring}
        for j in new:
            ring[j] = r
        frontier = new
    for i in range(m.nCells):
        want = om.F if i in F else om.I1 if ring.get(i) in (1, 2) else \
            om.I2 if ring.get(i) == 3 else om.C
        assert R.cell[i] == want
    F1 = {i for i in F if any(R.cell[j] == om.I1 for j in nb[i])}
    F2 = {i for i in F - F1 if nb[i] & F1}
    assert set(np.nonzero(R.cell_fbar)[0]) == F1 | F2
    Fin = F - F1 - F2
    for e in range(m.nEdges):
        c0, c1 = m.cellsOnEdge[e]
        assert R.edge[e] == max(R.cell[c0], R.cell[c1])
        fb = bool({c0, c1} & (F1 | F2)) and not ({c0, c1} & Fin)
        assert bool(R.edge_fbar[e]) == fb


def test_region_errors(hex8):
    o = Oracle(hex8)
    with pytest.raises(ValueError):
        o.regions(np.zeros(hex8.nCells, np.uint8))
    with pytest.raises(ValueError):
        o.regions(np.ones(hex8.nCells, np.uint8))
    with pytest.raises(ValueError):
        o.regions(strip_fine_mask(hex8, 2, 3, 1e4), 0, 2)


# ---------------------------------------------------------------- LTS
def test_predict_coeffs_taylor_consistency():
    """The interface-1 prediction a x_old + b x_1st + c x_2nd must agree to
    second order with the fine SSPRK3 stage it stands in for.  For y' = z y over
    one coarse step: x_old = 1, x_1st = 1 + z, x_2nd = 1 + z/2 + z^2/4; the
    fine stage values at substep k (w = z/M) are S_k, S_k (1 + w) and
    S_k (1 + w/2 + w^2/4) with S_k = e^{k w} + O(w^4).  Solving for (a, b, c)
    from these polynomials reproduces the printed alpha/beta/gamma formulas."""
    P = np.polynomial.polynomial
    basis = np.array([[1, 0, 0], [1, 1, 0], [1, 0.5, 0.25]]).T  # columns: x_old,x_1st,x_2nd
    for M in (1, 2, 3, 4, 8, 25):
        for k in range(M):
            Sk = np.array([1, k / M, (k / M) ** 2 / 2])  # e^{k w} to O(z^2)
            def first3(p):
                p = np.asarray(p, float)
                return np.concatenate([p, np.zeros(3)])[:3]
            stages = [Sk, P.polymul(Sk, [1, 1.0 / M]),
                      P.polymul(Sk, [1, 0.5 / M, 0.25 / M ** 2])]
            for s, target in enumerate(stages):
                want = np.linalg.solve(basis, first3(target))
                got = om.predict_coeffs(3, s, k, M)
                np.testing.assert_allclose(got, want, atol=1e-14)
            # LTS2: first-order agreement with x_old, x_1st only
            for s, frac in enumerate((k / M, (k + 1) / M)):
                got = om.predict_coeffs(2, s, k, M)
                np.testing.assert_allclose(got, [1 - frac, frac, 0.0], atol=1e-15)
    # M = 1 returns the coarse stages themselves
    for s in range(3):
        np.testing.assert_allclose(om.predict_coeffs(3, s, 0, 1), np.eye(3)[s], atol=1e-15)


@pytest.fixture(scope="module")
def igw_case(hex64):
    o = Oracle(hex64)
    p = igw_parameters(hex64)
    h0, u0 = igw_state(hex64, p, 0.0)
    R = o.regions(strip_fine_mask(hex64, 28, 35, 1e4), 2, 2)
    return hex64, o, h0, u0, R


@pytest.mark.parametrize("order", [3, 2])
def test_lts_m1_equals_ssprk(igw_case, order):
    """Remark 2.3: with M = 1 LTS reproduces SSPRK of the same order to machine
    precision (Step 5 is the Butcher form of the Shu-Osher stages)."""
    m, o, h0, u0, R = igw_case
    h1, u1 = o.lts(h0, u0, 30.0, 1, R, n=1, order=order)
    h2, u2 = o.ssprk(h0, u0, 30.0, n=1, order=order)
    assert np.abs(h1 - h2).max() <= 1e-14 * np.abs(h2).max()
    assert np.abs(u1 - u2).max() <= 1e-14 * np.abs(u2).max() + 1e-16
    # SSPRK2 amplifies imaginary-axis modes (|p(iy)|^2 = 1 + y^4/4), so its
    # roundoff grows faster; the long run is checked for LTS3 over 200 steps
    # and for LTS2 over 20.
    nsteps = 200 if order == 3 else 20
    h1, u1 = o.lts(h0, u0, 30.0, 1, R, n=nsteps, order=order)
    h2, u2 = o.ssprk(h0, u0, 30.0, n=nsteps, order=order)
    assert _rel_l2(h1, h2, m.areaCell) < 1e-12
    # u is driven by differences of g(h+b) ~ gH whose ulp is 1.8e-12: each step
    # can move u by ~3 dt ulp(gH)/d_e = 1.6e-14 m/s, i.e. ~5e-12 of rms(u) ~ 0.04
    # m/s after 200 steps, so 1e-11 is the floor for two correct orderings.
    assert _rel_l2(u1, u2, m.dvEdge * m.dcEdge) < 1e-11


@pytest.mark.parametrize("order,M", [(3, 4), (3, 8), (2, 4)])
def test_lts_conserves_mass(igw_case, order, M):
    """Exact discrete mass conservation (the reason for interface layer 2):
    relative drift below 1e-13 over 200 coarse steps."""
    m, o, h0, u0, R = igw_case
    rng = np.random.default_rng(3)
    h = h0 + 0.3 * rng.standard_normal(m.nCells)
    m0, _ = o.diagnostics(h, u0)
    h1, u1 = o.lts(h, u0, 30.0, M, R, n=200, order=order)
    m1, _ = o.diagnostics(h1, u1)
    assert abs(m1 - m0) / m0 < 1e-13


def test_literal_readings_fail_the_pins(igw_case):
    """The printed text of two garbled passages, taken literally, is caught:
    Step 3.3.3 with the coarse dt leaks mass; 2/3 x^{1st} in Steps 3.3.3/4
    breaks the M = 1 identity."""
    m, o, h0, u0, R = igw_case
    rng = np.random.default_rng(3)
    h = h0 + 0.3 * rng.standard_normal(m.nCells)
    m0, _ = o.diagnostics(h, u0)
    with om.reading(1):
        h1, u1 = o.lts(h, u0, 30.0, 4, R, n=5)
    m1, _ = o.diagnostics(h1, u1)
    assert abs(m1 - m0) / m0 > 1e-9
    with om.reading(2):
        h1, u1 = o.lts(h0, u0, 30.0, 1, R, n=1)
    h2, u2 = o.ssprk(h0, u0, 30.0, n=1)
    assert np.abs(h1 - h2).max() > 1e-6
    assert om._load().om_get_reading() == 0


@pytest.mark.parametrize("meshname", ["hex16", "irregular"])
def test_weights_same_in_either_direction(meshname, request):
    """eq:weights may collect V_{i*} clockwise or counter-clockwise: the
    clockwise set is the complement (kite fractions sum to 1 - S) and v* is the
    other end of e (t_{e,v*} flips), so both give the same w_{e,e'}."""
    m = request.getfixturevalue(meshname)
    o = Oracle(m)
    with om.reading(3):
        o3 = Oracle(m)
    for e in range(m.nEdges):
        a, wa = o.weights(e)
        b, wb = o3.weights(e)
        assert np.array_equal(a, b)
        np.testing.assert_allclose(wb, wa, atol=2e-16)


@pytest.mark.parametrize("order,expect", [(3, 3.0), (2, 2.0)])
def test_lts_convergence_order(order, expect):
    """Coarse-step refinement against an RK4 reference at dt = 0.5 s (the
    paper measures LTS against a small-step RK4 reference, Section 3.1)."""
    n, dc = 32, 20e3
    m = periodic_hex_mesh(n, n, dc, f0=1e-4)
    o = Oracle(m)
    p = igw_parameters(m, amp=20.0)
    h0, u0 = igw_state(m, p, 0.0)
    R = o.regions(strip_fine_mask(m, 14, 17, dc), 2, 2)
    T = 1200.0
    hr, ur = o.rk4(h0, u0, 0.5, int(T / 0.5))
    errs = []
    for dtc in (120.0, 60.0, 30.0):
        h, u = o.lts(h0, u0, dtc, 4, R, n=int(T / dtc), order=order)
        errs.append(_rel_l2(h, hr, m.areaCell))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (slopes > expect - 0.25).all(), slopes


def test_lts_step2_ignores_interior_fine_values(igw_case):
    """Only the underlined-F ring is advanced in Step 1; Step 2 on I u C must
    not read the rest of the fine region.  Perturbing X1 on interior fine cells
    and edges leaves R(X1) on I u C bitwise unchanged."""
    m, o, h0, u0, R = igw_case
    dh, du = o.rhs(h0, u0)
    h1 = h0 + 30.0 * dh
    u1 = u0 + 30.0 * du
    a_h, a_u = o.rhs(h1, u1)
    interior_c = (R.cell == om.F) & (R.cell_fbar == 0)
    interior_e = (R.edge == om.F) & (R.edge_fbar == 0)
    h1p, u1p = h1.copy(), u1.copy()
    h1p[interior_c] += 3.0
    u1p[interior_e] -= 0.7
    b_h, b_u = o.rhs(h1p, u1p)
    keep_c = R.cell != om.F
    keep_e = R.edge != om.F
    assert np.array_equal(a_h[keep_c], b_h[keep_c])
    assert np.array_equal(a_u[keep_e], b_u[keep_e])


def test_threaded_timing_build_is_bitwise_identical(irregular):
    """The all-core timing build of the oracle (OpenMP over per-element loops,
    -O3 -march=native, contraction off) computes exactly what the plain build
    computes: each element's operations and their order are unchanged."""
    from paper_2106_07154_amd.inputs import random_state
    m = irregular
    o1 = Oracle(m)
    o4 = Oracle(m, threads=4)
    assert o1.threads == 1 and o4.threads == 4
    h, u = random_state(m, 3, H=100.0, amp_h=1.0, amp_u=0.5)
    fm = (np.arange(m.nCells) % 16 < 5).astype(np.uint8)
    R = o1.regions(fm, 1, 1)
    for fn in (lambda o: o.rhs(h, u), lambda o: o.lts(h, u, 30.0, 4, R, n=2),
               lambda o: o.ssprk(h, u, 20.0, n=2), lambda o: o.rk4(h, u, 20.0, n=2)):
        a, b = fn(o1), fn(o4)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
