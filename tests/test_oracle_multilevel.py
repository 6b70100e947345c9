"""Pins on the oracle's multi-level LTS3 (Remark 3.1: more than two LTS
regions, an integer step ratio between neighbouring levels).

The scheme is this build's reading of the remark (the paper gives no
algorithm): each fine substep of level l is an LTS3 step of level l+1 on
level l's fine region, and that step's coarse-stage evaluations supply level
l's interface accumulation.  Anchors that do not depend on the reading being
right, only on it being consistent:

* two levels are exactly Algorithm 2.2 (bitwise the two-level oracle);
* an inner ratio of 1 makes the inner LTS3 step an SSPRK3 step (Remark 2.3),
  so three levels equal two to rounding;
* all ratios 1 give global SSPRK3 to rounding;
* exact discrete mass conservation over 200 coarse steps;
* third-order convergence against a small-step RK4 reference;
* labels refuse inner regions that reach within two rings of the enclosing
  interface.
"""
import math

import numpy as np
import pytest

from oracle import Oracle
from paper_2106_07154_amd.inputs import (igw_parameters, igw_state, periodic_hex_mesh,
                                         strip_fine_mask)


def _rel_l2(a, b, w=None):
    w = np.ones_like(a) if w is None else w
    return math.sqrt((w * (a - b) ** 2).sum() / (w * b ** 2).sum())


@pytest.fixture(scope="module")
def nested():
    """32 x 32 periodic hexagonal mesh (dc = 20 km), inertia-gravity wave of
    20 m; level-0 fine strip of rows 6-25, level-1 fine strip of rows 14-17
    (its 2 + 2 interface rings reach rows 10-21, three rows inside the outer
    strip)."""
    n, dc = 32, 20e3
    m = periodic_hex_mesh(n, n, dc, f0=1e-4)
    o = Oracle(m)
    p = igw_parameters(m, amp=20.0)
    h0, u0 = igw_state(m, p, 0.0)
    masks = [strip_fine_mask(m, 6, 25, dc), strip_fine_mask(m, 14, 17, dc)]
    R = o.ml_regions(masks, 2, 2)
    return m, o, h0, u0, masks, R


def test_region_labels_nest(nested):
    m, o, h0, u0, masks, R = nested
    assert R.cell.shape == (2, m.nCells)
    # each level's labels are those of the two-level labelling of its mask
    for l in range(2):
        r = o.regions(masks[l], 2, 2)
        assert np.array_equal(R.cell[l], r.cell) and np.array_equal(R.edge[l], r.edge)
        assert np.array_equal(R.cell_fbar[l], r.cell_fbar)
    # level 1's fine and interface cells are fine cells of level 0
    inner = R.cell[1] != 0
    assert np.all(R.cell[0][inner] == 3)
    # the underlined-F rings of level 0 are coarse at level 1
    assert np.all(R.cell[1][R.cell_fbar[0] != 0] == 0)


def test_nesting_too_close_is_rejected(nested):
    m, o, h0, u0, masks, R = nested
    dc = 20e3
    # inner strip rows 10-21: its interface rings reach rows 6-9 and 22-25,
    # within two rings of the outer interface
    with pytest.raises(ValueError):
        o.ml_regions([masks[0], strip_fine_mask(m, 10, 21, dc)], 2, 2)
    # an inner region outside the outer fine region
    with pytest.raises(ValueError):
        o.ml_regions([masks[0], strip_fine_mask(m, 28, 30, dc)], 2, 2)


def test_two_levels_are_algorithm_2_2_bitwise(nested):
    m, o, h0, u0, masks, R = nested
    R2 = o.ml_regions(masks[:1], 2, 2)
    r = o.regions(masks[0], 2, 2)
    a = o.mlts(h0, u0, 60.0, [4], R2, n=3)
    b = o.lts(h0, u0, 60.0, 4, r, n=3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_inner_ratio_one_equals_two_levels(nested):
    """With M = 1 at the inner level the inner LTS3 step is SSPRK3 (Remark
    2.3): the three-level step equals the two-level one up to rounding (the
    inner interface correction is the Butcher form of the same stages)."""
    m, o, h0, u0, masks, R = nested
    r = o.regions(masks[0], 2, 2)
    a = o.mlts(h0, u0, 60.0, [3, 1], R, n=20)
    b = o.lts(h0, u0, 60.0, 3, r, n=20)
    assert _rel_l2(a[0], b[0], m.areaCell) < 1e-13
    assert _rel_l2(a[1], b[1], m.dvEdge * m.dcEdge) < 1e-11


def test_all_ratios_one_equal_ssprk3(nested):
    m, o, h0, u0, masks, R = nested
    a = o.mlts(h0, u0, 60.0, [1, 1], R, n=20)
    b = o.ssprk(h0, u0, 60.0, n=20)
    assert _rel_l2(a[0], b[0], m.areaCell) < 1e-13
    assert _rel_l2(a[1], b[1], m.dvEdge * m.dcEdge) < 1e-11


@pytest.mark.parametrize("Ms", [(2, 3), (3, 2)])
def test_multilevel_conserves_mass(nested, Ms):
    """Relative mass drift below 1e-13 over 200 coarse steps: each level's
    interface correction uses the same fluxes as the coarse stages of the
    level inside it."""
    m, o, h0, u0, masks, R = nested
    rng = np.random.default_rng(5)
    h = h0 + 0.3 * rng.standard_normal(m.nCells)
    m0, _ = o.diagnostics(h, u0)
    h1, u1 = o.mlts(h, u0, 60.0, list(Ms), R, n=200)
    m1, _ = o.diagnostics(h1, u1)
    assert np.all(np.isfinite(h1))
    assert abs(m1 - m0) / m0 < 1e-13


def test_inner_level_changes_the_inner_region(nested):
    """The inner ratio acts: M = (2, 2) and M = (2, 1) differ, and mostly
    inside the inner fine region (where the step is halved)."""
    m, o, h0, u0, masks, R = nested
    a = o.mlts(h0, u0, 60.0, [2, 2], R, n=5)
    b = o.mlts(h0, u0, 60.0, [2, 1], R, n=5)
    d = np.abs(a[0] - b[0])
    assert d.max() > 1e-9
    assert d[R.cell[1] != 0].max() >= d.max() * 0.5


def test_multilevel_third_order(nested):
    """Coarse-step refinement against an RK4 reference at dt = 0.5 s, as the
    two-level convergence pin."""
    m, o, h0, u0, masks, R = nested
    T = 1200.0
    hr, ur = o.rk4(h0, u0, 0.5, int(T / 0.5))
    errs = []
    for dtc in (120.0, 60.0, 30.0):
        h, u = o.mlts(h0, u0, dtc, [2, 2], R, n=int(T / dtc))
        errs.append(_rel_l2(h, hr, m.areaCell))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (slopes > 2.75).all(), (errs, slopes)
