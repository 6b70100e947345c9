"""GPU parity of the layered path: L independent layers on one mesh, every
layer against the FP64 oracle run on that layer alone.  Tolerances as in the
single-layer parity tests (1e-12 relative L2 on h in FP64, 1e-11 on u, 1e-5
in FP32); the mass of all layers to 1e-13."""
import math
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2106_07154_amd import lts
from paper_2106_07154_amd.inputs import gaussian_bump_state

pytestmark = pytest.mark.gpu

L = 3


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b, w=None):
    w = np.ones_like(b) if w is None else w
    return math.sqrt((w * (a - b) ** 2).sum() / max((w * b ** 2).sum(), 1e-300))


@pytest.fixture(scope="module")
def case(lloyd_mesh):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m = lloyd_mesh.copy()
    m.bottom = 5.0 * np.random.default_rng(31).standard_normal(m.nCells)
    fm = (np.hypot(m.xCell - 2e5, m.yCell - 2e5) < 5e4).astype(np.uint8)
    o = Oracle(m)
    R = o.regions(fm, 2, 2)
    hs, us = [], []
    for l in range(L):
        # bumps of 10-30 m set up flows of ~0.5 m/s, well above the FP64 floor
        # of u (ulp(g H) dt / d_e per step, see the single-layer tests)
        h, u = gaussian_bump_state(m, 500.0, 10.0 + 10.0 * l, 3.0e4 + 1.0e4 * l, 1.8e5 + 2e4 * l,
                                   2.1e5)
        h, u = o.ssprk(h - m.bottom, u, 30.0, n=8)
        hs.append(h)
        us.append(u)
    dt = 0.3 * 8.0e3 / math.sqrt(9.81 * 510.0) * 4
    return m, fm, o, R, np.array(hs), np.array(us), dt


def _ctx(m, fm, prec):
    c = lts.LTSContext(0, prec, layers=L)
    c.upload_mesh(m, fm, 2, 2)
    return c


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_layers_lts3(case, prec):
    m, fm, o, R, hs, us, dt = case
    say("layers lts3", prec, L)
    c = _ctx(m, fm, prec)
    c.init_state(hs, us)
    c.step(dt, 4, 5)
    gh, gu = c.get_state()
    assert gh.shape == (L, m.nCells) and gu.shape == (L, m.nEdges)
    tol_h, tol_u = (1e-12, 1e-11) if prec == "fp64" else (1e-5, 1e-5)
    mass = 0.0
    for l in range(L):
        rh, ru = o.lts(hs[l], us[l], dt, 4, R, n=5)
        eh, eu = rel_l2(gh[l], rh, m.areaCell), rel_l2(gu[l], ru, m.dvEdge * m.dcEdge)
        say("layer", l, "rel L2 h", eh, "u", eu)
        assert eh < tol_h and eu < tol_u
        mass += o.diagnostics(hs[l], us[l])[0]
    if prec == "fp64":
        d = c.diagnostics()
        assert abs(d.mass - mass) <= 1e-13 * mass
    c.close()


@pytest.mark.parametrize("scheme", ["ssprk3", "rk4", "lts2"])
def test_layers_schemes_fp64(case, scheme):
    m, fm, o, R, hs, us, dt = case
    say("layers", scheme)
    c = _ctx(m, fm, "fp64")
    c.init_state(hs, us)
    if scheme == "lts2":
        c.step_scheme("lts2", dt, 4, 3)
    else:
        c.step_scheme(scheme, dt / 4, 1, 6)
    gh, gu = c.get_state()
    for l in range(L):
        if scheme == "lts2":
            rh, ru = o.lts(hs[l], us[l], dt, 4, R, n=3, order=2)
        elif scheme == "rk4":
            rh, ru = o.rk4(hs[l], us[l], dt / 4, n=6)
        else:
            rh, ru = o.ssprk(hs[l], us[l], dt / 4, n=6)
        assert rel_l2(gh[l], rh, m.areaCell) < 1e-12
        assert rel_l2(gu[l], ru) < 1e-11
    c.close()


def test_layers_rhs_and_identical_layers(case):
    """The right-hand side of every layer, and two identical layers staying
    identical to each other and to the single-layer path."""
    m, fm, o, R, hs, us, dt = case
    say("layers rhs")
    c = _ctx(m, fm, "fp64")
    dh, du = c.eval_rhs(hs.ravel(), us.ravel())
    dh, du = dh.reshape(L, -1), du.reshape(L, -1)
    for l in range(L):
        rh, ru = o.rhs(hs[l], us[l])
        assert rel_l2(dh[l], rh) < 1e-12
        scale = np.abs(ru).max()
        assert np.abs(du[l] - ru).max() <= 1e-11 * scale
    same_h = np.array([hs[1]] * L)
    same_u = np.array([us[1]] * L)
    c.init_state(same_h, same_u)
    c.step(dt, 4, 3)
    gh, gu = c.get_state()
    one = lts.LTSContext(0, "fp64")
    one.upload_mesh(m, fm, 2, 2)
    one.init_state(hs[1], us[1])
    one.step(dt, 4, 3)
    h1, u1 = one.get_state()
    for l in range(L):
        assert np.array_equal(gh[l], gh[0]) and np.array_equal(gu[l], gu[0])
    assert rel_l2(gh[0], h1, m.areaCell) < 1e-13 and rel_l2(gu[0], u1) < 1e-12
    c.close()
    one.close()


@pytest.mark.parametrize("prec,nl", [("fp64", 70), ("fp32", 70), ("fp64", 56), ("fp64", 64)])
def test_many_layers_wave_map(case, prec, nl):
    """From 56 layers on the layered kernels take the wave-per-cell map: 56
    (the first count that does, one ragged chunk), 64 (one full chunk) and
    70 (a full chunk and a ragged chunk of 6).  The three states of the
    fixture repeat over the layers: every layer matches the oracle run of its
    state, and layers with the same state agree bit for bit whatever their
    lane."""
    m, fm, o, R, hs, us, dt = case
    say("many layers", prec, nl)
    c = lts.LTSContext(0, prec, layers=nl)
    c.upload_mesh(m, fm, 2, 2)
    idx = np.arange(nl) % L
    c.init_state(hs[idx], us[idx])
    c.step(dt, 4, 3)
    gh, gu = c.get_state()
    tol_h, tol_u = (1e-12, 1e-11) if prec == "fp64" else (1e-5, 1e-5)
    for k in range(L):
        rh, ru = o.lts(hs[k], us[k], dt, 4, R, n=3)
        ls = np.flatnonzero(idx == k)
        for l in ls:
            assert np.array_equal(gh[l], gh[ls[0]]) and np.array_equal(gu[l], gu[ls[0]])
        eh = rel_l2(gh[ls[0]], rh, m.areaCell)
        eu = rel_l2(gu[ls[0]], ru, m.dvEdge * m.dcEdge)
        say("state", k, "rel L2 h", eh, "u", eu)
        assert eh < tol_h and eu < tol_u
    c.close()
