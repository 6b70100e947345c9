"""GPU parity: liblts (HIP, through the C ABI) against the FP64 oracle.

Tolerances.  FP64: relative L2 per field of 1e-12 for h and for one RHS
evaluation; u after a long run is held to 1e-11 because its tendency is a
difference of g(h+b) ~ gH terms (ulp 1.8e-12), which moves u by ~1.6e-14 m/s
per step under any change of rounding order (the oracle's own M = 1 identity
sits at 1.1e-12 after 200 steps).  FP32: relative L2 of 1e-5 on total h and u.
"""
import math
import sys

import numpy as np
import pytest

import oracle as om
from oracle import Oracle
from paper_2106_07154_amd import lts
from paper_2106_07154_amd.inputs import (gaussian_bump_state, igw_parameters, igw_state,
                                         periodic_hex_mesh, random_state, strip_fine_mask)

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


def make_ctx(mesh, fm, n1=2, n2=2, prec="fp64"):
    c = lts.LTSContext(0, prec)
    c.upload_mesh(mesh, fm, n1, n2)
    return c


def _cases(request):
    m64 = request.getfixturevalue("hex64")
    irr = request.getfixturevalue("irregular")
    ll = request.getfixturevalue("lloyd_mesh")
    return [
        ("hex64-strip", m64, strip_fine_mask(m64, 28, 35, 1e4)),
        ("irregular-disk", irr, (np.hypot(irr.xCell - irr.Lx / 2, irr.yCell - irr.Ly / 2) < 3.5e4).astype(np.uint8)),
        ("lloyd-disk", ll, (np.hypot(ll.xCell - 2e5, ll.yCell - 2e5) < 5e4).astype(np.uint8)),
    ]


def test_rhs_parity_fp64(request):
    for name, m, fm in _cases(request):
        say("rhs fp64", name, m.nCells)
        c = make_ctx(m, fm)
        o = Oracle(m)
        for seed in (1, 2):
            h, u = random_state(m, seed, H=1000.0, amp_h=3.0, amp_u=1.0)
            dh, du = c.eval_rhs(h, u)
            rh, ru = o.rhs(h, u)
            assert rel_l2(dh, rh) < 1e-12, name
            assert rel_l2(du, ru) < 1e-12, name
            assert np.abs(dh - rh).max() <= 1e-10 * np.abs(rh).max()
            assert np.abs(du - ru).max() <= 1e-10 * np.abs(ru).max()
        c.close()


def test_regions_match_oracle(request):
    for name, m, fm in _cases(request):
        say("regions", name)
        c = make_ctx(m, fm)
        cr, er, cf, ef = c.regions()
        R = Oracle(m).regions(fm, 2, 2)
        assert np.array_equal(cr, R.cell) and np.array_equal(er, R.edge)
        assert np.array_equal(cf, R.cell_fbar) and np.array_equal(ef, R.edge_fbar)
        cells, edges, fbar = c.region_counts()
        assert [int(x) for x in cells] == [int((R.cell == k).sum()) for k in range(4)]
        c.close()


@pytest.fixture(scope="module")
def igw(hex64):
    p = igw_parameters(hex64)
    h0, u0 = igw_state(hex64, p, 0.0)
    fm = strip_fine_mask(hex64, 28, 35, 1e4)
    o = Oracle(hex64)
    R = o.regions(fm, 2, 2)
    return hex64, fm, o, R, h0, u0


def test_lts3_igw_full_run_fp64(igw):
    """The 64x64 inertia-gravity-wave workload: 200 coarse steps, M = 4."""
    m, fm, o, R, h0, u0 = igw
    say("lts3 igw 200 steps fp64")
    c = make_ctx(m, fm)
    c.init_state(h0, u0)
    c.step(30.0, 4, 200)
    h, u = c.get_state()
    rh, ru = o.lts(h0, u0, 30.0, 4, R, n=200)
    assert rel_l2(h, rh, m.areaCell) < 1e-12
    assert rel_l2(u, ru, m.dvEdge * m.dcEdge) < 1e-11
    # also against the perturbation, element by element
    assert np.abs(h - rh).max() < 1e-9
    assert np.abs(u - ru).max() < 1e-11
    d = c.diagnostics()
    assert d.steps == 200 and abs(d.t - 6000.0) < 1e-9
    c.close()


@pytest.mark.parametrize("M", [1, 2, 3, 8])
def test_lts3_short_runs_fp64(igw, M):
    m, fm, o, R, h0, u0 = igw
    say("lts3 short", M)
    rng = np.random.default_rng(M)
    h = h0 + 0.2 * rng.standard_normal(m.nCells)
    u = u0 + 0.05 * rng.standard_normal(m.nEdges)
    c = make_ctx(m, fm)
    c.init_state(h, u)
    c.step(30.0, M, 5)
    gh, gu = c.get_state()
    rh, ru = o.lts(h, u, 30.0, M, R, n=5)
    assert rel_l2(gh, rh, m.areaCell) < 1e-12
    assert rel_l2(gu, ru) < 1e-12
    c.close()


def test_rk3_parity_and_m1_identity(igw):
    m, fm, o, R, h0, u0 = igw
    say("rk3 vs oracle, lts3 M=1 vs rk3")
    c = make_ctx(m, fm)
    c.init_state(h0, u0)
    c.step_rk3(30.0, 50)
    h, u = c.get_state()
    rh, ru = o.ssprk(h0, u0, 30.0, n=50)
    assert rel_l2(h, rh, m.areaCell) < 1e-12
    assert rel_l2(u, ru) < 1e-11
    c2 = make_ctx(m, fm)
    c2.init_state(h0, u0)
    c2.step(30.0, 1, 50)
    h2, u2 = c2.get_state()
    assert rel_l2(h2, h, m.areaCell) < 1e-12
    assert rel_l2(u2, u) < 1e-11
    c.close()
    c2.close()


@pytest.mark.parametrize("M", [4, 8])
def test_mass_conservation_gpu(igw, M):
    m, fm, o, R, h0, u0 = igw
    say("mass", M)
    rng = np.random.default_rng(5)
    h = h0 + 0.3 * rng.standard_normal(m.nCells)
    c = make_ctx(m, fm)
    c.init_state(h, u0)
    d0 = c.diagnostics()
    om0, oe0 = o.diagnostics(h, u0)
    assert abs(d0.mass - om0) / om0 < 1e-14
    assert abs(d0.energy - oe0) / oe0 < 1e-13
    c.step(30.0, M, 200)
    d1 = c.diagnostics()
    assert abs(d1.mass - d0.mass) / d0.mass < 1e-13
    c.close()


def test_irregular_meshes_lts3_fp64(request):
    for name, m, fm in _cases(request)[1:]:
        for n1, n2 in ((2, 2), (1, 1)):
            say("lts3 irregular", name, n1, n2)
            o = Oracle(m)
            R = o.regions(fm, n1, n2)
            h, u = gaussian_bump_state(m, 500.0, 5.0, 3 * m.dcEdge.min(),
                                       m.xCell[np.argmax(fm)], m.yCell[np.argmax(fm)])
            dt = 0.2 * m.dcEdge.min() / math.sqrt(9.81 * 500.0) * 4
            c = make_ctx(m, fm, n1, n2)
            c.init_state(h, u)
            c.step(dt, 4, 10)
            gh, gu = c.get_state()
            rh, ru = o.lts(h, u, dt, 4, R, n=10)
            assert rel_l2(gh, rh, m.areaCell) < 1e-12, name
            assert rel_l2(gu, ru) < 1e-11, name
            c.close()


def test_determinism_and_step_splitting(igw):
    m, fm, o, R, h0, u0 = igw
    say("determinism")
    outs = []
    for split in ((20,), (7, 13)):
        c = make_ctx(m, fm)
        c.init_state(h0, u0)
        for n in split:
            c.step(30.0, 4, n)
        outs.append(c.get_state())
        c.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_checkpoint_restart(igw):
    """Stopping after 7 steps, reading the state back and restarting in a new
    context reproduces the uninterrupted 20-step run: bitwise in FP64; in FP32
    the restart re-derives the reference surface, so within 1e-6."""
    m, fm, o, R, h0, u0 = igw
    say("checkpoint restart")
    for prec in ("fp64", "fp32"):
        a = make_ctx(m, fm, prec=prec)
        a.init_state(h0, u0)
        a.step(30.0, 4, 20)
        ha, ua = a.get_state()
        b = make_ctx(m, fm, prec=prec)
        b.init_state(h0, u0)
        b.step(30.0, 4, 7)
        hc, uc = b.get_state()
        b.close()
        c = make_ctx(m, fm, prec=prec)
        c.init_state(hc, uc, t0=7 * 30.0)
        c.step(30.0, 4, 13)
        hb, ub = c.get_state()
        d = c.diagnostics()
        assert abs(d.t - 600.0) < 1e-9 and d.steps == 13
        if prec == "fp64":
            assert np.array_equal(ha, hb) and np.array_equal(ua, ub)
        else:
            assert rel_l2(hb, ha) < 1e-6 and rel_l2(ub, ua) < 1e-5
        a.close(), c.close()


def test_edge_cases(hex8):
    say("edge cases")
    m = periodic_hex_mesh(30, 18, 1e4, f0=1e-4)  # 540 cells: ragged vs 256-thread blocks
    o = Oracle(m)
    h, u = random_state(m, 3, amp_h=0.5, amp_u=0.1)
    for fm, n1, n2 in ((strip_fine_mask(m, 8, 8, 1e4), 1, 1),
                       (np.eye(1, m.nCells, 270, dtype=np.uint8)[0], 2, 2)):
        R = o.regions(fm, n1, n2)
        c = make_ctx(m, fm, n1, n2)
        c.init_state(h, u)
        c.step(30.0, 3, 0)  # no-op
        gh, gu = c.get_state()
        assert np.array_equal(gh, h) and np.array_equal(gu, u)
        c.step(30.0, 3, 4)
        gh, gu = c.get_state()
        rh, ru = o.lts(h, u, 30.0, 3, R, n=4)
        assert rel_l2(gh, rh) < 1e-12 and rel_l2(gu, ru) < 1e-12
        c.close()
    c = make_ctx(m, strip_fine_mask(m, 8, 9, 1e4))
    with pytest.raises(lts.LTSError) as ei:
        c.step(30.0, 4, 1)
    assert ei.value.status == lts.LTS_ESTATE
    c.init_state(h, u)
    for bad in ((0.0, 4), (-1.0, 4), (30.0, 0)):
        with pytest.raises(lts.LTSError) as ei:
            c.step(bad[0], bad[1], 1)
        assert ei.value.status == lts.LTS_EINVAL
    c.close()


def test_nonfinite_is_sticky_until_init(igw):
    m, fm, o, R, h0, u0 = igw
    say("nonfinite")
    c = make_ctx(m, fm)
    c.init_state(h0, u0)
    c.step(3000.0, 1, 40)  # far beyond the CFL limit
    st, d = c.diagnostics_status()
    assert st == lts.LTS_ENONFINITE
    with pytest.raises(lts.LTSError) as ei:
        c.step(30.0, 4, 1)
    assert ei.value.status == lts.LTS_ENONFINITE
    c.init_state(h0, u0)
    d = c.diagnostics()
    assert d.n_nonfinite == 0
    c.close()


def test_device_state_roundtrip(igw):
    import torch
    m, fm, o, R, h0, u0 = igw
    say("device state roundtrip")
    c = make_ctx(m, fm)
    th = torch.tensor(h0, device="cuda", dtype=torch.float64)
    tu = torch.tensor(u0, device="cuda", dtype=torch.float64)
    c.init_state_device(th, tu)
    h, u = c.get_state()
    assert np.array_equal(h, h0) and np.array_equal(u, u0)
    oh = torch.empty_like(th)
    ou = torch.empty_like(tu)
    c.step(30.0, 4, 3)
    c.get_state_device(oh, ou)
    h, u = c.get_state()
    assert np.array_equal(oh.cpu().numpy(), h) and np.array_equal(ou.cpu().numpy(), u)
    c.close()


def test_lts3_fp32_parity(igw):
    """FP32 state and tendencies, FP64 prediction coefficients and sums:
    relative L2 within 1e-5 on total h and u against the FP64 oracle."""
    m, fm, o, R, h0, u0 = igw
    say("lts3 fp32 200 steps")
    c = make_ctx(m, fm, prec="fp32")
    c.init_state(h0, u0)
    c.step(30.0, 4, 200)
    h, u = c.get_state()
    rh, ru = o.lts(h0, u0, 30.0, 4, R, n=200)
    eh = rel_l2(h, rh, m.areaCell)
    eu = rel_l2(u, ru, m.dvEdge * m.dcEdge)
    say("fp32 errors", eh, eu, "perturbation-relative",
        rel_l2(h - 1000.0, rh - 1000.0, m.areaCell))
    assert eh < 1e-5 and eu < 1e-5
    c.close()


@pytest.mark.parametrize("scheme", ["lts3", "ssprk3"])
def test_fp32_stage_updates_do_not_drift(igw, scheme):
    """FP32 against FP64 on the GPU over 200 coarse steps (800 fine steps) of
    the IGW, relative to the perturbation: rounding level (measured 4.7e-7
    for LTS3 and 1.0e-6 for SSPRK3).  Evaluating x_old/3 + 2 x_cur/3 with the
    FP32-rounded weights, whose sum is 1 + 3.0e-8, would scale the state by
    that factor every fine step: a drift of 2.4e-5 over this run."""
    m, fm, o, R, h0, u0 = igw
    say("fp32 drift", scheme)
    out = {}
    for prec in ("fp64", "fp32"):
        c = make_ctx(m, fm, prec=prec)
        c.init_state(h0, u0)
        if scheme == "lts3":
            c.step(30.0, 4, 200)
        else:
            c.step_rk3(7.5, 800)
        out[prec] = c.get_state()
        c.close()
    (h64, u64), (h32, u32) = out["fp64"], out["fp32"]
    eh = rel_l2(h32 - 1000.0, h64 - 1000.0)
    eu = rel_l2(u32, u64)
    say("fp32 - fp64", scheme, eh, eu)
    assert eh < 5e-6 and eu < 5e-6


def test_rhs_parity_fp32(request):
    for name, m, fm in _cases(request):
        say("rhs fp32", name)
        c = make_ctx(m, fm, prec="fp32")
        h, u = random_state(m, 4, H=1000.0, amp_h=3.0, amp_u=1.0)
        c.init_state(h, u)  # sets the thickness reference of the perturbation form
        dh, du = c.eval_rhs(h, u)
        rh, ru = Oracle(m).rhs(h, u)
        assert rel_l2(dh, rh) < 1e-5 and rel_l2(du, ru) < 1e-5, name
        c.close()


@pytest.mark.parametrize("scheme,M,n", [("lts2", 4, 20), ("lts2", 1, 10), ("ssprk2", 1, 10),
                                        ("rk4", 1, 20), ("lts3", 4, 10)])
def test_scheme_parity(igw, scheme, M, n):
    """Every scheme of lts_step_scheme against the oracle's implementation."""
    m, fm, o, R, h0, u0 = igw
    say("scheme", scheme, M, n)
    rng = np.random.default_rng(11)
    h = h0 + 0.2 * rng.standard_normal(m.nCells)
    c = make_ctx(m, fm)
    c.init_state(h, u0)
    c.step_scheme(scheme, 30.0, M, n)
    gh, gu = c.get_state()
    if scheme == "lts2":
        rh, ru = o.lts(h, u0, 30.0, M, R, n=n, order=2)
    elif scheme == "lts3":
        rh, ru = o.lts(h, u0, 30.0, M, R, n=n, order=3)
    elif scheme == "ssprk2":
        rh, ru = o.ssprk(h, u0, 30.0, n=n, order=2)
    else:
        rh, ru = o.rk4(h, u0, 30.0, n=n)
    assert rel_l2(gh, rh, m.areaCell) < 1e-12
    assert rel_l2(gu, ru) < 1e-11
    if scheme in ("lts2", "lts3"):
        d0m, _ = o.diagnostics(h, u0)
        assert abs(c.diagnostics().mass - d0m) / d0m < 1e-13
    c.close()
