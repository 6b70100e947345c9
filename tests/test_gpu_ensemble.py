"""GPU ensemble: members of all three size classes advanced together in batched
launches must reproduce each member advanced alone through lts_step (same
kernel bodies), and the oracle."""
import math
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2106_07154_amd import lts
from paper_2106_07154_amd.inputs import gaussian_bump_state, periodic_hex_mesh, random_state
from paper_2106_07154_amd.inputs.cases import disk_fine_mask

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return math.sqrt(((a - b) ** 2).sum() / max((b ** 2).sum(), 1e-300))


@pytest.fixture(scope="module")
def members(hex64, irregular, lloyd_mesh):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = []
    for m, M, frac in ((hex64, 4, 0.15), (irregular, 2, 0.2), (lloyd_mesh, 8, 0.12),
                       (periodic_hex_mesh(200, 160, 5e3, f0=1e-4), 2, 0.1),
                       (periodic_hex_mesh(400, 320, 2.5e3, f0=1e-4), 8, 0.1)):
        cx, cy = m.Lx / 2, m.Ly / 2
        fm = disk_fine_mask(m, cx, cy, frac * m.Lx)
        h, u = gaussian_bump_state(m, 500.0, 3.0, 0.1 * m.Lx, cx, cy)
        h2, u2 = random_state(m, 5, H=0.0, amp_h=0.05, amp_u=0.02)
        h, u = h + h2, u + u2
        dt = 0.3 * m.dcEdge.min() / math.sqrt(9.81 * 500.0)  # coarse Courant 0.3
        out.append((m, fm, h, u, dt, M))
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ensemble_matches_members_alone(members, prec):
    say("ensemble", prec, [m.nCells for m, *_ in members])
    ens = lts.Ensemble(0, prec)
    for m, fm, h, u, dt, M in members:
        ens.add_member(m, fm, dt, M)
    for j, (m, fm, h, u, dt, M) in enumerate(members):
        ens.init_member(j, h, u)
    ens.build(autotune=True)
    info = ens.info()
    say("ensemble info", info)
    assert all(c > 0 for c in info["class_cells"])
    ens.step(4)
    tol = 1e-14 if prec == "fp64" else 1e-6
    for j, (m, fm, h, u, dt, M) in enumerate(members):
        gh, gu = ens.get_member(j)
        c = lts.LTSContext(0, prec)
        c.upload_mesh(m, fm, 2, 2)
        c.init_state(h, u)
        c.step(dt, M, 4)
        rh, ru = c.get_state()
        c.close()
        say("member", j, m.nCells, "bitwise", np.array_equal(gh, rh) and np.array_equal(gu, ru))
        assert rel_l2(gh, rh) <= tol and rel_l2(gu, ru) <= tol * 10
        d = ens.diagnostics(j)
        assert d.steps == 4 and d.n_nonfinite == 0
    # every member against the FP64 oracle (h and u)
    tol_h, tol_u = (1e-12, 1e-11) if prec == "fp64" else (1e-5, 1e-5)
    for j, (m, fm, h, u, dt, M) in enumerate(members):
        o = Oracle(m)
        rh, ru = o.lts(h, u, dt, M, o.regions(fm, 2, 2), n=4)
        gh, gu = ens.get_member(j)
        eh, eu = rel_l2(gh, rh), rel_l2(gu, ru)
        say("member", j, m.nCells, "M", M, "oracle rel L2 h", eh, "u", eu)
        assert eh < tol_h and eu < tol_u, j
    ens.close()


def test_ensemble_errors(hex8):
    ens = lts.Ensemble(0, "fp64")
    with pytest.raises(lts.LTSError) as ei:
        ens.step(1)
    assert ei.value.status == lts.LTS_ESTATE
    with pytest.raises(lts.LTSError) as ei:
        ens.build()
    assert ei.value.status == lts.LTS_ESTATE
    ens.close()


@pytest.fixture(scope="module")
def config4_members():
    """Six members of the 64-member ensemble workload, built by its own
    generator (seed 7000 + j) from the cached relaxed points: two of each size
    class (< 30k, < 120k, larger), one of 352k cells, M in {2, 4, 8}."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_07154_amd.inputs import workloads
    sizes = workloads.ensemble_sizes(64)
    return [workloads.ensemble_member(j, int(sizes[j])) for j in workloads.ENS_CACHED]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config4_members_match_oracle(config4_members, prec):
    ws = config4_members
    say("config-4 members", prec, [(w.name, w.mesh.nCells, w.M) for w in ws])
    assert {w.M for w in ws} == {2, 4, 8}
    n = [w.mesh.nCells for w in ws]
    assert min(n) < 30_000 and any(30_000 <= x < 120_000 for x in n) and max(n) >= 300_000
    ens = lts.Ensemble(0, prec)
    for w in ws:
        ens.add_member(w.mesh, w.fine_mask, w.dt_coarse, w.M, w.n_if1, w.n_if2, w.gravity)
    for j, w in enumerate(ws):
        ens.init_member(j, w.h0, w.u0)
    ens.build(autotune=False)
    ens.step(2)
    tol_h, tol_u = (1e-12, 1e-11) if prec == "fp64" else (1e-5, 1e-5)
    for j, w in enumerate(ws):
        m = w.mesh
        o = Oracle(m, w.gravity)
        rh, ru = o.lts(w.h0, w.u0, w.dt_coarse, w.M, o.regions(w.fine_mask, w.n_if1, w.n_if2),
                       n=2)
        gh, gu = ens.get_member(j)
        eh = math.sqrt((m.areaCell * (gh - rh) ** 2).sum() / (m.areaCell * rh ** 2).sum())
        eu = rel_l2(gu, ru)
        ep = math.sqrt((m.areaCell * (gh - rh) ** 2).sum() /
                       (m.areaCell * (rh - w.extra["H"]) ** 2).sum())
        say(w.name, m.nCells, "M", w.M, "rel L2 h", eh, "u", eu, "h - H", ep)
        assert eh < tol_h and eu < tol_u, w.name
        d = ens.diagnostics(j)
        assert d.steps == 2 and d.n_nonfinite == 0
    ens.close()


def test_batched_ssprk3_and_kernel_stats(members):
    """The ensemble's SSPRK3 mode (M_j steps of dt_j / M_j per ensemble step,
    the same batched work lists) equals each member's own SSPRK3 in FP64 to
    1e-14 and the FP64 oracle to 1e-12 (h) / 1e-11 (u); the event-stamped
    timing mode advances the members like lts_ens_step and reports every
    launch with its algorithmic bytes."""
    say("ensemble ssprk3 + kernel stats")
    ens = lts.Ensemble(0, "fp64")
    for m, fm, h, u, dt, M in members:
        ens.add_member(m, fm, dt, M)
    for j, (m, fm, h, u, dt, M) in enumerate(members):
        ens.init_member(j, h, u)
    dts = np.array([dt for *_, dt, M in members]) * 0.75
    ens.set_scheme("ssprk3", dts)
    ens.build(autotune=False)
    ens.step(2)
    for j, (m, fm, h, u, dt, M) in enumerate(members):
        gh, gu = ens.get_member(j)
        c = lts.LTSContext(0, "fp64")
        c.upload_mesh(m, fm, 2, 2)
        c.init_state(h, u)
        c.step_rk3(dts[j] / M, 2 * M)
        rh, ru = c.get_state()
        c.close()
        assert rel_l2(gh, rh) <= 1e-14 and rel_l2(gu, ru) <= 1e-13, j
        if m.nCells <= 20000:
            oh, ou = Oracle(m).ssprk(h, u, dts[j] / M, n=2 * M)
            assert rel_l2(gh, oh) < 1e-12 and rel_l2(gu, ou) < 1e-11, j
        assert ens.diagnostics(j).steps == 2
    # timing mode: same result as graph replay, every launch counted
    info = ens.info()
    for j, (m, fm, h, u, dt, M) in enumerate(members):
        ens.init_member(j, h, u)
    st = ens.kernel_stats(2)
    assert sum(v["launches"] for v in st.values()) == 2 * info["launches_per_step"]
    for k, v in st.items():
        assert v["launches"] > 0 and v["ms"] > 0, k
        assert abs(v["bytes"] - 2 * info["step_bytes"][k]) <= 1e-6 * v["bytes"], k
    for j, (m, fm, h, u, dt, M) in enumerate(members):
        gh, gu = ens.get_member(j)
        c = lts.LTSContext(0, "fp64")
        c.upload_mesh(m, fm, 2, 2)
        c.init_state(h, u)
        c.step_rk3(dts[j] / M, 2 * M)
        rh, ru = c.get_state()
        c.close()
        assert np.array_equal(gh, rh) or rel_l2(gh, rh) <= 1e-14, j
    # back to LTS3 at the original steps, keeping the tuning
    for j, (m, fm, h, u, dt, M) in enumerate(members):
        ens.init_member(j, h, u)
    ens.set_scheme("lts3", np.array([dt for *_, dt, M in members]))
    ens.build(autotune=False)
    ens.step(1)
    m, fm, h, u, dt, M = members[0]
    gh, gu = ens.get_member(0)
    o = Oracle(m)
    rh, ru = o.lts(h, u, dt, M, o.regions(fm, 2, 2), n=1)
    assert rel_l2(gh, rh) < 1e-12 and rel_l2(gu, ru) < 1e-11
    ens.close()


def _ensemble(members, prec, fused, spin_limit=0):
    ens = lts.Ensemble(0, prec)
    for m, fm, h, u, dt, M in members:
        ens.add_member(m, fm, dt, M)
    for j, (m, fm, h, u, dt, M) in enumerate(members):
        ens.init_member(j, h, u)
    if fused:
        ens.set_fused(True, spin_limit)
    ens.build(autotune=False)
    return ens


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fused_step_matches_batched_launches(members, prec):
    """One persistent fused kernel per ensemble step (grid barriers between
    the vertex, cell and edge work of each phase) computes every element with
    the arithmetic of the batched launches: bitwise equal members, and each
    step is one launch."""
    say("fused ensemble", prec)
    a = _ensemble(members, prec, True)
    b = _ensemble(members, prec, False)
    a.step(3)
    b.step(3)
    for j in range(len(members)):
        ha, ua = a.get_member(j)
        hb, ub = b.get_member(j)
        assert np.array_equal(ha, hb) and np.array_equal(ua, ub), j
        assert a.diagnostics(j).steps == 3
    st = a.kernel_stats(2)
    assert st["cell_tendency"]["launches"] == 2 and st["vertex_pv"]["launches"] == 0
    assert st["cell_tendency"]["ms"] > 0
    a.close()
    b.close()


def test_fused_barrier_that_gives_up_is_an_error(members):
    """A grid-barrier wait bounded to one poll runs out (forced from the
    host): every block leaves the kernel, the step reports LTS_EDEVICE, and
    after re-initialisation the default bound steps normally again."""
    say("fused ensemble forced barrier timeout")
    a = _ensemble(members, "fp64", True, spin_limit=1)
    with pytest.raises(lts.LTSError) as ei:
        a.step(1)
    assert ei.value.status == lts.LTS_EDEVICE
    with pytest.raises(lts.LTSError):
        a.step(1)                      # states undefined until re-initialised
    a.set_fused(True, 0)
    for j, (m, fm, h, u, dt, M) in enumerate(members):
        a.init_member(j, h, u)
    a.build(autotune=False)
    a.step(2)
    b = _ensemble(members, "fp64", False)
    b.step(2)
    for j in range(len(members)):
        ha, ua = a.get_member(j)
        hb, ub = b.get_member(j)
        assert np.array_equal(ha, hb) and np.array_equal(ua, ub), j
    a.close()
    b.close()
