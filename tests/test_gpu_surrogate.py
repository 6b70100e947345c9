"""GPU checks of the learned fine-region surrogate, through the C ABI, against
the FP64 reference network (oracle/mpnn.py) and the FP64 solver oracle.

Tolerances.  The matrix-core GEMMs take BF16 inputs and accumulate in FP32:
|Y - Y_exact| <= K 2^-24 sum_k |a_k w_k| per entry (held at 4x that).  The
network keeps activations in BF16: every layer output, neighbour mean and
input feature is rounded to 8 significant bits (relative error <= 2^-9).
With 9 such roundings on the forward path, errors of random sign and a
depth-3 ReLU network that roughly preserves relative size, the expected
relative L2 error of the outputs is ~ sqrt(9) 2^-9 / sqrt(3) ~ 3.4e-3; the
bound used is 2e-2.  The backward pass adds a BF16 rounding of every dZ: the
per-block relative L2 error of the gradient is held to 4e-2.  Weights given
to both sides are BF16-representable, so weight rounding is not part of the
error.  Everything that is not network arithmetic (node set, fine edges,
features, the surrogate step's SSPRK3 stages on I u C and its trapezoid
residual) is FP64 in an FP64 context and held to the solver's own 1e-12.
"""
import math
import sys

import numpy as np
import pytest

from oracle import F, I1, I2, Oracle
from oracle import mpnn
from paper_2106_07154_amd import lts
from paper_2106_07154_amd.inputs import gaussian_bump_state, igw_parameters, igw_state, strip_fine_mask

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return math.sqrt(float(np.sum((np.asarray(a, np.float64) - b) ** 2)) /
                     max(float(np.sum(np.asarray(b, np.float64) ** 2)), 1e-300))


def bf16_bits(x):
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)


def bf16_round(x):
    return (bf16_bits(x).astype(np.uint32) << 16).view(np.float32)


@pytest.fixture(scope="module", autouse=True)
def gpu_lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return lts.load_library()


# ------------------------------------------------------------------ GEMMs
@pytest.mark.parametrize("N,K", [(200, 16), (333, 128), (64, 64), (1, 32)])
def test_mfma_gemm_layout(N, K):
    say("gemm", N, K)
    rng = np.random.default_rng(N * 1000 + K)
    A = bf16_round(rng.standard_normal((N, K)))
    W = bf16_round(rng.standard_normal((K, 64)) / math.sqrt(K))
    b = rng.standard_normal(64).astype(np.float32)
    Y = lts.nn_gemm_bf16(bf16_bits(A), bf16_bits(W), b)
    ref = A.astype(np.float64) @ W.astype(np.float64) + b
    bound = 4 * K * 2.0 ** -24 * (np.abs(A).astype(np.float64) @ np.abs(W) + np.abs(b)) + 1e-30
    assert np.all(np.abs(Y - ref) <= bound)


@pytest.mark.parametrize("N,K", [(61419, 128), (333, 16), (0, 32)])
def test_mfma_gemm_device_form(N, K):
    """The device-pointer entry point: its FP32 output equals the host entry
    point's bit for bit (same kernel, same operands) and its BF16 output is
    relu of that value rounded to nearest even; N = 0 writes nothing."""
    import torch
    say("gemm device", N, K)
    rng = np.random.default_rng(N + 7 * K)
    A = bf16_round(rng.standard_normal((N, K)))
    W = bf16_round(rng.standard_normal((K, 64)) / math.sqrt(K))
    b = rng.standard_normal(64).astype(np.float32)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    Yf = torch.full((N, 64), -7.0, dtype=torch.float32, device="cuda")
    Yb = torch.full((N, 64), 12345, dtype=torch.int16, device="cuda")
    s = torch.cuda.Stream()
    lts.nn_gemm_bf16_device(dev(bf16_bits(A).view(np.int16)), dev(bf16_bits(W).view(np.int16)),
                            Y_f32=Yf, Y_bf16=Yb, bias=dev(b), stream=s)
    s.synchronize()
    if N == 0:
        return
    Y = lts.nn_gemm_bf16(bf16_bits(A), bf16_bits(W), b)
    assert np.array_equal(Yf.cpu().numpy(), Y)
    want = bf16_bits(np.maximum(Y, 0.0)).view(np.int16)
    assert np.array_equal(Yb.cpu().numpy(), want)


@pytest.mark.parametrize("N,K", [(1000, 128), (37, 16), (1100, 64)])
def test_mfma_gemm_tn_layout(N, K):
    say("gemm_tn", N, K)
    rng = np.random.default_rng(N + K)
    A = bf16_round(rng.standard_normal((N, K)))
    D = bf16_round(rng.standard_normal((N, 64)))
    P = lts.nn_gemm_tn_bf16(bf16_bits(A), bf16_bits(D))
    ref = A.astype(np.float64).T @ D.astype(np.float64)
    bound = 4 * N * 2.0 ** -24 * (np.abs(A).astype(np.float64).T @ np.abs(D)) + 1e-30
    assert np.all(np.abs(P - ref) <= bound)


# ------------------------------------------------------------ network parity
def _lloyd_case(lloyd_mesh):
    m = lloyd_mesh
    fm = (np.hypot(m.xCell - 2e5, m.yCell - 2e5) < 5e4).astype(np.uint8)
    h, u = gaussian_bump_state(m, 500.0, 5.0, 4.0e4, 2.1e5, 1.9e5)
    return m, fm, h, u


def _test_params(seed):
    rng = np.random.default_rng(seed)
    P = {}
    for name, s in mpnn.param_shapes():
        fan = s[0] if len(s) == 2 else 64
        P[name] = rng.standard_normal(s) * (math.sqrt(2.0 / fan) if len(s) == 2 else 0.1)
    return bf16_round(mpnn.pack(P)).astype(np.float64)


def _norm_from(raw, th, tu):
    mu = raw[:, :5].mean(axis=0)
    sd = raw[:, :5].std(axis=0)
    inv = np.where(sd > 1e-5 * (np.abs(mu) + 1e-30), 1.0 / np.maximum(sd, 1e-300), 0.0)
    rh = math.sqrt(np.mean(th ** 2)) or 1.0
    ru = math.sqrt(np.mean(tu ** 2)) or 1.0
    n = np.zeros(16)
    n[:5], n[5:10], n[10], n[11], n[12], n[13] = mu, inv, 1 / rh, 1 / ru, rh, ru
    return n.astype(np.float32)


@pytest.fixture(scope="module")
def lloyd_setup(lloyd_mesh):
    m, fm, h, u = _lloyd_case(lloyd_mesh)
    o = Oracle(m)
    reg = o.regions(fm, 2, 2)
    ctx = lts.LTSContext(0, "fp64")
    ctx.upload_mesh(m, fm, 2, 2)
    ctx.init_state(h, u)
    sur = lts.Surrogate(ctx, seed=1, max_samples=4)
    nodes, fedges = sur.node_map()
    G = mpnn.build_graph(m, reg, node_order=nodes, edge_order=fedges)
    return dict(m=m, fm=fm, h=h, u=u, o=o, reg=reg, ctx=ctx, sur=sur, G=G)


def test_node_set_and_features(lloyd_setup):
    S = lloyd_setup
    m, reg, sur, G = S["m"], S["reg"], S["sur"], S["G"]
    say("surrogate node set / features", m.nCells)
    nodes, fedges = sur.node_map()
    want = np.flatnonzero((reg.cell == F) | (reg.cell == I1) | (reg.cell == I2))
    assert sorted(nodes.tolist()) == want.tolist()
    assert np.all(reg.cell[nodes[:sur.n_fine_cells]] == F)
    assert np.all(reg.cell[nodes[sur.n_fine_cells:]] != F)
    assert sorted(fedges.tolist()) == np.flatnonzero(reg.edge == F).tolist()
    raw = sur.features()
    ref = mpnn.raw_features(m, S["o"], reg, S["h"], S["u"], nodes)
    for f in range(16):
        scale = max(np.abs(ref[:, f]).max(), 1e-30)
        err = np.abs(raw[:, f] - ref[:, f])
        assert np.all(err <= 2 ** -23 * np.abs(ref[:, f]) + 1e-6 * scale), f


def test_fp32_features_follow_the_state(lloyd_mesh):
    """FP32 contexts store eta = h - href with href taken from the mean
    surface at each lts_init_state: the features must still be those of h
    (feature 0 is h + b, not h + b minus that surface), for two initial
    states whose mean surfaces differ by 30 m."""
    m, fm, h, u = _lloyd_case(lloyd_mesh)
    say("fp32 surrogate features", m.nCells)
    o = Oracle(m)
    reg = o.regions(fm, 2, 2)
    ctx = lts.LTSContext(0, "fp32")
    ctx.upload_mesh(m, fm, 2, 2)
    for shift in (0.0, 30.0):
        ctx.init_state(h + shift, u)
        sur = lts.Surrogate(ctx, seed=1)
        nodes, _ = sur.node_map()
        raw = sur.features()
        ref = mpnn.raw_features(m, o, reg, h + shift, u, nodes)
        for f in range(16):
            scale = max(np.abs(ref[:, f]).max(), 1e-30)
            err = np.abs(raw[:, f] - ref[:, f])
            tol = 2 ** -22 * np.abs(ref[:, f]) + (1e-5 * scale if 2 <= f <= 4 else 0.0)
            say("feature", f, "max err", float(err.max()), "scale", scale)
            assert np.all(err <= tol + 1e-30), (shift, f)
        sur.close()
    ctx.close()


def test_forward_parity(lloyd_setup):
    S = lloyd_setup
    sur, G = S["sur"], S["G"]
    say("surrogate forward parity")
    p = _test_params(11)
    ref_raw = mpnn.raw_features(S["m"], S["o"], S["reg"], S["h"], S["u"], G.nodes)
    norm = _norm_from(ref_raw, np.ones(3), np.ones(3))
    norm[:5] = bf16_round(norm[:5])
    sur.set_params(p.astype(np.float32))
    sur.set_norm(norm)
    oh, ou = sur.predict()
    X = mpnn.normalise(ref_raw, norm.astype(np.float64))
    rh, ru, _ = mpnn.forward(p, G, X)
    say("forward rel L2", rel_l2(oh, rh), rel_l2(ou, ru))
    assert rel_l2(oh, rh) < 2e-2 and rel_l2(ou, ru) < 2e-2


def test_gradient_parity(lloyd_setup):
    S = lloyd_setup
    sur, G, o, ctx = S["sur"], S["G"], S["o"], S["ctx"]
    say("surrogate gradient parity")
    m = S["m"]
    dt = 0.3 * 3.0e3 / math.sqrt(9.81 * 500.0) * 4
    ctx.init_state(S["h"], S["u"])
    sur.record(dt, 4, 1)
    h1, u1 = o.lts(S["h"], S["u"], dt, 4, S["reg"], n=1)
    R0h, R0u = o.rhs(S["h"], S["u"])
    th = (h1 - S["h"] - dt * R0h)[G.nodes[:G.fine]]
    tu = (u1 - S["u"] - dt * R0u)[G.edges]
    ref_raw = mpnn.raw_features(m, o, S["reg"], S["h"], S["u"], G.nodes)
    norm = _norm_from(ref_raw, th, tu)
    p = _test_params(12)
    sur.set_params(p.astype(np.float32))
    sur.set_norm(norm)
    loss, g = sur.grad(0)
    X = mpnn.normalise(ref_raw, norm.astype(np.float64))
    rl, rg = mpnn.loss_and_grad(p, G, X, th * float(norm[10]), tu * float(norm[11]))
    say("loss", loss, rl)
    assert abs(loss - rl) <= 2e-2 * rl
    off = 0
    for name, s in mpnn.param_shapes():
        n = int(np.prod(s))
        e = rel_l2(g[off:off + n], rg[off:off + n])
        say("grad", name, e)
        assert e < 4e-2, name
        off += n


def test_adam_update_matches_oracle(lloyd_setup):
    """Two Adam steps of lts_sur_train against the FP64 Adam of oracle/mpnn.py
    fed the library's own gradients (lts_sur_grad runs the same deterministic
    kernels as the training step) and its FP32 hyperparameters.  Each step
    rounds once to FP32 and carries a few FP32 roundings in its update
    term: |p - p_ref| <= 2^-23 |p_ref| + 1e-5 |p_ref - p_prev| + 1e-12."""
    S = lloyd_setup
    sur, ctx = S["sur"], S["ctx"]
    say("surrogate adam parity")
    if sur.n_samples == 0:
        dt = 0.3 * 3.0e3 / math.sqrt(9.81 * 500.0) * 4
        ctx.init_state(S["h"], S["u"])
        sur.record(dt, 4, 1)
    ref_raw = mpnn.raw_features(S["m"], S["o"], S["reg"], S["h"], S["u"], S["G"].nodes)
    sur.set_norm(_norm_from(ref_raw, np.ones(3), np.ones(3)))
    p0 = _test_params(13).astype(np.float32)
    sur.set_params(p0)                      # also clears the Adam state
    lr = 3e-3
    b1, b2, eps = (float(np.float32(x)) for x in (0.9, 0.999, 1e-8))
    m = v = np.zeros(p0.size)
    prev = p0.astype(np.float64)
    for t in (1, 2):
        _, g = sur.grad(0)
        sur.train(np.array([0], np.int32), lr=lr)
        p = sur.get_params().astype(np.float64)
        want, m, v = mpnn.adam_step(prev, g, m, v, t, float(np.float32(lr)), b1, b2, eps)
        err = np.abs(p - want)
        bound = 2.0 ** -23 * np.abs(want) + 1e-5 * np.abs(want - prev) + 1e-12
        say("adam step", t, "max err/bound", float((err / bound).max()),
            "moved", int(np.count_nonzero(p != prev)))
        assert np.all(err <= bound), t
        prev = p


# --------------------------------------------------------- step and the gate
@pytest.fixture(scope="module")
def igw():
    from paper_2106_07154_amd.inputs.workloads import igw_hex
    return igw_hex()


def _ctx(w, prec="fp64"):
    c = lts.LTSContext(0, prec)
    c.upload_mesh(w.mesh, w.fine_mask, w.n_if1, w.n_if2)
    c.init_state(w.h0, w.u0)
    return c


def surrogate_step_reference(o, reg, A, h0, u0, ph, pu, dt, M):
    """The surrogate coarse step from the oracle's right-hand side, with the
    prediction (ph on F cells, pu on fine edges) given.  I and C follow
    Algorithm 2.2 with the fine substeps replaced by the prediction: Steps 1
    and 2 (coarse stages), the interface accumulation of Step 3 over the 3M
    fine stages with F read linearly in time between x_n and the prediction
    (stage times t_k, t_k + dt/M, t_k + dt/(2M)), interface 1 predicted from
    X0, X1, X2 and I2, C at the coarse stage, then Step 4 on C and Step 5 on
    I.  F takes the prediction, shifted uniformly so that the step changes no
    mass."""
    import oracle as om
    fc, fe = reg.cell == F, reg.edge == F
    ic = (reg.cell == I1) | (reg.cell == I2)
    ie = (reg.edge == I1) | (reg.edge == I2)
    cc, ce = reg.cell == 0, reg.edge == 0
    i1c, i1e = reg.cell == I1, reg.edge == I1
    s1c = ~fc | (reg.cell_fbar != 0)
    s1e = ~fe | (reg.edge_fbar != 0)
    R0 = o.rhs(h0, u0)
    X0 = (h0, u0)
    X1 = (np.where(s1c, h0 + dt * R0[0], h0), np.where(s1e, u0 + dt * R0[1], u0))
    R1 = o.rhs(*X1)
    X2 = (np.where(~fc, 0.75 * h0 + 0.25 * X1[0] + 0.25 * dt * R1[0], h0),
          np.where(~fe, 0.75 * u0 + 0.25 * X1[1] + 0.25 * dt * R1[1], u0))
    X = (X0, X1, X2)
    theta = (1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0)
    acc_h, acc_u = np.zeros_like(h0), np.zeros_like(u0)
    for k in range(M):
        for st in range(3):
            tau = (k + (0.0, 1.0, 0.5)[st]) / M
            cf = om.predict_coeffs(3, st, k, M)
            zh, zu = X[st][0].copy(), X[st][1].copy()
            zh[fc] = h0[fc] + tau * (ph[fc] - h0[fc])
            zu[fe] = u0[fe] + tau * (pu[fe] - u0[fe])
            zh[i1c] = cf[0] * X0[0][i1c] + cf[1] * X1[0][i1c] + cf[2] * X2[0][i1c]
            zu[i1e] = cf[0] * X0[1][i1e] + cf[1] * X1[1][i1e] + cf[2] * X2[1][i1e]
            gh, gu = o.rhs(zh, zu)
            acc_h[ic] += theta[st] * gh[ic]
            acc_u[ie] += theta[st] * gu[ie]
    R2 = o.rhs(*X2)
    nh, nu = h0.copy(), u0.copy()
    nh[ic] = h0[ic] + dt / M * acc_h[ic]
    nu[ie] = u0[ie] + dt / M * acc_u[ie]
    nh[cc] = h0[cc] / 3.0 + 2.0 / 3.0 * X2[0][cc] + 2.0 / 3.0 * dt * R2[0][cc]
    nu[ce] = u0[ce] / 3.0 + 2.0 / 3.0 * X2[1][ce] + 2.0 / 3.0 * dt * R2[1][ce]
    nh[fc], nu[fe] = ph[fc], pu[fe]
    nh[fc] -= np.sum(A * (nh - h0)) / np.sum(A[fc])
    return nh, nu


def test_zero_network_step_matches_oracle(igw):
    """All-zero parameters leave the forward-Euler prediction x_n + dt R(x_n)
    on F; the rest of the step and the gate value r = ||(x_new - x_n)/dt -
    (R(x_n) + R(x_new))/2|| / ((||R(x_n)|| + ||R(x_new)||)/2) on F then follow
    from the oracle's right-hand side (surrogate_step_reference)."""
    w = igw
    say("zero-network surrogate step", w.name)
    c = _ctx(w)
    sur = lts.Surrogate(c, seed=0)
    sur.set_params(np.zeros(sur.n_params, np.float32))
    sur.set_norm(np.array([0] * 5 + [1] * 9 + [0, 0], np.float32))
    acc, res = sur.step(w.dt_coarse, w.M, 1, tau=1e30)
    assert acc == 1
    h, u = c.get_state()
    o = Oracle(w.mesh)
    reg = o.regions(w.fine_mask, w.n_if1, w.n_if2)
    fc, fe = reg.cell == F, reg.edge == F
    x0h, x0u, dt = w.h0, w.u0, w.dt_coarse
    R0 = o.rhs(x0h, x0u)
    ph, pu = x0h + dt * R0[0], x0u + dt * R0[1]      # forward-Euler prediction on F
    nh, nu = surrogate_step_reference(o, reg, w.mesh.areaCell, x0h, x0u, ph, pu, dt, w.M)
    # the u tendency is a difference of g(h + b) ~ gH terms: its FP64 floor
    # is ~1e-12 relative, held at 1e-11 as in the solver's own parity tests
    assert rel_l2(u[fe] - x0u[fe], pu[fe] - x0u[fe]) < 1e-11
    assert rel_l2(h, nh) < 1e-12 and rel_l2(u - x0u, nu - x0u) < 1e-10
    R1 = o.rhs(nh, nu)

    def r(x1, x0, a, b, m):
        d = ((x1 - x0) / dt - 0.5 * (a + b))[m]
        return np.linalg.norm(d) / (0.5 * (np.linalg.norm(a[m]) + np.linalg.norm(b[m])))
    want = max(r(nh, x0h, R0[0], R1[0], fc), r(nu, x0u, R0[1], R1[1], fe))
    say("residual", res[0], want)
    assert abs(res[0] - want) <= 1e-9 * want


def test_surrogate_steps_conserve_mass(igw):
    """Accepted surrogate steps change the total mass by rounding only
    (relative 1e-13 over 20 steps), whatever the network predicts: an
    untrained network with random weights here."""
    w = igw
    say("surrogate mass", w.name)
    c = _ctx(w)
    m0 = c.diagnostics().mass
    sur = lts.Surrogate(c, seed=11)
    # outputs scaled to 1e-3 m and 1e-3 m/s per step
    sur.set_norm(np.array([0] * 5 + [1] * 7 + [1e-3, 1e-3, 0, 0], np.float32))
    acc, res = sur.step(w.dt_coarse, w.M, 20, tau=1e30)
    assert acc == 20 and np.all(np.isfinite(res))
    d = c.diagnostics()
    say("mass drift", abs(d.mass - m0) / m0)
    assert d.n_nonfinite == 0 and abs(d.mass - m0) / m0 < 1e-13


def test_save_and_load_round_trip(igw, tmp_path):
    """lts_sur_save writes shape, normalisation and parameters; lts_sur_load
    into a surrogate on another context restores them bitwise, so both
    predict the same; a truncated file, a file of another kind and a missing
    file are LTS_EINVAL and leave the loaded network as it was."""
    w = igw
    say("surrogate save / load", w.name)
    a, b = _ctx(w), _ctx(w)
    sa, sb = lts.Surrogate(a, seed=5), lts.Surrogate(b, seed=9)
    sa.set_norm(np.array([0.1] * 5 + [1] * 7 + [1e-3, 2e-3, 0, 0], np.float32))
    assert not np.array_equal(sa.get_params(), sb.get_params())
    path = tmp_path / "net.bin"
    sa.save(path)
    sb.load(path)
    assert np.array_equal(sa.get_params(), sb.get_params())
    assert np.array_equal(sa.get_norm(), sb.get_norm())
    pa, pb = sa.predict(), sb.predict()
    assert np.array_equal(pa[0], pb[0]) and np.array_equal(pa[1], pb[1])
    data = path.read_bytes()
    (tmp_path / "short.bin").write_bytes(data[:-4])
    (tmp_path / "long.bin").write_bytes(data + b"\0")
    (tmp_path / "junk.bin").write_bytes(b"x" * len(data))
    for bad in ("short.bin", "long.bin", "junk.bin", "missing.bin"):
        with pytest.raises(lts.LTSError) as ei:
            sb.load(tmp_path / bad)
        assert ei.value.status == lts.LTS_EINVAL, bad
    assert np.array_equal(sa.get_params(), sb.get_params())
    for x in (sa, sb, a, b):
        x.close()


def test_timed_surrogate_step_matches_replayed_graph(igw):
    """In the context's timing mode a surrogate step is launched pass by pass
    with event stamps instead of replaying its graph: the same states and gate
    values bitwise, and five right-hand-side passes per step (R(x_n) and
    R(x_new) on F, Steps 1, 2 and 4) in the kernel statistics."""
    w = igw
    say("surrogate timing mode", w.name)
    a, b = _ctx(w), _ctx(w)
    sa, sb = lts.Surrogate(a, seed=11), lts.Surrogate(b, seed=11)
    norm = np.array([0] * 5 + [1] * 7 + [1e-3, 1e-3, 0, 0], np.float32)
    sa.set_norm(norm)
    sb.set_norm(norm)
    acc_a, ra = sa.step(w.dt_coarse, w.M, 3, tau=1e30)
    b.set_timing(True)
    acc_b, rb = sb.step(w.dt_coarse, w.M, 3, tau=1e30)
    st = b.kernel_stats()
    b.set_timing(False)
    ha, ua = a.get_state()
    hb, ub = b.get_state()
    assert acc_a == acc_b == 3
    assert np.array_equal(ra, rb)
    assert np.array_equal(ha, hb) and np.array_equal(ua, ub)
    for k in ("vertex_pv", "cell_tendency", "edge_tendency"):
        assert st[k]["launches"] == 15 and st[k]["ms"] > 0 and st[k]["bytes"] > 0, (k, st[k])
    sa.close()
    sb.close()
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gate_rejects_fall_back_to_lts3_bitwise(igw, prec):
    w = igw
    say("surrogate fallback", prec)
    a, b = _ctx(w, prec), _ctx(w, prec)
    sur = lts.Surrogate(a, seed=3)
    sur.set_norm(np.array([0] * 5 + [1] * 9 + [0, 0], np.float32))
    acc, res = sur.step(w.dt_coarse, w.M, 3, tau=0.0)     # tau = 0 rejects every step
    assert acc == 0 and res.shape == (3,)
    p = sur.get_params()
    p[-1] = np.nan            # corrupted head bias (ReLU maps a NaN inside the net to 0)
    sur.set_params(p)
    acc2, res2 = sur.step(w.dt_coarse, w.M, 2, tau=1e30)
    assert acc2 == 0 and not np.any(np.isfinite(res2))
    b.step(w.dt_coarse, w.M, 5)
    ha, ua = a.get_state()
    hb, ub = b.get_state()
    assert np.array_equal(ha, hb) and np.array_equal(ua, ub)
    da, db = a.diagnostics(), b.diagnostics()
    assert da.n_nonfinite == 0 and da.steps == db.steps == 5 and da.t == db.t


def test_training_reduces_loss_and_gate_accepts(igw):
    w = igw
    say("surrogate training", w.name)
    c = _ctx(w)
    sur = lts.Surrogate(c, seed=5, max_samples=40)
    sur.record(w.dt_coarse, w.M, 40)
    sur.normalize()
    rng = np.random.default_rng(0)
    idx = rng.integers(0, 32, 600)
    losses = sur.train(idx, lr=2e-3)
    say("loss first/last", losses[:10].mean(), losses[-50:].mean())
    assert np.all(np.isfinite(losses))
    assert losses[-50:].mean() < 0.2 * losses[:10].mean()
    # held-out samples 32..39 are never trained on: their loss stays bounded
    held = [sur.grad(k)[0] for k in range(32, 40)]
    assert np.all(np.isfinite(held))
    # gated steps from the recorded end state: with a loose tau they are kept
    acc, res = sur.step(w.dt_coarse, w.M, 4, tau=1e30)
    assert acc == 4 and np.all(np.isfinite(res))
    d = c.diagnostics()
    assert d.n_nonfinite == 0 and d.steps == 44


def test_trained_network_gains_over_forward_euler(igw):
    """What training buys.  All-zero parameters make the network output zero,
    so the prediction on F is the forward-Euler step x_n + dt R(x_n), the
    method without a learned correction.  From three held-out states (the
    40 recorded LTS3 steps are followed by plain LTS3 steps never trained
    on), one surrogate coarse step with the trained network and one with the
    zero network are each compared with one plain LTS3 step from the same
    state: the trained network's error in the step's height and velocity
    increments, and its gate residual, are smaller on every state."""
    w = igw
    say("surrogate gain over forward Euler", w.name)
    c = _ctx(w)
    sur = lts.Surrogate(c, seed=5, max_samples=40)
    sur.record(w.dt_coarse, w.M, 40)
    sur.normalize()
    sur.train(np.random.default_rng(0).integers(0, 32, 600), lr=2e-3)
    trained = sur.get_params()
    zero = np.zeros(sur.n_params, np.float32)
    rows = []
    for k in range(3):
        c.step(w.dt_coarse, w.M, 1)            # a state no sample was taken from
        h0, u0 = c.get_state()
        c.step(w.dt_coarse, w.M, 1)
        hl, ul = c.get_state()
        got = {}
        for name, p in (("trained", trained), ("zero", zero)):
            sur.set_params(p)
            c.init_state(h0, u0)
            acc, res = sur.step(w.dt_coarse, w.M, 1, tau=1e30)
            assert acc == 1
            h, u = c.get_state()
            got[name] = (rel_l2(h - h0, hl - h0), rel_l2(u - u0, ul - u0), float(res[0]))
        rows.append(got)
        say("state", k, "trained (eh, eu, r)", got["trained"], "zero", got["zero"])
        c.init_state(hl, ul)
    for got in rows:
        for j in range(3):
            assert got["trained"][j] < got["zero"][j], (j, got)


def test_gate_backoff_schedule(igw):
    w = igw
    say("surrogate back-off")
    a, b = _ctx(w), _ctx(w)
    sur = lts.Surrogate(a, seed=4)
    sur.set_norm(np.array([0] * 5 + [1] * 9 + [0, 0], np.float32))
    acc, res = sur.step(w.dt_coarse, w.M, 8, tau=0.0, max_backoff=4)
    assert acc == 0
    assert [k for k in range(8) if res[k] >= 0] == [0, 2, 5]     # skips of 1, 2, 4 steps
    assert np.all(res[[1, 3, 4, 6, 7]] == -1.0)
    b.step(w.dt_coarse, w.M, 8)
    ha, ua = a.get_state()
    hb, ub = b.get_state()
    assert np.array_equal(ha, hb) and np.array_equal(ua, ub)
    assert a.diagnostics().steps == 8
