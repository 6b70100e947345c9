"""Pins of the FP64 surrogate reference (oracle/mpnn.py) against what
mathematics fixes independently of its own formulas:

* the hand-written gradient against central finite differences of the loss;
* the neighbour mean against a brute-force scan of the edge list, and its
  transpose against the adjoint identity <mean(A), B> = <A, mean^T(B)>;
* equivariance of the outputs under a relabelling of nodes and edges, and
  the sign flip of the edge head under a reversed edge orientation;
* the divergence and vorticity features against the closed form of the
  linear inertia-gravity wave (div u = -(A w / H) sin phi, zeta = (A f / H)
  cos phi, the wave has no potential-vorticity anomaly), converging at
  second order on the hexagonal mesh, and their exact telescoping sums on a
  periodic irregular mesh.
"""
import numpy as np
import pytest

from oracle import F, I1, I2, Oracle
from oracle import mpnn
from paper_2106_07154_amd.inputs import periodic_hex_mesh
from paper_2106_07154_amd.inputs.cases import igw_parameters, igw_state, strip_fine_mask


def _graph(mesh, rows=(3, 4)):
    o = Oracle(mesh)
    fm = strip_fine_mask(mesh, rows[0], rows[1], 1.0e4)
    reg = o.regions(fm, 1, 1)
    return o, reg, mpnn.build_graph(mesh, reg)


def _random_params(rng, scale=1.0):
    P = {}
    for name, s in mpnn.param_shapes():
        fan = s[0] if len(s) == 2 else 64
        P[name] = scale * rng.standard_normal(s) / np.sqrt(fan)
    return mpnn.pack(P)


def _random_inputs(G, rng):
    N = len(G.nodes)
    X = np.zeros((N, mpnn.NFEAT))
    X[:, :9] = rng.standard_normal((N, 9))
    th = rng.standard_normal(G.fine)
    tu = rng.standard_normal(len(G.edges))
    return X, th, tu


def test_layout_size():
    assert mpnn.N_PARAMS == 16 * 64 + 64 + 3 * (128 * 64 + 64) + 64 + 64 + 1 == 25985


def test_gradient_matches_finite_differences(hex8):
    _, _, G = _graph(hex8)
    rng = np.random.default_rng(5)
    p = _random_params(rng)
    X, th, tu = _random_inputs(G, rng)
    loss, g = mpnn.loss_and_grad(p, G, X, th, tu)
    L = lambda q: mpnn.loss_and_grad(q, G, X, th, tu)[0]
    eps = 1e-6
    # a random direction through every parameter
    d = rng.standard_normal(p.size)
    fd = (L(p + eps * d) - L(p - eps * d)) / (2 * eps)
    assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(fd))
    # single coordinates in every block
    off = 0
    for name, s in mpnn.param_shapes():
        n = int(np.prod(s))
        for i in rng.choice(n, size=min(n, 4), replace=False):
            e = np.zeros(p.size)
            e[off + i] = 1.0
            fd = (L(p + eps * e) - L(p - eps * e)) / (2 * eps)
            assert abs(fd - g[off + i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, i)
        off += n
    assert loss > 0


def test_neighbour_mean_matches_edge_scan(lloyd_mesh):
    o = Oracle(lloyd_mesh)
    m = lloyd_mesh
    fm = (np.hypot(m.xCell - 2e5, m.yCell - 2e5) < 5e4).astype(np.uint8)
    reg = o.regions(fm, 2, 2)
    G = mpnn.build_graph(m, reg)
    pos = {int(c): i for i, c in enumerate(G.nodes)}
    nb = [set() for _ in G.nodes]
    for e in range(m.nEdges):
        a, b = (int(x) for x in m.cellsOnEdge[e])
        if a in pos and b in pos:
            nb[pos[a]].add(pos[b])
            nb[pos[b]].add(pos[a])
    rng = np.random.default_rng(1)
    H = rng.standard_normal((len(G.nodes), 5))
    ref = np.array([H[sorted(s)].mean(axis=0) if s else np.zeros(5) for s in nb])
    assert np.allclose(mpnn.mean_nbr(G, H), ref, rtol=1e-14, atol=1e-14)
    B = rng.standard_normal(H.shape)
    lhs = np.sum(mpnn.mean_nbr(G, H) * B)
    rhs = np.sum(H * mpnn.mean_nbr_transpose(G, B))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # every fine edge joins two nodes, at least one of them fine
    assert np.all((G.ec0 < G.fine) | (G.ec1 < G.fine))


def test_outputs_equivariant_and_edge_head_odd(hex16):
    o, reg, G = _graph(hex16, rows=(6, 8))
    rng = np.random.default_rng(2)
    p = _random_params(rng)
    X, _, _ = _random_inputs(G, rng)
    oh, ou, _ = mpnn.forward(p, G, X)
    # relabel: shuffle the fine nodes among themselves, the rest among
    # themselves, and the edges
    nF = G.fine
    pn = np.concatenate([rng.permutation(nF), nF + rng.permutation(len(G.nodes) - nF)])
    pe = rng.permutation(len(G.edges))
    G2 = mpnn.build_graph(hex16, reg, node_order=G.nodes[pn], edge_order=G.edges[pe])
    oh2, ou2, _ = mpnn.forward(p, G2, X[pn])
    assert np.allclose(oh2, oh[pn[:nF]], rtol=1e-12, atol=1e-12)
    assert np.allclose(ou2, ou[pe], rtol=1e-12, atol=1e-12)
    G3 = mpnn.Graph(G.nodes, G.fine, G.nbrs, G.edges, G.ec1, G.ec0)
    _, ou3, _ = mpnn.forward(p, G3, X)
    assert np.array_equal(ou3, -ou)


def _igw_feature_errors(n):
    m = periodic_hex_mesh(n, n, 6.4e5 / n, f0=1.0e-4)
    p = igw_parameters(m, g=9.81, H=1000.0, f=1.0e-4, amp=1.0, mode=(2, 1))
    h, u = igw_state(m, p, 0.0)
    o = Oracle(m)
    reg = o.regions(strip_fine_mask(m, n // 2 - 2, n // 2 + 1, 6.4e5 / n), 2, 2)
    raw = mpnn.raw_features(m, o, reg, h, u, np.arange(m.nCells))
    phi = p.k * m.xCell + p.l * m.yCell
    div_ex = -(p.amp * p.omega / p.H) * np.sin(phi)
    vort_ex = (p.amp * p.f / p.H) * np.cos(phi)
    e_div = np.abs(raw[:, 2] - div_ex).max() / np.abs(div_ex).max()
    e_vort = np.abs(raw[:, 3] - vort_ex).max() / np.abs(vort_ex).max()
    assert np.allclose(raw[:, 0], h + m.bottom) and np.allclose(raw[:, 1], m.bottom)
    onehot = raw[:, 5:9]
    assert np.all(onehot.sum(axis=1) <= 1) and np.all(onehot[reg.cell == 0] == 0)
    assert np.all(onehot[(reg.cell == F) & (reg.cell_fbar == 0), 0] == 1)
    assert np.all(onehot[(reg.cell == F) & (reg.cell_fbar == 1), 1] == 1)
    assert np.all(onehot[reg.cell == I1, 2] == 1)
    assert np.all(onehot[reg.cell == I2, 3] == 1)
    return e_div, e_vort


def test_features_igw_closed_form_second_order():
    d32, v32 = _igw_feature_errors(32)
    d64, v64 = _igw_feature_errors(64)
    assert d64 < 5e-3 and v64 < 5e-3
    assert d64 < d32 / 3.0 and v64 < v32 / 3.0


def test_feature_sums_telescope(irregular):
    m = irregular
    o = Oracle(m)
    reg = o.regions(np.zeros(m.nCells, np.uint8) + (np.arange(m.nCells) < 20), 1, 1)
    rng = np.random.default_rng(3)
    h = 1000.0 + rng.standard_normal(m.nCells)
    u = rng.standard_normal(m.nEdges)
    raw = mpnn.raw_features(m, o, reg, h, u, np.arange(m.nCells))
    scale = np.sum(m.areaCell * np.abs(raw[:, 2]))
    assert abs(np.sum(m.areaCell * raw[:, 2])) <= 1e-12 * scale
    scale = np.sum(m.areaCell * np.abs(raw[:, 3]))
    assert abs(np.sum(m.areaCell * raw[:, 3])) <= 1e-12 * scale


def test_adam_first_step_closed_form():
    """Bias-corrected first step: m_hat = g and v_hat = g^2, so every
    parameter moves by -lr g / (|g| + eps) whatever the scale of g."""
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-6, 3, 50)
    lr, eps = 1e-3, 1e-8
    p1, m1, v1 = mpnn.adam_step(p0, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    np.testing.assert_allclose(p1 - p0, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-12)


def test_adam_constant_gradient_and_sign_flip():
    """A constant gradient keeps m_hat = g and v_hat = g^2 at every step
    (the bias corrections undo the geometric sums exactly), so each step is
    the first step's.  Gradients +1 then -1 with (b1, b2) = (0.9, 0.999):
    m = -0.01, v = 0.001999, m_hat = -1/19, v_hat = 1, a step of
    +lr / (19 (1 + eps))."""
    lr, eps = 2e-3, 1e-8
    p, m, v = np.array([0.5]), np.zeros(1), np.zeros(1)
    for t in range(1, 6):
        q, m, v = mpnn.adam_step(p, np.array([-3.0]), m, v, t, lr, eps=eps)
        np.testing.assert_allclose(q - p, lr * 3.0 / (3.0 + eps), rtol=1e-9)
        p = q
    p, m, v = mpnn.adam_step(np.array([0.0]), np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr,
                             eps=eps)
    np.testing.assert_allclose(p, -lr / (1.0 + eps), rtol=1e-14)
    p2, m, v = mpnn.adam_step(p, np.array([-1.0]), m, v, 2, lr, eps=eps)
    np.testing.assert_allclose(m, -0.01, rtol=1e-12)
    np.testing.assert_allclose(v, 0.001999, rtol=1e-12)
    np.testing.assert_allclose(p2 - p, lr / (19.0 * (1.0 + eps)), rtol=1e-9)
