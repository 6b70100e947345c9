"""FP64 reference of the fine-region surrogate network: node features, forward
pass, loss and its gradient by hand-written back-propagation.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.

The surrogate is not part of the paper (it replaces Step 3 of Algorithm 2.2,
the fine substeps on F, by a learned map); what this module fixes is the
definition of the network that the library evaluates:

  nodes      cells of F, I1 and I2 (regions as labelled by the oracle);
             neighbours share an edge and are both nodes
  features   [h + b, b, div u, cell vorticity, K, one-hot(F interior,
             underlined F, I1, I2)], zero-padded to 16 columns, where
             div u  = (1/A_i) sum_{e in EC(i)} n_{e,i} l_e u_e,
             vort   = sum_{v in VC(i)} (A_{i,v} / A_i) zeta_v  (the kite
                      weights of the vertex-to-cell map of the TRiSK
                      appendix), zeta_v the vertex vorticity,
             K      = the kinetic energy of eq:sweTimeStepping at cell i;
             normalised columns 0-4: (x - mu) * inv_sd
  layers     H0 = relu(X W0 + b0), Hl = relu([H | mean_nbr H] Wl + bl), l=1..3
  heads      out_h = H3 wh + bh (fine cells), out_u = (H3[c1] - H3[c0]) wu
             (fine edges, normal from c0 to c1)
  loss       mean_F (out_h - th)^2 + mean_Fe (out_u - tu)^2

Parameter vector layout (row-major): W0[16][64], b0[64], W1[128][64], b1,
W2, b2, W3, b3, wh[64], wu[64], bh.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import F, I1, I2

HID = 64
NFEAT = 16
N_LAYERS = 3


def param_shapes():
    shapes = [("W0", (NFEAT, HID)), ("b0", (HID,))]
    for l in range(1, N_LAYERS + 1):
        shapes += [(f"W{l}", (2 * HID, HID)), (f"b{l}", (HID,))]
    shapes += [("wh", (HID,)), ("wu", (HID,)), ("bh", (1,))]
    return shapes


N_PARAMS = sum(int(np.prod(s)) for _, s in param_shapes())


def unpack(p):
    p = np.asarray(p, np.float64)
    assert p.size == N_PARAMS
    out, o = {}, 0
    for name, s in param_shapes():
        n = int(np.prod(s))
        out[name] = p[o:o + n].reshape(s)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in param_shapes()])


@dataclass
class Graph:
    nodes: np.ndarray        # caller cell index of each node
    fine: np.ndarray         # number of fine cells (nodes 0..fine-1 are F)
    nbrs: list               # neighbour node lists
    edges: np.ndarray        # caller edge index of each fine edge
    ec0: np.ndarray          # node index of c0 / c1 of each fine edge
    ec1: np.ndarray


def build_graph(mesh, regions, node_order=None, edge_order=None) -> Graph:
    """Nodes = cells of F, I1, I2; fine cells first.  node_order / edge_order
    (caller indices) fix the order when given, else ascending by region then
    index."""
    cr = regions.cell
    if node_order is None:
        fine = np.flatnonzero(cr == F)
        rest = np.flatnonzero((cr == I1) | (cr == I2))
        node_order = np.concatenate([fine, rest])
    node_order = np.asarray(node_order, np.int64)
    nF = int(np.count_nonzero(cr[node_order] == F))
    assert np.all(cr[node_order[:nF]] == F)
    pos = -np.ones(mesh.nCells, np.int64)
    pos[node_order] = np.arange(node_order.size)
    nbrs = []
    for c in node_order:
        lst = []
        for j in range(mesh.nEdgesOnCell[c]):
            d = mesh.cellsOnCell[c, j]
            if d >= 0 and pos[d] >= 0:
                lst.append(int(pos[d]))
        nbrs.append(lst)
    if edge_order is None:
        edge_order = np.flatnonzero(regions.edge == F)
    edge_order = np.asarray(edge_order, np.int64)
    ec0 = pos[mesh.cellsOnEdge[edge_order, 0]]
    ec1 = pos[mesh.cellsOnEdge[edge_order, 1]]
    assert np.all(ec0 >= 0) and np.all(ec1 >= 0)
    return Graph(node_order, nF, nbrs, edge_order, ec0, ec1)


def raw_features(mesh, oracle, regions, h, u, cells):
    """Unnormalised features [len(cells) x 16] of the state (h, u)."""
    K, _, zeta, _ = oracle.diag_fields(h, u)
    out = np.zeros((len(cells), NFEAT))
    for r, c in enumerate(cells):
        A = mesh.areaCell[c]
        div = 0.0
        for j in range(mesh.nEdgesOnCell[c]):
            e = mesh.edgesOnCell[c, j]
            n = 1.0 if mesh.cellsOnEdge[e, 0] == c else -1.0
            div += n * mesh.dvEdge[e] * u[e]
        vort = 0.0
        for j in range(mesh.nEdgesOnCell[c]):
            v = mesh.verticesOnCell[c, j]
            k = list(mesh.cellsOnVertex[v]).index(c)
            vort += mesh.kiteAreasOnVertex[v, k] / A * zeta[v]
        out[r, 0] = h[c] + mesh.bottom[c]
        out[r, 1] = mesh.bottom[c]
        out[r, 2] = div / A
        out[r, 3] = vort
        out[r, 4] = K[c]
        reg = regions.cell[c]
        if reg == F:
            out[r, 5 if not regions.cell_fbar[c] else 6] = 1.0
        elif reg == I1:
            out[r, 7] = 1.0
        elif reg == I2:
            out[r, 8] = 1.0
    return out


def normalise(raw, norm):
    X = np.zeros_like(raw)
    X[:, :5] = (raw[:, :5] - norm[:5]) * norm[5:10]
    X[:, 5:9] = raw[:, 5:9]
    return X


def relu(x):
    return np.maximum(x, 0.0)


def mean_nbr(G: Graph, H):
    out = np.zeros_like(H)
    for i, lst in enumerate(G.nbrs):
        if lst:
            out[i] = H[lst].mean(axis=0)
    return out


def mean_nbr_transpose(G: Graph, D):
    """Adjoint of mean_nbr: out[j] = sum over i with j in nbrs(i) of D[i]/deg_i."""
    out = np.zeros_like(D)
    for i, lst in enumerate(G.nbrs):
        for j in lst:
            out[j] += D[i] / len(lst)
    return out


def forward(p, G: Graph, X):
    P = unpack(p)
    cache = {"X": X}
    H = relu(X @ P["W0"] + P["b0"])
    cache["H0"] = H
    for l in range(1, N_LAYERS + 1):
        HC = np.concatenate([H, mean_nbr(G, H)], axis=1)
        cache[f"HC{l}"] = HC
        H = relu(HC @ P[f"W{l}"] + P[f"b{l}"])
        cache[f"H{l}"] = H
    out_h = H[:G.fine] @ P["wh"] + P["bh"][0]
    out_u = (H[G.ec1] - H[G.ec0]) @ P["wu"]
    return out_h, out_u, cache


def loss_and_grad(p, G: Graph, X, th, tu):
    """Loss and its gradient with respect to p (same layout)."""
    P = unpack(p)
    out_h, out_u, cache = forward(p, G, X)
    dh = out_h - th
    du = out_u - tu
    nF, nE = len(dh), len(du)
    loss = float(np.dot(dh, dh) / nF + np.dot(du, du) / nE)
    gh = 2.0 * dh / nF
    gu = 2.0 * du / nE
    grads = {}
    H3 = cache[f"H{N_LAYERS}"]
    grads["wh"] = H3[:nF].T @ gh
    grads["bh"] = np.array([gh.sum()])
    dH3e = H3[G.ec1] - H3[G.ec0]
    grads["wu"] = dH3e.T @ gu
    dH = np.zeros_like(H3)
    dH[:nF] += np.outer(gh, P["wh"])
    np.add.at(dH, G.ec1, np.outer(gu, P["wu"]))
    np.add.at(dH, G.ec0, -np.outer(gu, P["wu"]))
    for l in range(N_LAYERS, 0, -1):
        dZ = dH * (cache[f"H{l}"] > 0)
        HC = cache[f"HC{l}"]
        grads[f"W{l}"] = HC.T @ dZ
        grads[f"b{l}"] = dZ.sum(axis=0)
        dHC = dZ @ P[f"W{l}"].T
        dH = dHC[:, :HID] + mean_nbr_transpose(G, dHC[:, HID:])
    dZ = dH * (cache["H0"] > 0)
    grads["W0"] = cache["X"].T @ dZ
    grads["b0"] = dZ.sum(axis=0)
    return loss, pack(grads)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One step of Adam (Kingma and Ba, 2015, Algorithm 1) in FP64: the
    biased moment estimates m <- b1 m + (1 - b1) g and v <- b2 v + (1 - b2) g^2,
    their bias corrections m / (1 - b1^t) and v / (1 - b2^t) for step t >= 1,
    and p <- p - lr m_hat / (sqrt(v_hat) + eps).  Returns (p, m, v)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
