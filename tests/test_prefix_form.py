"""The cell kernel's O(n) form of the per-cell PV sum, checked on the CPU.

For a cell with slots 0..n-1 (edges counter-clockwise), kite fractions k_j of
the vertex after slot j, and R_ab the fractions summed counter-clockwise from
slot a up to (not including) slot b, the PV share of edge b needs

    P_b = sum_{a != b} (R_ab - 1/2) X_a          (eq:weights, split by cell)

The kernel evaluates it from prefix sums: with S_b = k_0 + ... + k_{b-1},
S_n the total, t = sum X, p = sum S X and c_b = X_0 + ... + X_b,

    P_b = (S_b + S_n - 1/2) t + X_b / 2 - p - S_n c_b.

This test compares that form with the direct O(n^2) double sum, for random
cells of 3 to 16 sides, and checks the regular-hexagon weights it implies.
"""
import numpy as np
import pytest


def direct(k, X):
    n = len(k)
    P = np.zeros(n)
    for b in range(n):
        for a in range(n):
            if a == b:
                continue
            R = sum(k[j % n] for j in range(a, a + (b - a) % n))
            P[b] += (R - 0.5) * X[a]
    return P


def prefix_form(k, X):
    S = np.concatenate([[0.0], np.cumsum(k)[:-1]])  # S_b
    Sn = k.sum()
    t, p, c = X.sum(), (S * X).sum(), np.cumsum(X)
    return (S + Sn - 0.5) * t + 0.5 * X - p - Sn * c


@pytest.mark.parametrize("n", [3, 4, 5, 6, 7, 8, 11, 16])
def test_prefix_form_equals_direct_sum(n):
    rng = np.random.default_rng(100 + n)
    for _ in range(20):
        k = rng.uniform(0.2, 1.0, n)
        k /= k.sum() * rng.uniform(0.999, 1.001)  # S_n near 1, not exactly 1
        X = rng.standard_normal(n)
        np.testing.assert_allclose(prefix_form(k, X), direct(k, X), rtol=0, atol=1e-13)


def test_regular_hexagon_weights():
    """On a regular hexagon every kite is 1/6 of the cell, so the weight of
    slot a in P_b is R_ab - 1/2 = (b - a mod 6)/6 - 1/2: -1/3, -1/6, 0, 1/6,
    1/3 for a one to five slots before b (the magnitudes 1/3, 1/6, 0 of the
    regular-mesh TRiSK weights)."""
    k = np.full(6, 1.0 / 6.0)
    for a in range(6):
        X = np.zeros(6)
        X[a] = 1.0
        P = prefix_form(k, X)
        for b in range(6):
            if b == a:
                continue
            want = ((b - a) % 6) / 6.0 - 0.5
            assert abs(P[b] - want) < 1e-15, (a, b, P[b], want)
