"""Pins for the oracle's finite-difference weights and CFL limit (eq. fdSpace,
eq. eulerfwd). Checked against things other than the closed form itself:
an exact Vandermonde solve, Fornberg's recursion, polynomial exactness and the
textbook table of centred second-derivative weights."""
from fractions import Fraction

import numpy as np
import pytest


def _vandermonde_weights(M):
    """Solve sum_{j=-M}^{M} w_j j^p = 2 [p == 2], p = 0..2M, exactly."""
    n = 2 * M + 1
    js = list(range(-M, M + 1))
    A = [[Fraction(j) ** p for j in js] for p in range(n)]
    b = [Fraction(2) if p == 2 else Fraction(0) for p in range(n)]
    # Gauss-Jordan in rationals
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        inv = 1 / A[col][col]
        A[col] = [x * inv for x in A[col]]
        b[col] *= inv
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
                b[r] -= f * b[col]
    return dict(zip(js, b))


def _fornberg(M, deriv=2):
    """Fornberg's (1988) recursion for weights at x0 = 0 on nodes ordered
    0, 1, -1, 2, -2, ... (written from the published recursion)."""
    nodes = [0]
    for j in range(1, M + 1):
        nodes += [j, -j]
    N = len(nodes) - 1
    x0 = Fraction(0)
    delta = [[[Fraction(0)] * (N + 1) for _ in range(N + 1)] for _ in range(deriv + 1)]
    delta[0][0][0] = Fraction(1)
    c1 = Fraction(1)
    for n in range(1, N + 1):
        c2 = Fraction(1)
        for v in range(n):
            c3 = Fraction(nodes[n] - nodes[v])
            c2 *= c3
            for mm in range(min(n, deriv) + 1):
                prev = delta[mm - 1][n - 1][v] if mm > 0 else 0
                delta[mm][n][v] = ((nodes[n] - x0) * delta[mm][n - 1][v] - mm * prev) / c3
        for mm in range(min(n, deriv) + 1):
            prev = delta[mm - 1][n - 1][n - 1] if mm > 0 else 0
            delta[mm][n][n] = c1 / c2 * (mm * prev - (nodes[n - 1] - x0) * delta[mm][n - 1][n - 1])
        c1 = c2
    return {nodes[v]: delta[deriv][N][v] for v in range(N + 1)}


@pytest.mark.parametrize("k", [2, 4, 6, 8, 10, 12, 14, 16])
def test_closed_form_matches_vandermonde_and_fornberg(oracle_mod, k):
    a = oracle_mod.fd_weights(k)
    M = k // 2
    vdm = _vandermonde_weights(M)
    frn = _fornberg(M)
    assert vdm[0] == a[0] and frn[0] == a[0]
    for j in range(1, M + 1):
        assert vdm[j] == a[j] and vdm[-j] == a[j]
        assert frn[j] == a[j] and frn[-j] == a[j]


@pytest.mark.parametrize("k", [2, 4, 6, 8, 10, 12, 14, 16])
def test_polynomial_exactness(oracle_mod, k):
    """The centred stencil differentiates x^p exactly for p <= k+1 (odd powers
    by symmetry) and fails at p = k+2: the order is exactly k."""
    a = oracle_mod.fd_weights(k)
    M = k // 2

    def d2(p, x0=Fraction(3, 7)):
        s = a[0] * x0 ** p
        for j in range(1, M + 1):
            s += a[j] * ((x0 + j) ** p + (x0 - j) ** p)
        return s

    for p in range(0, k + 2):
        exact = p * (p - 1) * Fraction(3, 7) ** (p - 2) if p >= 2 else Fraction(0)
        assert d2(p) == exact, p
    p = k + 2
    assert d2(p) != p * (p - 1) * Fraction(3, 7) ** (p - 2)


def test_textbook_table(oracle_mod):
    """Standard centred second-derivative weights (Fornberg's table)."""
    F = Fraction
    table = {
        2: [F(-2), F(1)],
        4: [F(-5, 2), F(4, 3), F(-1, 12)],
        6: [F(-49, 18), F(3, 2), F(-3, 20), F(1, 90)],
        8: [F(-205, 72), F(8, 5), F(-1, 5), F(8, 315), F(-1, 560)],
    }
    for k, w in table.items():
        assert oracle_mod.fd_weights(k) == w


@pytest.mark.parametrize("k", [2, 4, 8, 12, 16])
def test_moments(oracle_mod, k):
    a = oracle_mod.fd_weights(k)
    assert a[0] + 2 * sum(a[1:]) == 0
    assert 2 * sum(j * j * a[j] for j in range(1, len(a))) == 2


def test_critical_dt_vs_spectral_radius(oracle_mod):
    """dt_crit from the symbol bound versus the spectral radius of -L from power
    iteration: the bound is an upper bound that a moderate Dirichlet grid nearly
    reaches; 1.2 dt_crit diverges and 0.95 dt_crit stays bounded."""
    o = oracle_mod
    for ndim, k in [(2, 4), (2, 8), (3, 8)]:
        shape = (40, 40) if ndim == 2 else (24, 24, 24)
        h = (10.0,) * ndim
        g = o.Grid(shape, h, k)
        rng = np.random.default_rng(1)
        x = rng.standard_normal(shape)
        lam = 0.0
        for _ in range(300):
            y = -o.laplacian(g, x)
            lam = float(np.sum(x * y) / np.sum(x * x))
            x = y / np.linalg.norm(y)
        bound = float(o.abs_weight_sum(k)) * sum(1 / hh ** 2 for hh in h)
        assert lam <= bound * (1 + 1e-12)
        assert lam >= 0.9 * bound
        v = 2.0
        dtc = o.critical_dt(ndim, h, k, v)
        assert abs(dtc - 2.0 / (v * np.sqrt(bound))) < 1e-15 * dtc
        m = np.full(shape, 1.0 / v ** 2)
        eta = np.zeros(shape)
        for fac, grows in [(1.2, True), (0.95, False)]:
            u0 = rng.standard_normal(shape)
            u1 = u0.copy()
            n0 = np.linalg.norm(u0)
            for _ in range(400):
                u2 = o.step(g, m, eta, fac * dtc, u0, u1)
                u0, u1 = u1, u2
            growth = np.linalg.norm(u1) / n0
            if grows:
                assert growth > 1e3
            else:
                assert growth < 10.0
