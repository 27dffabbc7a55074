"""Pins for the oracle's operators against independent constructions:
the Laplacian as a Kronecker sum of 1D matrices (scipy.sparse), the forward
and adjoint as dense block-triangular solves of A(m) (matrix view, Section
"Temporal discretization"), the dot test (eq. AdjTestPrRatio), energy
conservation of the undamped leapfrog, the sparse operators' transposition
and multilinear exactness (Section "Sparse point interpolation")."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

HERE = os.path.dirname(os.path.abspath(__file__))
PAPER = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))


def _d2_1d(n, h, k, oracle_mod):
    """1D order-k second-difference matrix with the stencil truncated at the
    edges (values beyond the grid are zero)."""
    a = oracle_mod.fd_weights_float(k)
    M = k // 2
    diags = [np.full(n, a[0])]
    offs = [0]
    for j in range(1, M + 1):
        if j < n:
            diags += [np.full(n - j, a[j]), np.full(n - j, a[j])]
            offs += [j, -j]
    return sp.diags(diags, offs, shape=(n, n), format="csr") / (h * h)


def _laplacian_matrix(shape, spacing, k, oracle_mod):
    mats = [_d2_1d(n, h, k, oracle_mod) for n, h in zip(shape, spacing)]
    L = None
    for a in range(len(shape)):
        term = None
        for b in range(len(shape)):
            f = mats[b] if a == b else sp.identity(shape[b], format="csr")
            term = f if term is None else sp.kron(term, f, format="csr")
        L = term if L is None else L + term
    return L


def _setup(oracle_mod, shape_phys, nbl, k, seed=0, nsrc=1, nrec=5, h=10.0, nt=12, damp=True):
    o = oracle_mod
    rng = np.random.default_rng(seed)
    nd = len(shape_phys)
    spacing = (h,) * nd
    v = 1.5 + 1.5 * rng.random(shape_phys)
    vp = o.pad_edge(v, nbl)
    m = 1.0 / vp ** 2
    shape = vp.shape
    g = o.Grid(shape, spacing, k)
    eta = o.damping_eta(shape_phys, nbl, spacing, float(v.max())) if damp else np.zeros(shape)
    ext = [(n - 1) * h for n in shape_phys]
    src_xyz = np.stack([rng.uniform(-nbl * h, e + nbl * h, nsrc) for e in ext], axis=1)
    rec_xyz = np.stack([rng.uniform(-nbl * h, e + nbl * h, nrec) for e in ext], axis=1)
    src = o.sparse_points(src_xyz, spacing, nbl, shape)
    rec = o.sparse_points(rec_xyz, spacing, nbl, shape)
    dt = 0.5 * o.critical_dt(nd, spacing, k, float(v.max()))
    return g, m, eta, dt, nt, src, rec, rng


def _P(node, w, N):
    n, K = node.shape
    rows = np.repeat(np.arange(n), K)
    return sp.csr_matrix((w.ravel(), (rows, node.ravel())), shape=(n, N))


def _assemble_A(g, m, eta, dt, nt, L):
    """Block lower-triangular A(m) for unknowns u^1..u^{nt-1}; row n (0..nt-2):
    a u^{n+1} - (2m + dt^2 L) u^n + b u^{n-1}."""
    N = g.size
    a = sp.diags(m.ravel() + 0.5 * eta.ravel() * dt)
    b = sp.diags(m.ravel() - 0.5 * eta.ravel() * dt)
    C = -(sp.diags(2.0 * m.ravel()) + dt * dt * L)
    blocks = [[None] * (nt - 1) for _ in range(nt - 1)]
    for n in range(nt - 1):
        blocks[n][n] = a                     # u^{n+1} is unknown n
        if n >= 1:
            blocks[n][n - 1] = C             # u^n
        if n >= 2:
            blocks[n][n - 2] = b             # u^{n-1}
    return sp.bmat(blocks, format="csc")


@pytest.mark.parametrize("ndim,k", [(2, 2), (2, 4), (2, 8), (3, 4), (3, 6)])
def test_laplacian_is_kronecker_sum(oracle_mod, ndim, k):
    o = oracle_mod
    shape = (9, 11) if ndim == 2 else (7, 6, 9)
    spacing = (10.0, 12.5) if ndim == 2 else (10.0, 7.5, 12.5)
    g = o.Grid(shape, spacing, k)
    L = _laplacian_matrix(shape, spacing, k, o)
    assert abs(L - L.T).max() < 1e-15
    u = np.random.default_rng(3).standard_normal(shape)
    got = o.laplacian(g, u).ravel()
    ref = L @ u.ravel()
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("ndim,k", [(2, 4), (2, 8), (3, 4)])
def test_forward_equals_dense_solve(oracle_mod, ndim, k):
    """O2 as a whole against a sparse-direct solve of the assembled A(m)."""
    o = oracle_mod
    shape_phys = (6, 5) if ndim == 2 else (4, 3, 4)
    g, m, eta, dt, nt, src, rec, rng = _setup(o, shape_phys, 2, k, nt=12)
    N = g.size
    L = _laplacian_matrix(g.shape, g.spacing, k, o)
    A = _assemble_A(g, m, eta, dt, nt, L)
    q = rng.standard_normal((nt, src[0].shape[0]))
    Ps = _P(*src, N)
    Pr = _P(*rec, N)
    rhs = np.concatenate([dt * dt * (Ps.T @ q[n]) for n in range(nt - 1)])
    U = spla.spsolve(A, rhs).reshape(nt - 1, N)
    d_ref = np.vstack([np.zeros((1, Pr.shape[0]))] + [Pr @ U[n] for n in range(nt - 1)])
    d, us = o.forward(g, m, eta, dt, nt, src, q, rec, save=True)
    scale = np.max(np.abs(U))
    assert np.max(np.abs(us[1:].reshape(nt - 1, N) - U)) <= 1e-12 * scale
    assert np.max(np.abs(us[0])) == 0.0
    assert np.max(np.abs(d - d_ref)) <= 1e-12 * np.max(np.abs(d_ref))


@pytest.mark.parametrize("ndim,k", [(2, 4), (3, 4)])
def test_adjoint_equals_dense_transpose_solve(oracle_mod, ndim, k):
    o = oracle_mod
    shape_phys = (6, 5) if ndim == 2 else (4, 3, 4)
    g, m, eta, dt, nt, src, rec, rng = _setup(o, shape_phys, 2, k, nt=10)
    N = g.size
    L = _laplacian_matrix(g.shape, g.spacing, k, o)
    A = _assemble_A(g, m, eta, dt, nt, L)
    y = rng.standard_normal((nt, rec[0].shape[0]))
    Ps = _P(*src, N)
    Pr = _P(*rec, N)
    # A^T W = P_r^T Y, Y block n <-> unknown u^{n+1} <-> y^{n+1}; x^n = dt^2 P_s W_n
    rhs = np.concatenate([Pr.T @ y[n + 1] for n in range(nt - 1)])
    W = spla.spsolve(A.T.tocsc(), rhs).reshape(nt - 1, N)
    x_ref = np.vstack([dt * dt * (Ps @ W[n]) for n in range(nt - 1)] + [np.zeros((1, Ps.shape[0]))])
    x = o.adjoint(g, m, eta, dt, nt, rec, y, src)
    assert np.max(np.abs(x - x_ref)) <= 1e-11 * np.max(np.abs(x_ref))


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("k", [2, 4, 6, 8, 10, 12])
def test_dot_test(oracle_mod, ndim, k):
    """<F x, y> = <x, F^T y> in FP64 (eq. AdjTestPrRatio). The paper's tables
    report <= 6.5e-16; the bound here is 1e-12."""
    o = oracle_mod
    from synthetic import band_limited_noise
    shape_phys = (40, 36) if ndim == 2 else (14, 12, 16)
    nbl = 6
    g, m, eta, dt, _, src, rec, rng = _setup(o, shape_phys, nbl, k, seed=k, nsrc=2, nrec=9)
    nt = 120
    # two-layer model as in the paper's tables
    v = np.full(shape_phys, 1.5)
    v[..., shape_phys[-1] // 2:] = 2.5
    m = 1.0 / o.pad_edge(v, nbl) ** 2
    dt = 0.5 * o.critical_dt(ndim, g.spacing, k, 2.5)
    x = band_limited_noise(nt, src[0].shape[0], dt, 40.0, seed=1)
    y = o.forward(g, m, eta, dt, nt, src, band_limited_noise(nt, src[0].shape[0], dt, 40.0, seed=2), rec)
    Fx = o.forward(g, m, eta, dt, nt, src, x, rec)
    FTy = o.adjoint(g, m, eta, dt, nt, rec, y, src)
    lhs = float(np.sum(Fx * y))
    rhs = float(np.sum(x * FTy))
    rel = abs(lhs - rhs) / abs(lhs)
    paper = PAPER["dot_test_rel_err_%dd" % ndim]
    assert max(paper["rel_err"]) < 1e-15  # the paper's own runs
    assert rel <= 1e-12, rel


def test_energy_conserved_without_damping(oracle_mod):
    """eta = 0, no source: E^{n+1/2} is invariant under the leapfrog update."""
    o = oracle_mod
    for ndim, k in [(2, 4), (2, 12), (3, 8)]:
        shape = (30, 34) if ndim == 2 else (14, 16, 12)
        h = (10.0,) * ndim
        g = o.Grid(shape, h, k)
        rng = np.random.default_rng(7)
        m = 1.0 / (1.5 + rng.random(shape)) ** 2
        eta = np.zeros(shape)
        dt = 0.5 * o.critical_dt(ndim, h, k, 2.5)
        u0 = rng.standard_normal(shape)
        u1 = u0 + 0.1 * rng.standard_normal(shape)
        E0 = o.energy(g, m, dt, u0, u1)
        for _ in range(200):
            u2 = o.step(g, m, eta, dt, u0, u1)
            u0, u1 = u1, u2
        E1 = o.energy(g, m, dt, u0, u1)
        assert E0 > 0
        assert abs(E1 - E0) <= 1e-12 * abs(E0)


def test_damping_profile_and_dissipation(oracle_mod):
    o = oracle_mod
    shape_phys = (30, 26)
    nbl = 8
    eta = o.damping_eta(shape_phys, nbl, (10.0, 10.0), 2.0)
    assert np.all(eta[nbl:-nbl, nbl:-nbl] == 0.0)
    assert np.all(eta >= 0)
    # grows monotonically toward the outer edge along an axis through the interior
    row = eta[:, nbl + 5]
    assert np.all(np.diff(row[:nbl + 1]) < 0) and np.all(np.diff(row[-nbl - 1:]) > 0)
    emax = 3 * math.log(1e3) / (2 * nbl * 10.0 * 2.0)
    assert abs(row[0] - emax) < 1e-15
    # the profile's exponent (quadratic in the depth d into the layer, the
    # reading of the smooth profile): constant second differences over d =
    # 0..nbl on both sides, equal to 2 emax / nbl^2, where a linear or cubic
    # profile would give zero or linearly varying ones
    for side in (row[:nbl + 1][::-1], row[-nbl - 1:]):
        d2 = np.diff(side, 2)
        assert np.allclose(d2, 2 * emax / nbl ** 2, rtol=1e-12, atol=0.0), d2
    for wrong in (1, 3):   # the check rejects another exponent
        r2 = o.damping_eta(shape_phys, nbl, (10.0, 10.0), 2.0, power=wrong)[:, nbl + 5]
        assert not np.allclose(np.diff(r2[-nbl - 1:], 2), 2 * emax / nbl ** 2, rtol=1e-12, atol=0.0)
    # separable: a node of a corner of the layer carries the sum of the two
    # axes' values
    c = nbl + 5
    for i, j in ((0, 0), (2, eta.shape[1] - 1), (eta.shape[0] - 3, 1)):
        assert abs(eta[i, j] - (eta[i, c] + eta[c, j])) <= 1e-15 * eta[i, j]
    # energy never increases with eta >= 0
    shape = eta.shape
    g = o.Grid(shape, (10.0, 10.0), 8)
    rng = np.random.default_rng(2)
    m = np.full(shape, 1.0 / 4.0)
    dt = 0.5 * o.critical_dt(2, (10.0, 10.0), 8, 2.0)
    u0 = rng.standard_normal(shape)
    u1 = u0.copy()
    E = o.energy(g, m, dt, u0, u1)
    for _ in range(300):
        u2 = o.step(g, m, eta, dt, u0, u1)
        u0, u1 = u1, u2
        E1 = o.energy(g, m, dt, u0, u1)
        assert E1 <= E * (1 + 1e-13)
        E = E1


def test_sparse_weights_exact_and_transposed(oracle_mod):
    o = oracle_mod
    rng = np.random.default_rng(11)
    for nd in (2, 3):
        shape_phys = (9, 7, 8)[:nd]
        nbl = 3
        spacing = (10.0, 12.0, 8.0)[:nd]
        shape = tuple(n + 2 * nbl for n in shape_phys)
        pts = np.stack([rng.uniform(-nbl * h, (n - 1 + nbl) * h, 50) for n, h in zip(shape_phys, spacing)], 1)
        # include exact nodes and the very last node of the grid
        pts[0] = [(n - 1 + nbl) * h for n, h in zip(shape_phys, spacing)]
        pts[1] = [-nbl * h for h in spacing]
        pts[2] = [2 * h for h in spacing]
        node, w = o.sparse_points(pts, spacing, nbl, shape)
        assert np.all(w >= 0) and np.allclose(w.sum(1), 1.0, atol=1e-15)
        # exact on multilinear fields f = c0 + sum c_a x_a + c_xy x y (+...)
        coords = np.meshgrid(*[(np.arange(n) - nbl) * h for n, h in zip(shape, spacing)], indexing="ij")
        c = rng.standard_normal(nd + 2)
        f = c[0] + sum(c[a + 1] * coords[a] for a in range(nd)) + c[-1] * coords[0] * coords[1]
        fp = c[0] + sum(c[a + 1] * pts[:, a] for a in range(nd)) + c[-1] * pts[:, 0] * pts[:, 1]
        got = np.sum(w * f.ravel()[node], axis=1)
        assert np.max(np.abs(got - fp)) <= 1e-11 * np.max(np.abs(fp))
        with pytest.raises(ValueError):
            o.sparse_points(np.array([[-(nbl + 0.01) * spacing[0]] + [0.0] * (nd - 1)]), spacing, nbl, shape)


def test_inject_and_sample_transposed_in_kernels(oracle_mod):
    """nt = 2 isolates the C injection and sampling: d^1 = P_r (dt^2/a) P_s^T q^0,
    and <P_r P_s^T q, y> == <q, P_s P_r^T y> through forward/adjoint."""
    o = oracle_mod
    g, m, eta, dt, nt, src, rec, rng = _setup(o, (7, 6, 5), 2, 4, nsrc=3, nrec=4, nt=2)
    N = g.size
    q = rng.standard_normal((2, 3))
    d = o.forward(g, m, eta, dt, 2, src, q, rec)
    a = m.ravel() + 0.5 * eta.ravel() * dt
    Ps, Pr = _P(*src, N), _P(*rec, N)
    ref = Pr @ ((dt * dt / a) * (Ps.T @ q[0]))
    assert np.allclose(d[1], ref, rtol=1e-14, atol=1e-300)
    assert np.all(d[0] == 0)
    y = rng.standard_normal((2, 4))
    x = o.adjoint(g, m, eta, dt, 2, rec, y, src)
    assert np.allclose(x[0], Ps @ ((dt * dt / a) * (Pr.T @ y[1])), rtol=1e-14)
    assert np.all(x[1] == 0)
