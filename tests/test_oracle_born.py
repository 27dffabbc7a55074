"""Pins for the oracle's linearised (Born) modelling dd = J dm.

J is the Jacobian of the discrete forward map (eq. Grad names it; the
adjoint-state gradient applies its transpose). Two independent pins:
the complex-step derivative of the forward map, Im F(m + i eps dm) / eps,
which equals J dm to rounding because F is analytic in m; and the adjoint
pair <J dm, r> = <dm, J^T r> with J^T r from the oracle gradient (itself
pinned by complex steps of the objective). A dropped term of the scattered
source, a wrong sign or a time shift fails both."""
import numpy as np
import pytest


def _setup(o, ndim, k=6, nbl=4, nt=50, seed=2):
    rng = np.random.default_rng(seed)
    shape_phys = (13, 11) if ndim == 2 else (7, 6, 8)
    h = (10.0,) * ndim
    shape = tuple(n + 2 * nbl for n in shape_phys)
    g = o.Grid(shape, h, k)
    eta = o.damping_eta(shape_phys, nbl, h, 2.6)
    dt = 0.5 * o.critical_dt(ndim, h, k, 2.6)
    v = 2.0 + 0.5 * rng.random(shape_phys)
    m = 1.0 / o.pad_edge(v, nbl) ** 2
    ext = [(n - 1) * 10.0 for n in shape_phys]
    src = o.sparse_points(np.array([[e / 2 + 2.3 for e in ext[:-1]] + [12.0]]), h, nbl, shape)
    rxyz = np.stack([np.linspace(0, ext[0], 7)] + [np.full(7, ext[1] / 3)] * (ndim - 2) + [np.full(7, 14.0)], 1)
    rec = o.sparse_points(rxyz, h, nbl, shape)
    from synthetic import ricker
    q = ricker(nt, dt, 40.0, t0=22.0)[:, None]
    dm = rng.standard_normal(shape) * 1e-3     # reaches into the damping layer too
    return g, eta, dt, nt, m, src, q, rec, dm


@pytest.mark.parametrize("ndim", [2, 3])
def test_born_is_the_complex_step_derivative(oracle_mod, ndim):
    o = oracle_mod
    g, eta, dt, nt, m, src, q, rec, dm = _setup(o, ndim)
    dd = o.born(g, m, eta, dt, nt, src, q, rec, dm)
    eps = 1e-30
    dz = o.forward(g, m + 1j * eps * dm, eta, dt, nt, src, q.astype(np.complex128), rec)
    cs = dz.imag / eps
    assert np.max(np.abs(dd)) > 0
    assert np.max(np.abs(dd - cs)) <= 1e-11 * np.max(np.abs(cs))
    assert np.all(dd[0] == 0)   # du^0 = 0


@pytest.mark.parametrize("ndim", [2, 3])
def test_born_adjoint_pair_with_gradient(oracle_mod, ndim):
    o = oracle_mod
    g, eta, dt, nt, m, src, q, rec, dm = _setup(o, ndim, seed=4)
    dd = o.born(g, m, eta, dt, nt, src, q, rec, dm)
    r = np.random.default_rng(9).standard_normal(dd.shape)
    jt = o.gradient(g, m, eta, dt, nt, src, q, rec, r)
    lhs = float(np.sum(dd * r))
    rhs = float(np.sum(dm * jt))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


def test_born_is_linear_in_dm(oracle_mod):
    o = oracle_mod
    g, eta, dt, nt, m, src, q, rec, dm = _setup(o, 2)
    dm2 = np.random.default_rng(3).standard_normal(dm.shape) * 1e-3
    a = o.born(g, m, eta, dt, nt, src, q, rec, dm)
    b = o.born(g, m, eta, dt, nt, src, q, rec, dm2)
    c = o.born(g, m, eta, dt, nt, src, q, rec, 2.0 * dm - 3.0 * dm2)
    assert np.max(np.abs(c - (2.0 * a - 3.0 * b))) <= 1e-12 * np.max(np.abs(c))
