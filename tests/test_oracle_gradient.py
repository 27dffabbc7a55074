"""Pins for the oracle's adjoint-state gradient (eqs. AS, Grad, Adj): the
complex-step derivative of the objective (exact to rounding because the
discrete objective is analytic in m), the Taylor test (Section "Propagators
verification for inversion", eqs. GrFWI and GrFWI:test) and the two
summation-by-parts forms of the imaging condition."""
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
PAPER = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))


def _problem(o, ndim=2, k=8, nbl=4, nt=60, seed=0):
    rng = np.random.default_rng(seed)
    shape_phys = (14, 12) if ndim == 2 else (7, 6, 8)
    h = (10.0,) * ndim
    v_true = 2.0 + 0.5 * rng.random(shape_phys)
    v0 = np.full(shape_phys, 2.0)
    shape = tuple(n + 2 * nbl for n in shape_phys)
    g = o.Grid(shape, h, k)
    eta = o.damping_eta(shape_phys, nbl, h, 2.5)
    dt = 0.5 * o.critical_dt(ndim, h, k, 2.5)
    ext = [(n - 1) * 10.0 for n in shape_phys]
    src = o.sparse_points(np.array([[e / 2 + 3.0 for e in ext]]), h, nbl, shape)
    rec_xyz = np.stack([np.linspace(0, ext[0], 7)] + [np.full(7, 13.0)] * (ndim - 1), 1)
    rec = o.sparse_points(rec_xyz, h, nbl, shape)
    from synthetic import ricker
    q = ricker(nt, dt, 40.0, t0=25.0)[:, None]
    m_true = 1.0 / o.pad_edge(v_true, nbl) ** 2
    m0 = 1.0 / o.pad_edge(v0, nbl) ** 2
    d_obs = o.forward(g, m_true, eta, dt, nt, src, q, rec)
    return g, m0, m_true, eta, dt, nt, src, rec, q, d_obs


def _phi_and_grad(o, g, m, eta, dt, nt, src, rec, q, d_obs, seg=None):
    d = o.forward(g, m, eta, dt, nt, src, q, rec)
    y = d - d_obs
    return o.misfit(d, d_obs), o.gradient(g, m, eta, dt, nt, src, q, rec, y, seg=seg)


@pytest.mark.parametrize("ndim", [2, 3])
def test_gradient_matches_complex_step(oracle_mod, ndim):
    o = oracle_mod
    g, m0, mt, eta, dt, nt, src, rec, q, d_obs = _problem(o, ndim=ndim, nt=50)
    _, grad = _phi_and_grad(o, g, m0, eta, dt, nt, src, rec, q, d_obs)
    rng = np.random.default_rng(5)
    flat = rng.choice(g.size, size=6, replace=False)
    eps = 1e-30
    scale = np.max(np.abs(grad))
    for c in flat:
        mz = m0.astype(np.complex128)
        mz.ravel()[c] += 1j * eps
        dz = o.forward(g, mz, eta, dt, nt, src, q.astype(np.complex128), rec)
        rz = dz - d_obs
        phi_z = 0.5 * np.sum(rz * rz)        # analytic continuation, y^2 not |y|^2
        cs = phi_z.imag / eps
        assert abs(cs - grad.ravel()[c]) <= 1e-11 * scale, (c, cs, grad.ravel()[c])
    # also a direction derivative over all nodes at once
    dm = rng.standard_normal(g.shape) * 1e-3
    dz = o.forward(g, m0 + 1j * eps * dm, eta, dt, nt, src, q.astype(np.complex128), rec)
    rz = dz - d_obs
    cs = (0.5 * np.sum(rz * rz)).imag / eps
    ip = float(np.sum(grad * dm))
    assert abs(cs - ip) <= 1e-11 * abs(ip)


def test_gradient_summation_by_parts_and_segments(oracle_mod):
    o = oracle_mod
    g, m0, mt, eta, dt, nt, src, rec, q, d_obs = _problem(o, nt=41)
    d = o.forward(g, m0, eta, dt, nt, src, q, rec)
    y = d - d_obs
    g1, g2 = o.gradient(g, m0, eta, dt, nt, src, q, rec, y, both=True)
    assert np.max(np.abs(g1 - g2)) <= 1e-12 * np.max(np.abs(g1))
    for seg in (1, 3, 7, 40, 100):
        gs = o.gradient(g, m0, eta, dt, nt, src, q, rec, y, seg=seg)
        assert np.max(np.abs(gs - g1)) <= 1e-13 * np.max(np.abs(g1))


def test_taylor(oracle_mod):
    """eps0 = Phi(m + h dm) - Phi(m) is O(h), eps1 = eps0 - h <g, dm> is O(h^2).
    The paper reports slopes 1.06 and 2.01 at order 8 in FP64."""
    o = oracle_mod
    g, m0, mt, eta, dt, nt, src, rec, q, d_obs = _problem(o, k=8, nt=80)
    phi0, grad = _phi_and_grad(o, g, m0, eta, dt, nt, src, rec, q, d_obs)
    dm = mt - m0
    # h small enough that the quadratic term dominates eps1 (for this dm the
    # cubic term still wins above h ~ 2^-8), large enough to stay clear of
    # FP64 rounding in Phi (~1e-13 relative)
    hs = 2.0 ** -np.arange(10, 17)
    e0, e1 = [], []
    gdm = float(np.sum(grad * dm))
    for hh in hs:
        phi = o.misfit(o.forward(g, m0 + hh * dm, eta, dt, nt, src, q, rec), d_obs)
        e0.append(abs(phi - phi0))
        e1.append(abs(phi - phi0 - hh * gdm))
    s0 = np.polyfit(np.log(hs), np.log(e0), 1)[0]
    s1 = np.polyfit(np.log(hs), np.log(e1), 1)[0]
    paper = PAPER["taylor_slopes"]
    assert abs(s0 - 1.0) < 0.1 and abs(s1 - 2.0) < 0.1, (s0, s1, paper)
