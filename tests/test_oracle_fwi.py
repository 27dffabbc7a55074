"""Pins for the oracle's multi-shot FWI objective, gradient and fixed-step
update (Section "FWI using Devito operators"; eq. AS summed over shots).

The summed gradient is pinned by the complex-step derivative of the summed
objective (exact to rounding: the discrete objective is analytic in m), which
fails for a dropped shot, a shot paired with another shot's data, or a sign
error in the residual; the update by its closed form and by descent."""
import numpy as np
import pytest


def _survey(o, ndim=2, k=4, nbl=4, nt=45, nshots=3, seed=1):
    rng = np.random.default_rng(seed)
    shape_phys = (13, 11) if ndim == 2 else (7, 6, 8)
    h = (10.0,) * ndim
    shape = tuple(n + 2 * nbl for n in shape_phys)
    g = o.Grid(shape, h, k)
    eta = o.damping_eta(shape_phys, nbl, h, 2.6)
    dt = 0.5 * o.critical_dt(ndim, h, k, 2.6)
    v_true = 2.0 + 0.6 * rng.random(shape_phys)
    m_true = 1.0 / o.pad_edge(v_true, nbl) ** 2
    m0 = 1.0 / o.pad_edge(np.full(shape_phys, 2.2), nbl) ** 2
    ext = [(n - 1) * 10.0 for n in shape_phys]
    from synthetic import ricker
    shots = []
    for s in range(nshots):
        sx = ext[0] * (s + 0.5) / nshots + 1.7
        src = o.sparse_points(np.array([[sx] + [e / 2 + 2.1 for e in ext[1:-1]] + [12.0]]), h, nbl, shape)
        nrec = 6 + s
        rxyz = np.stack([np.linspace(0, ext[0], nrec)] + [np.full(nrec, ext[1] / 3)] * (ndim - 2)
                        + [np.full(nrec, 14.0)], 1)
        rec = o.sparse_points(rxyz, h, nbl, shape)
        q = ricker(nt, dt, 40.0, t0=22.0 + 3 * s)[:, None]
        shots.append((src, q, rec))
    d_obs = [o.forward(g, m_true, eta, dt, nt, src, q, rec) for src, q, rec in shots]
    return g, eta, dt, nt, m0, m_true, shots, d_obs


@pytest.mark.parametrize("ndim", [2, 3])
def test_summed_gradient_matches_complex_step(oracle_mod, ndim):
    o = oracle_mod
    g, eta, dt, nt, m0, mt, shots, d_obs = _survey(o, ndim=ndim)
    phi, grad, preds = o.fwi_objective(g, m0, eta, dt, nt, shots, d_obs)
    assert phi > 0 and len(preds) == len(shots)
    rng = np.random.default_rng(7)
    eps = 1e-30
    for trial in range(2):
        dm = rng.standard_normal(g.shape) * 1e-3
        mz = m0 + 1j * eps * dm
        phi_z = 0.0
        for (src, q, rec), dob in zip(shots, d_obs):
            dz = o.forward(g, mz, eta, dt, nt, src, q.astype(np.complex128), rec)
            rz = dz - dob
            phi_z = phi_z + 0.5 * np.sum(rz * rz)
        cs = phi_z.imag / eps
        ip = float(np.sum(grad * dm))
        assert abs(cs - ip) <= 1e-11 * abs(ip), (cs, ip)
    # the real part is the objective itself
    assert abs(phi_z.real - phi) <= 1e-12 * phi


def test_summed_objective_is_sum_of_shots(oracle_mod):
    o = oracle_mod
    g, eta, dt, nt, m0, mt, shots, d_obs = _survey(o, nshots=3)
    phi, grad, _ = o.fwi_objective(g, m0, eta, dt, nt, shots, d_obs)
    parts = [o.fwi_objective(g, m0, eta, dt, nt, [sh], [d]) for sh, d in zip(shots, d_obs)]
    assert abs(sum(p[0] for p in parts) - phi) <= 1e-13 * phi
    gs = sum(p[1] for p in parts)
    assert np.max(np.abs(gs - grad)) <= 1e-13 * np.max(np.abs(grad))
    # every shot contributes (no shot's gradient is negligible)
    for p in parts:
        assert np.linalg.norm(p[1]) > 1e-3 * np.linalg.norm(grad)
    # at the true model the objective and gradient vanish
    phi_t, grad_t, _ = o.fwi_objective(g, mt, eta, dt, nt, shots, d_obs)
    assert phi_t == 0.0 and np.max(np.abs(grad_t)) == 0.0


def test_fixed_step_update(oracle_mod):
    o = oracle_mod
    g, eta, dt, nt, m0, mt, shots, d_obs = _survey(o)
    phi, grad, _ = o.fwi_objective(g, m0, eta, dt, nt, shots, d_obs)
    # closed form and projection
    m1 = o.fwi_update(m0, grad, 0.5)
    assert np.array_equal(m1, m0 - 0.5 * grad)
    lo, hi = 1.0 / 2.6 ** 2, 1.0 / 2.0 ** 2
    mb = o.fwi_update(m0, grad, 1e6, lo, hi)
    assert mb.min() >= lo and mb.max() <= hi
    assert np.any(mb == lo) and np.any(mb == hi)
    inside = (mb > lo) & (mb < hi)
    assert np.array_equal(mb[inside], (m0 - 1e6 * grad)[inside])
    # a small enough step along -g decreases the objective (first-order
    # decrease alpha ||g||^2 predicted within 10 %)
    alpha = 1e-3 * np.max(np.abs(m0)) / np.max(np.abs(grad))
    m_new = o.fwi_update(m0, grad, alpha)
    phi_new, _, _ = o.fwi_objective(g, m_new, eta, dt, nt, shots, d_obs)
    pred = alpha * float(np.sum(grad * grad))
    assert phi_new < phi
    assert abs((phi - phi_new) - pred) <= 0.1 * pred
