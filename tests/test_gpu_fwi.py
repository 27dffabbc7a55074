"""Multi-shot FWI gradient and fixed-step update on the GPU (Section "FWI
using Devito operators": a loop over the shots with the gradients summed, then
a fixed-step update), against the FP64 oracle's fwi_objective / fwi_update.

Bars: summed gradient rel. L2 <= 1e-3, predicted records <= 1e-4, misfit
<= 1e-3 relative (it is a sum of squared residuals whose FP32 error is about
the record's relative error divided by the residual's relative size). The
two-solve path must equal the three-solve path (forward, residual, gradient)
bitwise, and every checkpoint count must give the same bits.
"""
import numpy as np
import pytest

from _harness import away_mask, check_field, check_record, point_nodes, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _survey(ndim=2, nshots=3, steps=150, k=8, nbl=10, seed=3):
    import oracle
    from synthetic import ricker, smooth_random_velocity
    shape_phys = (60, 50) if ndim == 2 else (34, 30, 38)
    h = (10.0,) * ndim
    # a constant starting model against a smooth random true model with a
    # Gaussian anomaly: residuals of the size of the data, so that the FP32
    # misfit is well conditioned
    v0 = np.full(shape_phys, 2.2)
    c = [n // 2 for n in shape_phys]
    grids = np.meshgrid(*[np.arange(n) for n in shape_phys], indexing="ij")
    r2 = sum((g - cc) ** 2 for g, cc in zip(grids, c))
    v_true = (smooth_random_velocity(shape_phys, seed, sigma=6.0, vmin=1.8, vmax=2.6)
              + 0.3 * np.exp(-r2 / (2 * 5.0 ** 2)))
    m0 = (1.0 / oracle.pad_edge(v0, nbl) ** 2).astype(np.float32)
    mt = (1.0 / oracle.pad_edge(v_true, nbl) ** 2).astype(np.float32)
    vmax = float(v_true.max())
    dt = 0.5 * oracle.critical_dt(ndim, h, k, vmax)
    nt = steps + 1
    ext = [(n - 1) * hh for n, hh in zip(shape_phys, h)]
    rng = np.random.default_rng(seed)
    shots = []
    for s in range(nshots):
        src = np.array([[ext[0] * (s + 0.5) / nshots + 3.3] + [e / 2 + 1.1 for e in ext[1:-1]] + [20.0]])
        nrec = 40 + 7 * s
        cols = [np.sort(rng.uniform(0, e, nrec)) for e in ext[:-1]] + [np.full(nrec, 25.0)]
        rec = np.stack(cols, axis=1)
        q = ricker(nt, dt, 15.0)[:, None].astype(np.float32)
        shots.append((src, q, rec))
    shape = mt.shape
    g = oracle.Grid(shape, h, k)
    eta = oracle.damping_eta(shape_phys, nbl, h, vmax)
    pts = [(oracle.sparse_points(s, h, nbl, shape), q, oracle.sparse_points(r, h, nbl, shape))
           for s, q, r in shots]
    d_obs = [oracle.forward(g, mt.astype(np.float64), eta, dt, nt, ps, q.astype(np.float64), pr)
             .astype(np.float32) for ps, q, pr in pts]
    return dict(shape_phys=shape_phys, h=h, nbl=nbl, k=k, vmax=vmax, dt=dt, nt=nt, m0=m0, mt=mt,
                shots=shots, d_obs=d_obs, grid=g, eta=eta, pts=pts)


def _prop(S, m=None):
    from paper_1808_01995_amd import Propagator
    m = torch.from_numpy(np.ascontiguousarray(S["m0"] if m is None else m)).cuda()
    return Propagator(m=m, shape=S["shape_phys"], spacing=S["h"], nbl=S["nbl"],
                      space_order=S["k"], c_ref=S["vmax"])


def _gpu_shots(S):
    return [(s, torch.from_numpy(q).cuda(), r, torch.from_numpy(d).cuda())
            for (s, q, r), d in zip(S["shots"], S["d_obs"])]


@pytest.mark.parametrize("ndim", [2, 3])
def test_fwi_gradient_matches_oracle(ndim):
    import oracle
    S = _survey(ndim=ndim, steps=150 if ndim == 2 else 90)
    prop = _prop(S)
    phi, g, preds = prop.fwi_gradient(S["dt"], S["nt"], _gpu_shots(S), return_pred=True)
    torch.cuda.synchronize()
    phi_ref, g_ref, preds_ref = oracle.fwi_objective(
        S["grid"], S["m0"].astype(np.float64), S["eta"], S["dt"], S["nt"],
        [(ps, q.astype(np.float64), pr) for ps, q, pr in S["pts"]],
        [d.astype(np.float64) for d in S["d_obs"]])
    for i, (d, dr) in enumerate(zip(preds, preds_ref)):
        check_record(d.cpu().numpy(), dr, label="fwi %dD shot %d record" % (ndim, i))
    assert abs(phi - phi_ref) <= 1e-3 * phi_ref, (phi, phi_ref)
    print("fwi %dD: misfit %.6e vs %.6e" % (ndim, phi, phi_ref))
    nodes = np.vstack([point_nodes(p, S["h"], S["nbl"], S["m0"].shape) for s, q, r in S["shots"] for p in (s, r)])
    check_field(g.cpu().numpy(), g_ref, mask=away_mask(S["m0"].shape, nodes, S["k"] // 2),
                label="fwi %dD summed gradient" % ndim)


def test_two_solves_equal_three_solve_path():
    """One shot through wf_fwi_gradient (the residual formed from the
    gradient's own forward sweep) equals forward + residual + wf_gradient
    bitwise; the predicted record equals wf_forward's record bitwise."""
    S = _survey(nshots=1)
    prop = _prop(S)
    (s, q, r, d_obs), = _gpu_shots(S)
    phi, g, (dp,) = prop.fwi_gradient(S["dt"], S["nt"], [(s, q, r, d_obs)], return_pred=True)
    d = prop.forward(S["dt"], S["nt"], s, q, r)
    res = (d - d_obs).contiguous()
    g3 = prop.gradient(S["dt"], S["nt"], s, q, r, res)
    torch.cuda.synchronize()
    assert torch.equal(dp, d)
    assert torch.equal(g, g3)
    phi3 = 0.5 * float((res.double() ** 2).sum())
    assert abs(phi - phi3) <= 1e-12 * phi3


def test_fwi_checkpoint_counts_bitwise_and_sum_of_shots():
    S = _survey(nshots=3, steps=120)
    prop = _prop(S)
    shots = _gpu_shots(S)
    phi_a, g_a = prop.fwi_gradient(S["dt"], S["nt"], shots, n_checkpoints=-1)
    for nck in (2, 7, 0):
        phi_b, g_b = prop.fwi_gradient(S["dt"], S["nt"], shots, n_checkpoints=nck)
        assert phi_b == phi_a and torch.equal(g_b, g_a), nck
    # the sum of single-shot gradients (summation order differs: FP32 rounding)
    parts = [prop.fwi_gradient(S["dt"], S["nt"], [sh]) for sh in shots]
    assert abs(sum(p[0] for p in parts) - phi_a) <= 1e-12 * phi_a
    gs = sum(p[1].double() for p in parts)
    assert float((gs - g_a.double()).norm() / gs.norm()) <= 1e-5


def test_model_update_and_descent():
    import oracle
    from paper_1808_01995_amd import WaveFDError, _abi
    S = _survey(nshots=2, steps=120)
    prop = _prop(S)
    shots = _gpu_shots(S)
    phi0, g0 = prop.fwi_gradient(S["dt"], S["nt"], shots)
    m_before = prop.m.clone()
    # the update against its closed form (one FP32 fma per node, then the box)
    vmin, vmax = 1.9, 2.7
    alpha = 0.02 * float(m_before.abs().max()) / float(g0.abs().max())
    prop.update(g0, alpha, vmin=vmin, vmax=vmax)
    m_ref = oracle.fwi_update(m_before.cpu().numpy(), g0.cpu().numpy(), alpha,
                              1.0 / vmax ** 2, 1.0 / vmin ** 2)
    m_new = prop.m.cpu().numpy()
    assert np.max(np.abs(m_new - m_ref)) <= 2e-7 * np.max(np.abs(m_ref))
    assert m_new.min() >= np.float32(1.0 / vmax ** 2) and m_new.max() <= np.float32(1.0 / vmin ** 2)
    # the model now propagates with the new m: same bits as a fresh model
    fresh = _prop(S, m=m_new)
    s, q, r, _ = shots[0]
    d1 = prop.forward(S["dt"], S["nt"], s, q, r)
    d2 = fresh.forward(S["dt"], S["nt"], s, q, r)
    assert torch.equal(d1, d2)
    # a non-finite gradient is refused and m is left as it was
    bad = g0.clone()
    bad.view(-1)[17] = float("nan")
    keep = prop.m.clone()
    with pytest.raises(WaveFDError) as e:
        prop.update(bad, alpha)
    assert e.value.status == _abi.WF_E_NONFINITE
    d3 = prop.forward(S["dt"], S["nt"], s, q, r)
    assert torch.equal(d3, d1) and torch.equal(prop.m, keep)
    with pytest.raises(WaveFDError):
        _abi.wf_model_update(prop.handle, g0, alpha, 0.0, 1.0)
    # fixed-step descent: the misfit falls at every iteration
    prop2 = _prop(S)
    phis = []
    for it in range(3):
        phi, g = prop2.fwi_gradient(S["dt"], S["nt"], shots)
        phis.append(phi)
        step = 0.01 * float(prop2.m.abs().max()) / float(g.abs().max())
        prop2.update(g, step, vmin=1.5, vmax=3.0)
    phi_last, _ = prop2.fwi_gradient(S["dt"], S["nt"], shots)
    phis.append(phi_last)
    print("fwi misfit by iteration:", phis)
    assert all(b < a for a, b in zip(phis, phis[1:]))


def test_fwi_objective_autograd():
    """The multi-shot objective as a torch.autograd.Function on the physical
    grid (replicate-pad adjoint folds the layer): its value and gradient equal
    the sum of per-shot ModelingFunction losses and their autograd gradient."""
    from paper_1808_01995_amd import fwi_objective, model_data, pad_replicate
    S = _survey(nshots=2, steps=100)
    prop = _prop(S)
    shots = _gpu_shots(S)
    nbl = S["nbl"]
    inner = tuple(slice(nbl, nbl + n) for n in S["shape_phys"])
    m_phys = torch.from_numpy(np.ascontiguousarray(S["m0"][inner])).cuda().requires_grad_(True)
    phi = fwi_objective(pad_replicate(m_phys, nbl), prop, S["dt"], S["nt"], shots)
    phi.backward()
    g1 = m_phys.grad.clone()
    m2 = m_phys.detach().clone().requires_grad_(True)
    loss = 0.0
    for s, q, r, d_obs in shots:
        d = model_data(pad_replicate(m2, nbl), prop, S["dt"], S["nt"], s, q, r)
        loss = loss + 0.5 * ((d.double() - d_obs.double()) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert abs(float(phi) - float(loss)) <= 1e-9 * float(loss)
    err = float((g1.double() - m2.grad.double()).norm() / m2.grad.double().norm())
    print("FWIObjective vs ModelingFunction gradient rel %.2e" % err)
    assert err <= 1e-5
