"""Linearised (Born) modelling on the GPU, dd = J dm, against the FP64
oracle's born(); its adjoint pair with the GPU gradient (J^T); exact
linearity; the background record against wf_forward.

Bars: Born records rel. L2 <= 1e-4 (the FP32 bar of the forward records);
GPU dot test <J dm, r> vs <dm, J^T r> <= 1e-4.
"""
import numpy as np
import pytest

from _harness import check_record, make_problem, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dm(P, seed, scale=1e-3):
    """A smooth perturbation plus noise, reaching into the damping layer."""
    rng = np.random.default_rng(seed)
    shape = P.comp_shape
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    c = [n / 2.0 for n in shape]
    r2 = sum((g - cc) ** 2 for g, cc in zip(grids, c))
    dm = np.exp(-r2 / (2 * (min(shape) / 6.0) ** 2)) + 0.1 * rng.standard_normal(shape)
    return (scale * dm).astype(np.float32)


def _oracle_born(P, dm):
    import oracle
    return oracle.born(P.grid(), P.m64(), P.eta(), P.dt, P.nt, P.pts(P.src_xyz),
                       P.q32.astype(np.float64), P.pts(P.rec_xyz), dm.astype(np.float64))


@pytest.mark.parametrize("k", [4, 8, 12])
def test_born_2d_matches_oracle(k):
    P = make_problem((57, 49), 9, k, 140, seed=20 + k)
    prop = P.propagator()
    dm = _dm(P, k)
    dd, d = prop.born(P.dt, P.nt, P.src_xyz, torch.from_numpy(P.q32).cuda(), torch.from_numpy(dm).cuda(),
                      P.rec_xyz, return_background=True)
    torch.cuda.synchronize()
    check_record(dd.cpu().numpy(), _oracle_born(P, dm), label="Born 2D order %d" % k)
    # the background record is wf_forward's, bit for bit
    d2 = prop.forward(P.dt, P.nt, P.src_xyz, torch.from_numpy(P.q32).cuda(), P.rec_xyz)
    torch.cuda.synchronize()
    assert torch.equal(d, d2)


@pytest.mark.parametrize("k", [8, 16])
def test_born_3d_matches_oracle(k):
    P = make_problem((37, 29, 41), 8, k, 80, seed=30 + k, nrec=50)
    prop = P.propagator()
    dm = _dm(P, k)
    dd = prop.born(P.dt, P.nt, P.src_xyz, torch.from_numpy(P.q32).cuda(), torch.from_numpy(dm).cuda(),
                   P.rec_xyz)
    torch.cuda.synchronize()
    check_record(dd.cpu().numpy(), _oracle_born(P, dm), label="Born 3D order %d" % k)


@pytest.mark.parametrize("ndim", [2, 3])
def test_born_gradient_dot_test(ndim):
    """<J dm, r> = <dm, J^T r>: the GPU Born operator against the GPU
    gradient (which is the transpose the adjoint-state method applies)."""
    shape = (64, 52) if ndim == 2 else (36, 30, 40)
    P = make_problem(shape, 8, 8, 120 if ndim == 2 else 80, seed=40 + ndim, nrec=45)
    prop = P.propagator()
    q = torch.from_numpy(P.q32).cuda()
    dm = torch.from_numpy(_dm(P, 7)).cuda()
    dd = prop.born(P.dt, P.nt, P.src_xyz, q, dm, P.rec_xyz)
    from synthetic import band_limited_noise
    r = torch.from_numpy(band_limited_noise(P.nt, P.rec_xyz.shape[0], P.dt, 15.0, 3)
                         .astype(np.float32)).cuda()
    jt = prop.gradient(P.dt, P.nt, P.src_xyz, q, P.rec_xyz, r, n_checkpoints=-1)
    torch.cuda.synchronize()
    lhs = float((dd.double() * r.double()).sum())
    rhs = float((dm.double() * jt.double()).sum())
    print("born/gradient dot test %dD: %.9e %.9e rel %.2e" % (ndim, lhs, rhs, abs(lhs - rhs) / abs(lhs)))
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


def test_born_linear_deterministic_and_zero():
    P = make_problem((50, 44), 8, 8, 90, seed=51)
    prop = P.propagator()
    q = torch.from_numpy(P.q32).cuda()
    dm = torch.from_numpy(_dm(P, 3)).cuda()
    a = prop.born(P.dt, P.nt, P.src_xyz, q, dm, P.rec_xyz)
    b = prop.born(P.dt, P.nt, P.src_xyz, q, 2.0 * dm, P.rec_xyz)
    z = prop.born(P.dt, P.nt, P.src_xyz, q, torch.zeros_like(dm), P.rec_xyz)
    a2 = prop.born(P.dt, P.nt, P.src_xyz, q, dm, P.rec_xyz)
    torch.cuda.synchronize()
    assert torch.equal(a2, a)        # deterministic
    # scaling by 2 is exact in FP32 except where values fall into the range
    # that the kernels flush to zero (far below anything recorded)
    diff = float((b - 2.0 * a).abs().max())
    print("born 2 dm vs 2 born dm: max diff %.3e of %.3e" % (diff, float(a.abs().max())))
    assert diff <= 1e-6 * float(a.abs().max())
    assert float(z.abs().max()) == 0.0
    assert float(a.abs().max()) > 0.0
