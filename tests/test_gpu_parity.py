"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs, element by element over whole shot records.

Tolerances: receiver traces rel. L2 <= 1e-4, gradients rel. L2 <= 1e-3, GPU
dot test <= 1e-4 (the FP32 bars of the specification). Sizes span several
(y, z) tiles and x chunks with ragged tails; every space order 4..16 runs.
"""
import numpy as np
import pytest

from _harness import check_field, check_record, make_problem, noise, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu_forward(P, prop=None, save_every=None):
    prop = prop or P.propagator()
    out = prop.forward(P.dt, P.nt, P.src_xyz, torch.from_numpy(P.q32).cuda(), P.rec_xyz,
                       save_every=save_every)
    torch.cuda.synchronize()
    return out


def test_c1_2d_so4_full_config():
    """101 x 101, h = 10 m, v = 1.5 km/s, order 4, 500 steps, nbl 20, Ricker
    10 Hz at the centre, 101 receivers at 20 m depth."""
    from synthetic import config
    import oracle
    c = config("c1_2d")
    from _harness import Problem
    v = c.velocity()
    m32 = (1.0 / oracle.pad_edge(v, c.nbl) ** 2).astype(np.float32)
    dt = c.dt_factor * oracle.critical_dt(2, c.spacing, c.space_order, float(v.max()))
    from synthetic import ricker
    q = ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32)
    P = Problem(c.shape, c.spacing, c.nbl, c.space_order, c.nt, dt, float(v.max()), v, m32,
                c.src, c.rec, q)
    d_ref = P.oracle_forward()
    d = _gpu_forward(P).cpu().numpy()
    check_record(d, d_ref, label="C1")
    assert np.all(d[0] == 0)


@pytest.mark.parametrize("k", [4, 6, 8, 10, 12, 14, 16])
def test_2d_all_orders(k):
    P = make_problem((53, 47), 9, k, 120, seed=k)
    d = _gpu_forward(P).cpu().numpy()
    check_record(d, P.oracle_forward(), label="2D order %d" % k)


@pytest.mark.parametrize("k", [4, 8, 16])
def test_2d_long_rows(k):
    """Rows of 1106 nodes select the 512-wide 2D tile (three tiles, the last
    ragged); forward and adjoint against the oracle."""
    P = make_problem((45, 1090), 8, k, 120, seed=80 + k, nrec=70)
    d = _gpu_forward(P).cpu().numpy()
    check_record(d, P.oracle_forward(), label="2D long rows order %d forward" % k)
    y = noise(P.nt, P.rec_xyz.shape[0], P.dt, 15.0, 6)
    prop = P.propagator()
    x = prop.adjoint(P.dt, P.nt, P.rec_xyz, torch.from_numpy(y.astype(np.float32)).cuda(),
                     P.src_xyz).cpu().numpy()
    check_record(x, P.oracle_adjoint(y.astype(np.float32).astype(np.float64)),
                 label="2D long rows order %d adjoint" % k)


@pytest.mark.parametrize("k", [4, 8, 12, 16])
def test_3d_orders_ragged_tiles(k):
    """(y, z) tiles of 16 x 64 and x chunks: 71 x 37 x 93 computational nodes
    leave ragged tiles on every axis."""
    P = make_problem((55, 21, 77), 8, k, 90, seed=10 + k, nrec=60)
    d = _gpu_forward(P).cpu().numpy()
    check_record(d, P.oracle_forward(), label="3D ragged tiles order %d" % k)


@pytest.mark.parametrize("k,nz_phys", [(8, 174), (16, 174), (4, 260)])
def test_3d_wide_tiles(k, nz_phys):
    """Wider z lengths on the 128 x 8 tile: 190 nodes (last z tile half
    empty) and 276 nodes, with ragged y tiles and x chunks."""
    P = make_problem((30, 21, nz_phys), 8, k, 60, seed=70 + k, nrec=40)
    d = _gpu_forward(P).cpu().numpy()
    check_record(d, P.oracle_forward(), label="3D order %d nz %d" % (k, nz_phys + 16))


def test_3d_so8_two_layer_and_save():
    P = make_problem((40, 36, 44), 10, 8, 80, seed=3, kind="two_layer", nrec=50)
    d, u = _gpu_forward(P, save_every=20)
    d_ref, u_ref = P.oracle_forward(save=True)
    check_record(d.cpu().numpy(), d_ref, label="two-layer record")
    u = u.cpu().numpy()
    for i, n in enumerate(range(0, P.nt, 20)):
        if n == 0:
            assert np.all(u[i] == 0)
        else:
            check_field(u[i], u_ref[n], tol=1e-4, label="saved u^%d" % n)


@pytest.mark.parametrize("ndim", [2, 3])
def test_adjoint_parity_and_dot_test(ndim):
    shape = (48, 41) if ndim == 2 else (30, 26, 34)
    P = make_problem(shape, 8, 8, 100, seed=20 + ndim, nsrc=3, nrec=40)
    prop = P.propagator()
    x = noise(P.nt, 3, P.dt, 20.0, seed=1).astype(np.float32)
    y = noise(P.nt, 40, P.dt, 20.0, seed=2).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    yt = torch.from_numpy(y).cuda()
    Fx = prop.forward(P.dt, P.nt, P.src_xyz, xt, P.rec_xyz).cpu().numpy().astype(np.float64)
    FTy = prop.adjoint(P.dt, P.nt, P.rec_xyz, yt, P.src_xyz).cpu().numpy().astype(np.float64)
    # against the oracle's adjoint on the same y
    FTy_ref = P.oracle_adjoint(y.astype(np.float64))
    check_record(FTy, FTy_ref, label="adjoint %dD" % ndim)
    assert np.all(FTy[-1] == 0)
    lhs = float(np.sum(Fx * y))
    rhs = float(np.sum(x * FTy))
    rel = abs(lhs - rhs) / abs(lhs)
    print("GPU dot test", ndim, "D:", lhs, rhs, rel)
    assert rel <= 1e-4


def test_deterministic_bitwise():
    P = make_problem((40, 35, 50), 8, 8, 60, seed=7, nsrc=2)
    prop = P.propagator()
    a = _gpu_forward(P, prop).cpu().numpy()
    b = _gpu_forward(P, prop).cpu().numpy()
    assert np.array_equal(a, b)


def test_edge_cases():
    """nt = 1, no receivers, no sources, sources on the last node and in the
    layer, nz not a multiple of 4."""
    P = make_problem((23, 19), 5, 4, 40, seed=4)
    prop = P.propagator()
    q = torch.from_numpy(P.q32).cuda()
    d1 = prop.forward(P.dt, 1, P.src_xyz, q[:1].contiguous(), P.rec_xyz)
    torch.cuda.synchronize()
    assert d1.shape == (1, P.rec_xyz.shape[0]) and torch.all(d1 == 0)
    d0 = prop.forward(P.dt, P.nt, np.zeros((0, 2)), torch.zeros((P.nt, 0), device="cuda"), P.rec_xyz)
    assert torch.all(d0 == 0)
    prop.forward(P.dt, P.nt, P.src_xyz, q, np.zeros((0, 2)))
    # source exactly on the last node of the computational grid and one in the layer
    ext = [(n - 1 + P.nbl) * h for n, h in zip(P.shape_phys, P.spacing)]
    src = np.array([ext, [-P.nbl * P.spacing[0] * 0.5, 33.3]])
    q2 = np.tile(P.q32[:, :1], (1, 2))
    import oracle
    d = prop.forward(P.dt, P.nt, src, torch.from_numpy(q2).cuda(), P.rec_xyz).cpu().numpy()
    d_ref = oracle.forward(P.grid(), P.m64(), P.eta(), P.dt, P.nt, P.pts(src), q2.astype(np.float64),
                           P.pts(P.rec_xyz))
    check_record(d, d_ref, label="edge sources")


@pytest.mark.parametrize("ndim", [2, 3])
def test_anisotropic_spacing_origin_and_damping_options(ndim):
    """Different spacing per axis, a shifted origin, R = 1e-4 and a linear
    damping profile (eta_power 1), order 6; forward and adjoint vs oracle."""
    import oracle
    from paper_1808_01995_amd import Propagator
    from synthetic import ricker, smooth_random_velocity
    shape = (41, 35) if ndim == 2 else (27, 22, 31)
    h = (10.0, 7.5) if ndim == 2 else (10.0, 12.5, 7.5)
    origin = (250.0, -40.0) if ndim == 2 else (250.0, 1000.0, -40.0)
    nbl, k, R, pw = 7, 6, 1e-4, 1
    v = smooth_random_velocity(shape, 11, sigma=4.0, vmin=1.6, vmax=3.0)
    m32 = (1.0 / oracle.pad_edge(v, nbl) ** 2).astype(np.float32)
    vmax = float(v.max())
    dt = 0.5 * oracle.critical_dt(ndim, h, k, vmax)
    nt = 121
    ext = [(n - 1) * hh for n, hh in zip(shape, h)]
    rel_src = np.array([[e * 0.43 for e in ext[:-1]] + [17.0]])
    rng = np.random.default_rng(12)
    rel_rec = np.stack([rng.uniform(-nbl * h[a] * 0.5, ext[a] + nbl * h[a] * 0.5, 30) for a in range(ndim - 1)]
                       + [np.full(30, 21.0)], axis=1)
    q = ricker(nt, dt, 18.0)[:, None].astype(np.float32)
    prop = Propagator(m=torch.from_numpy(m32).cuda(), shape=shape, spacing=h, nbl=nbl, space_order=k,
                      c_ref=vmax, origin=origin, R=R, eta_power=pw)
    off = np.array(origin)
    d = prop.forward(dt, nt, rel_src + off, torch.from_numpy(q).cuda(), rel_rec + off).cpu().numpy()
    g = oracle.Grid(m32.shape, h, k)
    eta = oracle.damping_eta(shape, nbl, h, vmax, R=R, power=pw)
    ps = oracle.sparse_points(rel_src, h, nbl, m32.shape)
    pr = oracle.sparse_points(rel_rec, h, nbl, m32.shape)
    d_ref = oracle.forward(g, m32.astype(np.float64), eta, dt, nt, ps, q.astype(np.float64), pr)
    check_record(d, d_ref, label="anisotropic %dD forward" % ndim)
    y = noise(nt, 30, dt, 18.0, 4)
    x = prop.adjoint(dt, nt, rel_rec + off, torch.from_numpy(y.astype(np.float32)).cuda(),
                     rel_src + off).cpu().numpy()
    x_ref = oracle.adjoint(g, m32.astype(np.float64), eta, dt, nt, pr, y.astype(np.float32).astype(np.float64), ps)
    check_record(x, x_ref, label="anisotropic %dD adjoint" % ndim)


def test_host_side_rejections():
    """CFL, domain and shape errors are reported before any work is queued."""
    from paper_1808_01995_amd import WaveFDError, _abi
    P = make_problem((20, 22), 4, 8, 10, seed=5)
    prop = P.propagator()
    q = torch.from_numpy(P.q32).cuda()
    dcrit = prop.critical_dt()
    with pytest.raises(WaveFDError) as e:
        prop.forward(dcrit * 1.01, P.nt, P.src_xyz, q, P.rec_xyz)
    assert e.value.status == _abi.WF_E_CFL
    with pytest.raises(WaveFDError) as e:
        prop.forward(P.dt, P.nt, np.array([[-1000.0, 50.0]]), q, P.rec_xyz)
    assert e.value.status == _abi.WF_E_DOMAIN
    bad = P.m32.copy()
    bad[3, 3] = -1.0
    with pytest.raises(WaveFDError) as e:
        P.propagator(bad)
    assert e.value.status == _abi.WF_E_ARG


def test_c2_full_size_against_stored_oracle_record():
    """The 3D order-8 workload at full size (336^3 computational, 1000 updates,
    the launch configuration the benchmark times) against the FP64 oracle's
    record at every 8th receiver in x and y (written by
    tests/golden/make_golden.py, which calls only the oracle)."""
    import os
    from synthetic import config, ricker
    path = os.path.join(os.path.dirname(__file__), "golden", "c2_so8_record_sampled.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle record not generated")
    gold = np.load(path)
    c = config("c2_3d_so8")
    v = c.velocity()
    import oracle
    m32 = (1.0 / oracle.pad_edge(v, c.nbl) ** 2).astype(np.float32)
    dt = float(gold["dt"])
    assert abs(dt - c.dt_factor * oracle.critical_dt(3, c.spacing, 8, float(v.max()))) < 1e-15
    from paper_1808_01995_amd import Propagator
    prop = Propagator(m=torch.from_numpy(m32).cuda(), shape=c.shape, spacing=c.spacing, nbl=c.nbl,
                      space_order=8, c_ref=float(v.max()))
    q = torch.from_numpy(ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32)).cuda()
    d = prop.forward(dt, c.nt, c.src, q, c.rec).cpu().numpy()
    sel = gold["receiver_index"]
    # 1000 updates: every trace carries an FP32 error of about the record's
    # rel. L2 times the RMS trace (measured up to 1.1 x 1.05e-5 on traces at
    # 0.1 of the RMS), so the relative-to-itself bound applies down to 0.3
    # of the RMS trace and the absolute one (3e-5 of it) below
    check_record(d[:, sel], gold["record"], weak=0.3, label="C2 full size, every 8th receiver in x and y")
    prop.close()


@pytest.mark.parametrize("shape,k", [((37, 29, 41), 16), ((33, 27, 130), 8), ((57, 49), 8)])
def test_ghost_region_stays_zero(shape, k):
    """No kernel writes outside the grid: after forward (with saved fields),
    adjoint, gradients (store-all, revolve, boundary reconstruction) and Born
    modelling, the ghost planes and row padding of the model's fields and of
    its clean gradient workspace still hold only zeros."""
    from _harness import noise
    from paper_1808_01995_amd import _abi
    P = make_problem(shape, 7, k, 40, seed=90 + k, nsrc=3, nrec=37)
    prop = P.propagator()
    q = torch.from_numpy(P.q32).cuda()
    ghosts = lambda: _abi.wf_model_ghost_nonzero(prop.handle)   # noqa: E731
    assert ghosts() == 0
    d, u = prop.forward(P.dt, P.nt, P.src_xyz, q, P.rec_xyz, save_every=7)
    assert ghosts() == 0
    r = torch.from_numpy(noise(P.nt, P.rec_xyz.shape[0], P.dt, 15.0, 3).astype(np.float32)).cuda()
    prop.adjoint(P.dt, P.nt, P.rec_xyz, r, P.src_xyz)
    assert ghosts() == 0
    g_all = prop.gradient(P.dt, P.nt, P.src_xyz, q, P.rec_xyz, r, n_checkpoints=-1)
    assert ghosts() == 0
    g_rev = prop.gradient(P.dt, P.nt, P.src_xyz, q, P.rec_xyz, r, n_checkpoints=3)
    assert ghosts() == 0 and torch.equal(g_rev, g_all)
    prop.gradient(P.dt, P.nt, P.src_xyz, q, P.rec_xyz, r, n_checkpoints=-2)
    assert ghosts() == 0          # its slabs occupy workspace slots: those are not checked
    prop.gradient(P.dt, P.nt, P.src_xyz, q, P.rec_xyz, r, n_checkpoints=-1)
    assert ghosts() == 0          # cleared again, every slot checked
    dm = torch.full(prop.comp_shape, 1e-3, device="cuda")
    prop.born(P.dt, P.nt, P.src_xyz, q, dm, P.rec_xyz)
    assert ghosts() == 0
    prop.close()


def test_validation_reports_nonfinite_outputs():
    """With validation on, a NaN in a wavelet, an Inf in a residual or a NaN
    in dm makes the call return WF_E_NONFINITE; off, the same calls succeed
    and their outputs carry the non-finite values; finite inputs pass."""
    from paper_1808_01995_amd import WaveFDError, _abi
    P = make_problem((30, 27), 6, 8, 60, seed=12, nrec=25)
    prop = P.propagator()
    q = torch.from_numpy(P.q32).cuda()
    qbad = q.clone()
    qbad[10, 0] = float("nan")
    rbad = torch.zeros((P.nt, P.rec_xyz.shape[0]), device="cuda")
    rbad[30, 3] = float("inf")
    dmbad = torch.zeros(prop.comp_shape, device="cuda")
    dmbad[9, 9] = float("nan")
    try:
        _abi.wf_validate_enable(True)
        d = prop.forward(P.dt, P.nt, P.src_xyz, q, P.rec_xyz)   # finite: passes
        r = (0.1 * d).contiguous()
        prop.gradient(P.dt, P.nt, P.src_xyz, q, P.rec_xyz, r)
        prop.adjoint(P.dt, P.nt, P.rec_xyz, r, P.src_xyz)
        calls = [lambda: prop.forward(P.dt, P.nt, P.src_xyz, qbad, P.rec_xyz),
                 lambda: prop.adjoint(P.dt, P.nt, P.rec_xyz, rbad, P.src_xyz),
                 lambda: prop.gradient(P.dt, P.nt, P.src_xyz, q, P.rec_xyz, rbad),
                 lambda: prop.born(P.dt, P.nt, P.src_xyz, q, dmbad, P.rec_xyz),
                 lambda: prop.fwi_gradient(P.dt, P.nt, [(P.src_xyz, qbad, P.rec_xyz, d)])]
        for call in calls:
            with pytest.raises(WaveFDError) as e:
                call()
            assert e.value.status == _abi.WF_E_NONFINITE
    finally:
        _abi.wf_validate_enable(False)
    d_nan = prop.forward(P.dt, P.nt, P.src_xyz, qbad, P.rec_xyz)
    torch.cuda.synchronize()
    assert not torch.isfinite(d_nan).all()
    prop.close()


def test_calls_follow_the_callers_stream():
    """Work is enqueued on torch's current stream: inputs produced and outputs
    consumed by torch on a side stream (default priority), with no
    synchronisation in between, give the default stream's results."""
    from _harness import noise
    P = make_problem((34, 29, 31), 6, 8, 50, seed=33, nrec=30)
    prop = P.propagator()
    q = torch.from_numpy(P.q32).cuda()
    y = torch.from_numpy(noise(P.nt, 30, P.dt, 15.0, 4).astype(np.float32)).cuda()
    d_ref = prop.forward(P.dt, P.nt, P.src_xyz, 2.0 * q, P.rec_xyz) * 3.0
    g_ref = prop.gradient(P.dt, P.nt, P.src_xyz, q, P.rec_xyz, (0.5 * y).contiguous()) + 1.0
    x_ref = prop.adjoint(P.dt, P.nt, P.rec_xyz, y, P.src_xyz)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        q2 = 2.0 * q                       # produced on the side stream
        d = prop.forward(P.dt, P.nt, P.src_xyz, q2, P.rec_xyz) * 3.0
        y2 = (0.5 * y).contiguous()
        g = prop.gradient(P.dt, P.nt, P.src_xyz, q, P.rec_xyz, y2) + 1.0
        x = prop.adjoint(P.dt, P.nt, P.rec_xyz, y, P.src_xyz)
    side.synchronize()
    assert torch.equal(d, d_ref) and torch.equal(g, g_ref) and torch.equal(x, x_ref)
    prop.close()


def test_one_model_on_two_streams_in_turn():
    """A model used on one stream and then at once on another (no host
    synchronisation, the inputs ready on both) orders the second call after
    the first: both records equal those of calls made one after the other
    on one stream."""
    P = make_problem((40, 33, 37), 6, 8, 70, seed=35, nrec=30)
    prop = P.propagator()
    q1 = torch.from_numpy(P.q32).cuda()
    q2 = (-0.5 * q1).contiguous()
    ref1 = prop.forward(P.dt, P.nt, P.src_xyz, q1, P.rec_xyz)
    ref2 = prop.forward(P.dt, P.nt, P.src_xyz, q2, P.rec_xyz)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    for _ in range(3):
        d1 = prop.forward(P.dt, P.nt, P.src_xyz, q1, P.rec_xyz)            # default stream
        with torch.cuda.stream(side):
            d2 = prop.forward(P.dt, P.nt, P.src_xyz, q2, P.rec_xyz)        # at once, on the side
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        assert torch.equal(d1, ref1) and torch.equal(d2, ref2)
    prop.close()
