"""Two updates per launch (3D forward and adjoint loops of space order 4 and 8).

The two-update kernel forms every node of u^{n+1} (on its tile extended by M
rows, 4 ceil(M/4) z nodes and M planes) and of u^{n+2} with the arithmetic of
the single-update kernel in the same order, so records and saved fields must
equal the one-update-per-launch loop bit for bit: compared here with torch.equal
for both orders, odd and even update counts, x chunks of every length the
planner picks, many sources scattered over tile, chunk and grid edges, and
more receivers than blocks. The same runs stay within the record bar of the
FP64 oracle, and the fields' ghost planes stay zero.
"""
import numpy as np
import pytest

from _harness import check_record, make_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _forward(P, two, prop=None, save_every=None, src=None, q=None, rec=None):
    from paper_1808_01995_amd import _abi
    prop = prop or P.propagator()
    src = P.src_xyz if src is None else src
    q = P.q32 if q is None else q
    rec = P.rec_xyz if rec is None else rec
    _abi.wf_two_step_enable(2 if two else 0)
    try:
        _abi.wf_profile_step_launches(0, reset=True)
        out = prop.forward(P.dt, P.nt, src, torch.from_numpy(q).cuda(), rec, save_every=save_every)
        torch.cuda.synchronize()
        n1 = _abi.wf_profile_step_launches(0)
        n2 = _abi.wf_profile_step_launches(_abi.WF_STEP_LAUNCHES_TWO)
    finally:
        _abi.wf_two_step_enable(1)
    return out, n1, n2


def _scatter_sources(P, n, seed):
    """n sources: random nodes and cell interiors, plus the grid's corners
    and points just inside the physical grid's faces."""
    rng = np.random.default_rng(seed)
    nd = len(P.shape_phys)
    h = np.asarray(P.spacing)
    lo = -P.nbl * h
    hi = (np.asarray(P.shape_phys) - 1 + P.nbl) * h
    pts = [rng.uniform(lo, hi) for _ in range(n - 4)]
    pts.append(lo.copy())                   # first node of the computational grid
    pts.append(hi.copy())                   # last node
    pts.append(np.zeros(nd))                # the physical grid's corner
    pts.append((np.asarray(P.shape_phys) - 1) * h - 0.3 * h)
    src = np.stack(pts)
    q = np.stack([np.sin(0.07 * (i + 1) * np.arange(P.nt)) * (1.0 + 0.1 * i) for i in range(n)], axis=1)
    return src, q.astype(np.float32)


@pytest.mark.parametrize("k", [4, 8])
@pytest.mark.parametrize("steps", [1, 2, 3, 8, 9])
def test_two_step_equals_one_update_per_launch(k, steps):
    """Records bitwise equal with two updates per launch and with one, for
    1 (no two-update launch), 2, 3, 8 and 9 updates; the launch counts show
    which kernel ran. 56 x 33 x 131 computational nodes at order 8 (2 z tiles,
    the second ragged; 3 y tiles, the last ragged; x chunks of a few planes)."""
    P = make_problem((40, 17, 115), 8, k, steps, seed=200 + k + steps, nrec=70)
    src, q = _scatter_sources(P, 24, seed=k + steps)
    rec = np.vstack([P.rec_xyz, src])   # receivers on the sources see every update
    prop = P.propagator()
    d2, n1a, n2a = _forward(P, True, prop=prop, src=src, q=q, rec=rec)
    d1, n1b, n2b = _forward(P, False, prop=prop, src=src, q=q, rec=rec)
    assert (n2a, n1a) == (steps // 2, steps % 2), (n2a, n1a)
    assert (n2b, n1b) == (0, steps), (n2b, n1b)
    assert torch.equal(d2, d1), float((d2 - d1).abs().max())
    if steps >= 2:   # q^0 = 0: u^1 is zero, u^2 is not at the sources
        assert float(d1[-1, P.rec_xyz.shape[0]:].abs().max()) > 0


@pytest.mark.parametrize("k", [4, 8])
def test_two_step_saved_fields_and_oracle(k):
    """Saved wavefields (every update and every third) bitwise equal to the
    one-update loop's, the record within the oracle's bar, and the model's
    ghost planes (those of the second field pair included) still zero."""
    from paper_1808_01995_amd import _abi
    P = make_problem((30, 22, 126), 6, k, 11, seed=230 + k, nrec=50)
    prop = P.propagator()
    for every in (1, 3):
        (d2, u2), _, n2 = _forward(P, True, prop=prop, save_every=every)
        (d1, u1), _, _ = _forward(P, False, prop=prop, save_every=every)
        assert n2 == 5
        assert torch.equal(d2, d1)
        assert torch.equal(u2, u1), float((u2 - u1).abs().max())
    check_record(d2.cpu().numpy(), P.oracle_forward(), label="two updates per launch, order %d" % k)
    assert _abi.wf_model_ghost_nonzero(prop.handle) == 0


def test_two_step_many_blocks_and_receivers():
    """A grid of many tiles in one or two chunks (100 x 120 x 250 nodes at
    order 8) with more receivers than blocks: records bitwise equal to the
    one-update loop's over 40 updates."""
    P = make_problem((84, 104, 234), 8, 8, 40, seed=251, nrec=900)
    src, q = _scatter_sources(P, 12, seed=9)
    prop = P.propagator()
    d2, _, n2 = _forward(P, True, prop=prop, src=src, q=q)
    d1, _, _ = _forward(P, False, prop=prop, src=src, q=q)
    assert n2 == 20
    assert torch.equal(d2, d1), float((d2 - d1).abs().max())


def test_two_step_off_for_other_orders():
    """Orders other than 4 and 8 keep one update per launch (2D and 3D)."""
    for shape, k in (((30, 20, 40), 12), ((60, 70), 12), ((60, 70), 16)):
        P = make_problem(shape, 6, k, 6, seed=270 + k, nrec=20)
        _, n1, n2 = _forward(P, True)
        assert (n1, n2) == (6, 0)


@pytest.mark.parametrize("k", [4, 8])
@pytest.mark.parametrize("steps", [1, 2, 7, 12])
def test_two_step_2d_equals_one_update_per_launch(k, steps):
    """2D rows of 504-node tiles: 40 x 1100 physical nodes (3 z tiles, the
    last ragged) with sources on tile, chunk and grid edges and more
    receivers than blocks; records bitwise equal to one update per launch,
    forward and adjoint; the forward record within the oracle's bar."""
    from _harness import noise
    P = make_problem((40, 1100), 8, k, steps, seed=350 + k + steps, nrec=300)
    src, q = _scatter_sources(P, 20, seed=k + steps)
    rec = np.vstack([P.rec_xyz, src])
    prop = P.propagator()
    d2, n1a, n2a = _forward(P, True, prop=prop, src=src, q=q, rec=rec)
    d1, n1b, n2b = _forward(P, False, prop=prop, src=src, q=q, rec=rec)
    assert (n2a, n1a) == (steps // 2, steps % 2), (n2a, n1a)
    assert torch.equal(d2, d1), float((d2 - d1).abs().max())
    y = noise(P.nt, rec.shape[0], P.dt, 15.0, 11 + steps).astype(np.float32)
    x2, m2 = _adjoint(P, True, prop, rec, y, src)
    x1, _ = _adjoint(P, False, prop, rec, y, src)
    assert m2 == steps // 2
    assert torch.equal(x2, x1), float((x2 - x1).abs().max())
    if steps == 12:
        check_record(d2.cpu().numpy(), _oracle_forward(P, src, q, rec),
                     label="2D two updates per launch, order %d" % k)


def _oracle_forward(P, src, q, rec):
    import oracle
    return oracle.forward(P.grid(), P.m64(), P.eta(), P.dt, P.nt, P.pts(src), q.astype(np.float64),
                          P.pts(rec))


def _adjoint(P, two, prop, rec, y, src):
    from paper_1808_01995_amd import _abi
    _abi.wf_two_step_enable(2 if two else 0)
    try:
        _abi.wf_profile_step_launches(0, reset=True)
        x = prop.adjoint(P.dt, P.nt, rec, torch.from_numpy(y).cuda(), src)
        torch.cuda.synchronize()
        n2 = _abi.wf_profile_step_launches(_abi.WF_STEP_LAUNCHES_TWO)
    finally:
        _abi.wf_two_step_enable(1)
    return x, n2


@pytest.mark.parametrize("k", [4, 8])
@pytest.mark.parametrize("steps", [2, 3, 10])
def test_two_step_adjoint_equals_one_update_per_launch(k, steps):
    """The adjoint loop (receivers injected, sources sampled, time reversed):
    bitwise equal with two updates per launch and with one, and within the
    record bar of the oracle's adjoint."""
    from _harness import noise
    P = make_problem((36, 19, 117), 8, k, steps, seed=290 + k + steps, nrec=40)
    src, _ = _scatter_sources(P, 16, seed=30 + k)
    rec = np.vstack([P.rec_xyz, src[:6]])
    y = noise(P.nt, rec.shape[0], P.dt, 15.0, 7 + steps).astype(np.float32)
    prop = P.propagator()
    x2, n2 = _adjoint(P, True, prop, rec, y, src)
    x1, n1 = _adjoint(P, False, prop, rec, y, src)
    assert (n2, n1) == (steps // 2, 0)
    assert torch.equal(x2, x1), float((x2 - x1).abs().max())
    assert float(x1.abs().max()) > 0
    if steps == 10:
        import oracle
        ref = oracle.adjoint(P.grid(), P.m64(), P.eta(), P.dt, P.nt, P.pts(rec), y.astype(np.float64),
                             P.pts(src))
        check_record(x2.cpu().numpy(), ref, label="adjoint, two updates per launch, order %d" % k)


@pytest.mark.parametrize("k", [4, 8])
def test_two_step_loops_replay_from_graphs(k):
    """With capture on, a forward and an adjoint loop of two-update launches
    are captured on their second call and replayed after; every replay,
    with other eager work on the model in between, equals the eager
    one-update-per-launch run bit for bit."""
    from _harness import noise
    from paper_1808_01995_amd import _abi
    P = make_problem((30, 20, 118), 6, k, 13, seed=310 + k, nrec=30)
    prop = P.propagator()
    q = torch.from_numpy(P.q32).cuda()
    y = torch.from_numpy(noise(P.nt, P.rec_xyz.shape[0], P.dt, 15.0, 3).astype(np.float32)).cuda()
    rec = torch.empty((P.nt, P.rec_xyz.shape[0]), dtype=torch.float32, device="cuda")
    xs = torch.empty((P.nt, P.src_xyz.shape[0]), dtype=torch.float32, device="cuda")

    def fwd():
        _abi.wf_forward(prop.handle, P.dt, P.nt, P.src_xyz, q, P.rec_xyz, rec)
        return rec.clone()

    def adj():
        _abi.wf_adjoint(prop.handle, P.dt, P.nt, P.rec_xyz, y, P.src_xyz, xs)
        return xs.clone()

    _abi.wf_two_step_enable(0)
    ref_f, ref_a = fwd(), adj()
    torch.cuda.synchronize()
    _abi.wf_two_step_enable(2)
    _abi.wf_graph_enable(True)
    try:
        # a first round sizes the model's increment buffers for both loops (a
        # grown buffer changes a loop's signature; the adjoint's receivers need
        # the larger ones, so it goes first) and runs eagerly
        a0 = adj()
        outs = [(fwd(), a0)]
        torch.cuda.synchronize()
        g0 = _abi.wf_model_graph_launches(prop.handle)
        for _ in range(3):
            outs.append((fwd(), adj()))
            torch.cuda.synchronize()
        launched = _abi.wf_model_graph_launches(prop.handle) - g0
    finally:
        _abi.wf_graph_enable(False)
        _abi.wf_two_step_enable(1)
    assert launched == 6, launched   # per loop: capture and launch, then two replays
    for f, a in outs:
        assert torch.equal(f, ref_f)
        assert torch.equal(a, ref_a)


@pytest.mark.parametrize("k", [4, 8])
@pytest.mark.parametrize("shape,nbl", [((3, 5, 7), 2),        # fewer planes, rows and columns than one tile
                                       ((6, 4, 112), 4),      # 120 z nodes: exactly one z tile
                                       ((12, 12, 232), 4),    # 240 z nodes: exactly two; 20 y rows
                                       ((2, 2, 2), 2)])       # 6 x 6 x 6 nodes
def test_two_step_small_and_exact_tile_grids(k, shape, nbl):
    """Degenerate and exact-fit shapes: grids smaller than one tile in every
    axis, z extents that fill whole 120-node tiles, y extents that fill whole
    tiles; sources on the first and last nodes. Records bitwise equal to one
    update per launch, for an odd and an even number of updates."""
    for steps in (5, 6):
        P = make_problem(shape, nbl, k, steps, seed=330 + k + steps, nrec=12)
        src, q = _scatter_sources(P, 6, seed=steps)
        rec = np.vstack([P.rec_xyz, src])
        prop = P.propagator()
        d2, _, n2 = _forward(P, True, prop=prop, src=src, q=q, rec=rec)
        d1, _, _ = _forward(P, False, prop=prop, src=src, q=q, rec=rec)
        assert n2 == steps // 2
        assert torch.equal(d2, d1), (shape, steps, float((d2 - d1).abs().max()))


def test_two_step_falls_back_when_points_crowd_a_block():
    """An adjoint whose 400 receivers crowd a few planes of one 2D row tile
    (more injection entries than a block of the two-update kernel stages)
    keeps one update per launch, with the same record."""
    from _harness import noise
    P = make_problem((40, 300), 8, 4, 8, seed=370, nrec=10)
    rng = np.random.default_rng(5)
    h = P.spacing[0]
    rec = np.stack([rng.uniform(150.0, 150.0 + 3 * h, 400), rng.uniform(0.0, 2900.0, 400)], axis=1)
    src = P.src_xyz
    y = noise(P.nt, rec.shape[0], P.dt, 15.0, 4).astype(np.float32)
    prop = P.propagator()
    x2, n2 = _adjoint(P, True, prop, rec, y, src)
    x1, _ = _adjoint(P, False, prop, rec, y, src)
    assert n2 == 0
    assert torch.equal(x2, x1)
    assert float(x1.abs().max()) > 0
