"""Captured time loops: repeated wf_forward / wf_adjoint calls with one
signature are launched as a HIP graph (captured on the second call, replayed
after). Every replay must equal the eager run bitwise, with other eager work
on the same model and stream between replays, and must follow in-place
changes of the inputs (wavelet, m) exactly as a fresh eager run does.
All buffers are explicit so that the signatures, and so the launch counts,
do not depend on the caching allocator. Capture is switched on for these
tests (it is off by default).
"""
import numpy as np
import pytest

from _harness import check_record, make_problem, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _abi():
    from paper_1808_01995_amd import _abi
    return _abi


@pytest.fixture(autouse=True)
def _graphs_on():
    _abi().wf_graph_enable(True)
    yield
    _abi().wf_graph_enable(False)


def _setup(shape, k, steps, seed):
    P = make_problem(shape, 8, k, steps, seed=seed, nrec=40)
    prop = P.propagator()
    q = torch.from_numpy(P.q32).cuda()
    rec = torch.empty((P.nt, P.rec_xyz.shape[0]), dtype=torch.float32, device="cuda")
    return P, prop, q, rec


def _launches(prop):
    return _abi().wf_model_graph_launches(prop.handle)


@pytest.mark.parametrize("shape,k,save", [((60, 50), 8, 0), ((60, 50), 4, 7),
                                          ((34, 30, 38), 8, 0), ((34, 30, 38), 12, 9)])
def test_forward_replays_equal_eager(shape, k, save):
    P, prop, q, rec = _setup(shape, k, 70, seed=3 + k)
    u = None
    if save:
        u = torch.empty(((P.nt - 1) // save + 1,) + prop.comp_shape, dtype=torch.float32,
                        device="cuda")

    def run():
        _abi().wf_forward(prop.handle, P.dt, P.nt, P.src_xyz, q, P.rec_xyz, rec, u, save or 1)

    # size the model's buffers for the adjoint and gradient work done between
    # replays below (a grown buffer changes the signature: no replay then)
    y0 = torch.ones_like(rec)
    xa = torch.empty((P.nt, P.src_xyz.shape[0]), dtype=torch.float32, device="cuda")
    g = torch.empty(prop.comp_shape, dtype=torch.float32, device="cuda")
    _abi().wf_adjoint(prop.handle, P.dt, P.nt, P.rec_xyz, y0, P.src_xyz, xa)
    _abi().wf_gradient(prop.handle, P.dt, P.nt, P.src_xyz, q, P.rec_xyz, y0, g, 3)
    n0 = _launches(prop)
    run()                                   # eager
    torch.cuda.synchronize()
    assert _launches(prop) == n0
    ref = rec.clone()
    uref = u.clone() if save else None
    check_record(ref.cpu().numpy(), P.oracle_forward(), label="eager loop")
    for i in range(4):                      # capture, then three replays
        rec.fill_(float("nan"))
        if save:
            u.fill_(float("nan"))
        run()
        if i == 1:   # eager work on the same model between replays
            _abi().wf_adjoint(prop.handle, P.dt, P.nt, P.rec_xyz, ref, P.src_xyz, xa)
        if i == 2:
            _abi().wf_gradient(prop.handle, P.dt, P.nt, P.src_xyz, q, P.rec_xyz, ref, g, 3)
        torch.cuda.synchronize()
        assert torch.equal(rec, ref), "replay %d differs" % i
        if save:
            assert torch.equal(u, uref), "saved fields of replay %d differ" % i
    assert _launches(prop) == n0 + 4


def test_forward_replay_follows_inputs():
    """Replays read the wavelet and m at launch time: in-place changes between
    calls give the same result as a fresh model run eagerly."""
    P, prop, q, rec = _setup((64, 48), 8, 80, seed=21)

    def run():
        _abi().wf_forward(prop.handle, P.dt, P.nt, P.src_xyz, q, P.rec_xyz, rec)

    run()
    run()                                   # captured
    n0 = _launches(prop)
    q.mul_(-0.5)
    q[10:20] += 0.25
    m2 = torch.from_numpy(P.m32).cuda() * 1.1
    prop.set_m(m2)
    run()                                   # replay on new inputs
    torch.cuda.synchronize()
    assert _launches(prop) == n0 + 1
    fresh = P.propagator(m32=m2.cpu().numpy())
    rec2 = torch.empty_like(rec)
    _abi().wf_forward(fresh.handle, P.dt, P.nt, P.src_xyz, q, P.rec_xyz, rec2)
    torch.cuda.synchronize()
    assert _launches(fresh) == 0
    assert torch.equal(rec, rec2)
    assert not torch.equal(rec, torch.zeros_like(rec))


@pytest.mark.parametrize("shape", [(60, 50), (34, 30, 38)])
def test_adjoint_replays_equal_eager(shape):
    P, prop, q, rec = _setup(shape, 8, 60, seed=31)
    y = torch.from_numpy(np.random.default_rng(5).standard_normal(
        (P.nt, P.rec_xyz.shape[0])).astype(np.float32)).cuda()
    x = torch.empty((P.nt, P.src_xyz.shape[0]), dtype=torch.float32, device="cuda")

    def run():
        _abi().wf_adjoint(prop.handle, P.dt, P.nt, P.rec_xyz, y, P.src_xyz, x)

    run()
    torch.cuda.synchronize()
    ref = x.clone()
    n0 = _launches(prop)
    d_prev = None
    for i in range(4):
        x.fill_(float("nan"))
        run()
        # a forward on the same model between the adjoint calls
        rec.fill_(float("nan"))
        _abi().wf_forward(prop.handle, P.dt, P.nt, P.src_xyz, q, P.rec_xyz, rec)
        torch.cuda.synchronize()
        assert torch.equal(x, ref), "replay %d differs" % i
        if d_prev is not None:
            assert torch.equal(rec, d_prev)
        d_prev = rec.clone()
    # adjoint: captured at once (its signature ran just before), then three
    # replays; forward: eager, captured, two replays
    assert _launches(prop) == n0 + 7


def test_graph_cache_eviction():
    """Six output buffers in turn: each signature is captured on its second
    call, at most four loops are kept, and every call gives the eager result."""
    P, prop, q, rec = _setup((50, 40), 6, 40, seed=41)
    bufs = [torch.empty_like(rec) for _ in range(6)]
    n0 = _launches(prop)
    outs = []
    for _pass in range(3):
        for b in bufs:
            b.fill_(float("nan"))
            _abi().wf_forward(prop.handle, P.dt, P.nt, P.src_xyz, q, P.rec_xyz, b)
            torch.cuda.synchronize()
            outs.append(b.clone())
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    # pass 0: eager; pass 1: six captures (evicting the two oldest);
    # pass 2: buffers 0, 1 evicted -> not cached; recent eager signatures
    # were consumed by their capture, so they run eagerly again and the LRU
    # loops 2..5 replay
    assert _launches(prop) == n0 + 6 + 4


def test_capture_off_runs_eagerly():
    """With capture switched off, repeated calls never launch a graph."""
    P, prop, q, rec = _setup((50, 40), 4, 30, seed=43)
    _abi().wf_graph_enable(False)
    n0 = _launches(prop)
    outs = []
    for _ in range(3):
        _abi().wf_forward(prop.handle, P.dt, P.nt, P.src_xyz, q, P.rec_xyz, rec)
        torch.cuda.synchronize()
        outs.append(rec.clone())
    assert _launches(prop) == n0
    assert torch.equal(outs[1], outs[0]) and torch.equal(outs[2], outs[0])
