"""Serving engine (continuous batching): every result is the same alone and
in the mix (bitwise), matches the plain propagator and the oracle, admission
never exceeds the HBM budget, requests arriving while others run are admitted
and overlap, and an invalid request is rejected without disturbing the rest."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _specs():
    return [
        {"ndim": 2, "n": 120, "space_order": 4, "steps": 150, "kind": "forward", "seed": 11},
        {"ndim": 2, "n": 200, "space_order": 8, "steps": 90, "kind": "forward", "seed": 12},
        {"ndim": 2, "n": 96, "space_order": 12, "steps": 220, "kind": "forward", "seed": 13},
        {"ndim": 3, "n": 40, "space_order": 8, "steps": 70, "kind": "forward", "seed": 14},
        {"ndim": 2, "n": 80, "space_order": 8, "steps": 60, "kind": "gradient", "seed": 15, "perturb": 0.05},
        {"ndim": 3, "n": 30, "space_order": 4, "steps": 45, "kind": "gradient", "seed": 16, "perturb": 0.05},
    ]


def _build(specs, nbl=12):
    from paper_1808_01995_amd.serve import build_request
    return [build_request(s, nbl=nbl) for s in specs]


def _results(reqs):
    out = []
    for r in reqs:
        out.append((r.rec_out.clone(), None if r.grad_out is None else r.grad_out.clone(), r.misfit))
    return out


def test_mix_equals_alone_and_plain_propagator():
    from paper_1808_01995_amd.serve import Server, run_one_shot_baseline, run_stream
    reqs = _build(_specs())
    srv = Server(hbm_budget_bytes=2 << 30, max_slots=16)
    st = run_stream(srv, reqs)
    assert st["failed"] == 0
    mixed = _results(reqs)
    # each alone
    for i, r in enumerate(reqs):
        r.rec_out.zero_()
        if r.grad_out is not None:
            r.grad_out.zero_()
        run_stream(srv, [r])
        assert r.status == 0
        d, g, phi = _results([r])[0]
        assert torch.equal(d, mixed[i][0]), i
        if g is not None:
            assert torch.equal(g, mixed[i][1]), i
            assert phi == mixed[i][2]
    srv.close()
    # the plain propagator, one shot at a time
    base = run_one_shot_baseline(reqs)
    for i, (d, g) in enumerate(base["outputs"]):
        rel = float((d - mixed[i][0]).norm() / d.norm())
        assert rel <= 1e-6, (i, rel)
        if g is not None:
            relg = float((g - mixed[i][1]).norm() / g.norm())
            assert relg <= 1e-5, (i, relg)


def test_small_request_matches_oracle():
    import oracle
    from paper_1808_01995_amd.serve import Server, build_request, run_stream
    spec = {"ndim": 2, "n": 70, "space_order": 8, "steps": 120, "kind": "forward", "seed": 21}
    r = build_request(spec, nbl=10)
    srv = Server(hbm_budget_bytes=1 << 30, max_slots=4)
    run_stream(srv, [r])
    srv.close()
    g = r.geom
    shape = (g.n[0] + 2 * g.nbl, g.n[1] + 2 * g.nbl)
    m = r.m.cpu().numpy().astype(np.float64)
    og = oracle.Grid(shape, (g.h[0], g.h[1]), g.space_order)
    eta = oracle.damping_eta((g.n[0], g.n[1]), g.nbl, (g.h[0], g.h[1]), g.c_ref)
    ps = oracle.sparse_points(r.src_xyz, (g.h[0], g.h[1]), g.nbl, shape)
    pr = oracle.sparse_points(r.rec_xyz, (g.h[0], g.h[1]), g.nbl, shape)
    d_ref = oracle.forward(og, m, eta, r.dt, r.nt, ps, r.src_wav.cpu().numpy().astype(np.float64), pr)
    d = r.rec_out.cpu().numpy()
    from _harness import check_record
    check_record(d, d_ref, label="served 2D request")


def test_budget_admission_and_overlap():
    from paper_1808_01995_amd.serve import Server, run_stream
    specs = [{"ndim": 2, "n": 300, "space_order": 8, "steps": 400, "kind": "forward", "seed": 30 + i}
             for i in range(8)]
    reqs = _build(specs, nbl=20)
    # a budget that holds only a few of these at once
    budget = 96 << 20
    srv = Server(hbm_budget_bytes=budget, max_slots=64)
    peak = 0
    for r in reqs:
        srv.submit(r)
    while srv.inflight:
        srv.poll(wait_ms=2)
        s = srv.stats()
        peak = max(peak, s["bytes_in_use"])
        assert s["bytes_in_use"] <= budget
    assert all(r.status == 0 for r in reqs)
    # a short request arriving while a long one runs finishes first (the long
    # one is sized to run far longer than the 20 ms head start)
    long_r = _build([{"ndim": 2, "n": 400, "space_order": 8, "steps": 12000, "kind": "forward", "seed": 40}],
                    nbl=20)[0]
    short_r = _build([{"ndim": 2, "n": 100, "space_order": 4, "steps": 60, "kind": "forward", "seed": 41}],
                     nbl=20)[0]
    srv.submit(long_r)
    time.sleep(0.02)
    srv.submit(short_r)
    srv.drain()
    assert short_r.done < long_r.done
    srv.close()
    assert peak > 0


def test_invalid_request_rejected_without_disturbing():
    from paper_1808_01995_amd import WaveFDError, _abi
    from paper_1808_01995_amd.serve import Server
    reqs = _build(_specs()[:3])
    srv = Server(hbm_budget_bytes=1 << 30, max_slots=8)
    t = [srv.submit(r) for r in reqs[:2]]
    bad = reqs[2]
    bad.geom.space_order = 5
    with pytest.raises(WaveFDError) as e:
        srv.submit(bad)
    assert e.value.status == _abi.WF_E_ARG
    srv.inflight.pop(None, None)
    huge = _build([{"ndim": 2, "n": 100, "space_order": 4, "steps": 20, "kind": "forward", "seed": 50}])[0]
    srv2 = Server(hbm_budget_bytes=64 << 20, max_slots=2)
    huge.geom.n[0] = 20000
    huge.geom.n[1] = 20000
    with pytest.raises(WaveFDError) as e:
        srv2.submit(huge)
    assert e.value.status == _abi.WF_E_BUDGET
    srv2.close()
    srv.drain()
    assert all(r.status == 0 for r in reqs[:2])
    srv.close()


def test_gradient_checkpoints_in_a_quarter_of_the_budget():
    """A gradient request whose forward fields do not fit in a quarter of the
    engine budget runs with revolve checkpoints in that quarter; the
    one-shot baseline's memory rule gives the plain propagator the same
    schedule. Both gradients and misfits equal the store-all gradient of the
    plain propagator bitwise (the result does not depend on the schedule)."""
    from paper_1808_01995_amd import Propagator, _abi
    from paper_1808_01995_amd.serve import Server, gradient_memory, run_stream
    spec = {"ndim": 2, "n": 200, "space_order": 8, "steps": 1000, "kind": "gradient", "seed": 61,
            "perturb": 0.05}
    r = _build([spec], nbl=20)[0]
    budget = 256 << 20
    nd = r.geom.ndim
    shape = tuple(r.geom.n[a] for a in range(nd))
    prop = Propagator(m=r.m, shape=shape, spacing=tuple(r.geom.h[a] for a in range(nd)), nbl=r.geom.nbl,
                      space_order=r.geom.space_order, c_ref=r.geom.c_ref)
    fields = r.nt * prop.npoints * 4
    assert fields > budget // 4 and fields < budget   # store-all fits the budget, not the share
    shot = [(r.src_xyz, r.src_wav, r.rec_xyz, r.d_obs)]
    phi_all, g_all = prop.fwi_gradient(r.dt, r.nt, shot, n_checkpoints=-1)
    nck, cap = gradient_memory(budget, prop.npoints, r.nt, r.rec_xyz.shape[0])
    assert nck == 0 and cap < fields
    phi_b, g_b = prop.fwi_gradient(r.dt, r.nt, shot, n_checkpoints=nck, hbm_budget_bytes=cap)
    assert torch.equal(g_b, g_all) and phi_b == phi_all
    prop.close()
    srv = Server(hbm_budget_bytes=budget, max_slots=4)
    run_stream(srv, [r])
    srv.close()
    assert r.status == 0
    assert torch.equal(r.grad_out, g_all)
    assert r.misfit == phi_all


def test_one_sample_requests():
    """Requests with a one-sample record (no update): the engine completes
    them with a zero record and, for a gradient, a zero gradient and misfit
    1/2 |d_obs|^2 (d_obs of one sample is zero too)."""
    from paper_1808_01995_amd.serve import Server, run_stream
    specs = [{"ndim": 2, "n": 64, "space_order": 8, "steps": 0, "kind": "forward", "seed": 70},
             {"ndim": 3, "n": 20, "space_order": 4, "steps": 0, "kind": "forward", "seed": 71},
             {"ndim": 2, "n": 64, "space_order": 8, "steps": 0, "kind": "gradient", "seed": 72, "perturb": 0.05}]
    reqs = _build(specs, nbl=6)
    for r in reqs:
        r.rec_out.fill_(1.0)
        if r.grad_out is not None:
            r.grad_out.fill_(1.0)
    srv = Server(hbm_budget_bytes=1 << 30, max_slots=4)
    st = run_stream(srv, reqs)
    srv.close()
    assert st["failed"] == 0
    for r in reqs:
        assert r.nt == 1 and torch.all(r.rec_out == 0)
        if r.grad_out is not None:
            assert torch.all(r.grad_out == 0) and r.misfit == 0.0


def test_heavy_requests_match_plain_propagator():
    """Grids above the batching limit (5 M nodes) run on the workers, one at
    a time while the next is set up: three of them (two forward shots, one
    gradient) among small requests give the plain propagator's results."""
    from paper_1808_01995_amd.serve import Server, run_one_shot_baseline, run_stream
    specs = [{"ndim": 3, "n": 176, "space_order": 8, "steps": 25, "kind": "forward", "seed": 80},
             {"ndim": 2, "n": 150, "space_order": 4, "steps": 60, "kind": "forward", "seed": 81},
             {"ndim": 3, "n": 180, "space_order": 4, "steps": 20, "kind": "gradient", "seed": 82, "perturb": 0.05},
             {"ndim": 3, "n": 190, "space_order": 12, "steps": 15, "kind": "forward", "seed": 83},
             {"ndim": 2, "n": 120, "space_order": 8, "steps": 40, "kind": "gradient", "seed": 84, "perturb": 0.05}]
    reqs = _build(specs, nbl=12)
    assert sum(1 for r in reqs if r.m.numel() > (5 << 20)) == 3
    srv = Server(hbm_budget_bytes=24 << 30, max_slots=8)
    st = run_stream(srv, reqs)
    srv.close()
    assert st["failed"] == 0
    base = run_one_shot_baseline(reqs, 24 << 30)
    for i, (r, (d, g)) in enumerate(zip(reqs, base["outputs"])):
        assert torch.equal(r.rec_out, d), i
        if g is not None:
            assert torch.equal(r.grad_out, g), i


def test_reservation_bounds_what_a_request_allocates():
    """An engine whose whole budget is one request's reservation serves it:
    the admission footprint (wf_engine_request_bytes) bounds what the request
    allocates, including the fused injection tables of a 64 x 64 receiver
    grid (4 increment slots per group of 4 z nodes), for forward and gradient
    requests in 2D and 3D."""
    from paper_1808_01995_amd import _abi
    from paper_1808_01995_amd.serve import Server, request_struct, run_stream
    specs = [{"ndim": 3, "n": 48, "space_order": 8, "steps": 300, "kind": "forward", "seed": 90},
             {"ndim": 3, "n": 40, "space_order": 4, "steps": 200, "kind": "gradient", "seed": 91, "perturb": 0.05},
             {"ndim": 2, "n": 300, "space_order": 12, "steps": 400, "kind": "gradient", "seed": 92, "perturb": 0.05},
             {"ndim": 2, "n": 500, "space_order": 8, "steps": 300, "kind": "forward", "seed": 93}]
    reqs = _build(specs, nbl=20)
    for r in reqs:
        q = request_struct(r)
        b1 = _abi.wf_engine_request_bytes(q, 1 << 40)
        b2 = _abi.wf_engine_request_bytes(q, b1)     # the reservation under a budget of b1
        assert b2 <= b1
        budget = max(b2, 64 << 20)
        srv = Server(hbm_budget_bytes=budget, max_slots=1)
        st = run_stream(srv, [r])
        srv.close()
        print("%s: reservation %.1f MB, served with a %.1f MB budget" % (r.tag, b2 / 1e6, budget / 1e6))
        assert st["failed"] == 0 and r.status == 0, r.tag


def test_submission_is_stream_ordered_and_admits_during_a_heavy_request():
    """Submission waits for nothing on the host: a request whose wavelet is
    produced on a side stream behind 50 ms of queued GPU work is submitted
    at once and served from the finished wavelet (bitwise the plain
    propagator's record for that wavelet); and a small request submitted
    while a heavy 3D request runs returns from submit at once and completes
    before the heavy one."""
    from paper_1808_01995_amd import Propagator
    from paper_1808_01995_amd.serve import Server
    heavy = _build([{"ndim": 3, "n": 300, "space_order": 8, "steps": 1500, "kind": "forward", "seed": 95}],
                   nbl=12)[0]
    small = _build([{"ndim": 2, "n": 100, "space_order": 8, "steps": 200, "kind": "forward", "seed": 96}],
                   nbl=12)[0]
    torch.cuda.synchronize()
    wav0 = small.src_wav.clone()
    srv = Server(hbm_budget_bytes=8 << 30, max_slots=8)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        torch.cuda._sleep(100_000_000)            # queued work ahead of the wavelet
        small.src_wav = (wav0 * 1.0).contiguous()  # written only after it
        t0 = time.perf_counter()
        srv.submit(small)
        t_small = time.perf_counter() - t0
    srv.drain()
    assert small.status == 0
    nd = small.geom.ndim
    prop = Propagator(m=small.m, shape=tuple(small.geom.n[a] for a in range(nd)),
                      spacing=tuple(small.geom.h[a] for a in range(nd)), nbl=small.geom.nbl,
                      space_order=small.geom.space_order, c_ref=small.geom.c_ref)
    ref = prop.forward(small.dt, small.nt, small.src_xyz, wav0, small.rec_xyz)
    torch.cuda.synchronize()
    prop.close()
    print("submit behind queued side-stream work returned in %.2f ms" % (t_small * 1e3))
    assert t_small < 0.02
    assert torch.equal(small.rec_out, ref)
    # a small request arriving while a heavy one runs
    small.rec_out.zero_()
    small.arrival = 0.0
    srv.submit(heavy)
    time.sleep(0.03)
    t0 = time.perf_counter()
    srv.submit(small)
    t_sub = time.perf_counter() - t0
    srv.drain()
    srv.close()
    print("heavy %.1f ms, small submitted after 30 ms in %.2f ms, done after %.1f ms"
          % ((heavy.done - heavy.arrival) * 1e3, t_sub * 1e3, (small.done - heavy.arrival) * 1e3))
    assert heavy.status == 0 and small.status == 0
    assert t_sub < 0.02
    assert small.done < heavy.done
    assert torch.equal(small.rec_out, ref)


def test_resident_teams_equal_batched_launches_plain_propagator_and_oracle():
    """Forward shots whose two wavefields fit one work-group's LDS run as
    resident teams (2D 141^2 order 4 twice; 2D 90^2 order 8; 2D 80^2 order
    12; 3D 26^3 order 8; submitted at once, so in launches of each order):
    every record equals the batched launches' (resident teams switched off)
    and the plain propagator's bit for bit, and the oracle's to the record
    bar."""
    import os
    import oracle
    from _harness import check_record
    from paper_1808_01995_amd.serve import Server, build_request, run_one_shot_baseline, run_stream
    specs = [({"ndim": 2, "n": 101, "space_order": 4, "steps": 300, "kind": "forward", "seed": 110}, 20),
             ({"ndim": 2, "n": 101, "space_order": 4, "steps": 240, "kind": "forward", "seed": 111}, 20),
             ({"ndim": 2, "n": 70, "space_order": 8, "steps": 200, "kind": "forward", "seed": 112}, 10),
             ({"ndim": 2, "n": 60, "space_order": 12, "steps": 180, "kind": "forward", "seed": 113}, 10),
             ({"ndim": 3, "n": 10, "space_order": 8, "steps": 120, "kind": "forward", "seed": 114}, 8)]
    reqs = [build_request(sp, nbl=nbl) for sp, nbl in specs]
    srv = Server(hbm_budget_bytes=2 << 30, max_slots=16)
    st = run_stream(srv, reqs)
    paths = srv.paths()
    srv.close()
    assert st["failed"] == 0 and paths["teams"] == len(reqs), paths
    teams = [r.rec_out.clone() for r in reqs]
    os.environ["WAVEFD_TEAMS"] = "0"
    try:
        srv = Server(hbm_budget_bytes=2 << 30, max_slots=16)
        for r in reqs:
            r.rec_out.fill_(float("nan"))
        st = run_stream(srv, reqs)
        paths = srv.paths()
        srv.close()
    finally:
        del os.environ["WAVEFD_TEAMS"]
    assert st["failed"] == 0 and paths["batched"] == len(reqs), paths
    base = run_one_shot_baseline(reqs)
    for i, (r, (d, _)) in enumerate(zip(reqs, base["outputs"])):
        assert torch.equal(teams[i], r.rec_out), i
        assert torch.equal(teams[i], d), i
    for i in (0, 4):
        r = reqs[i]
        g = r.geom
        nd = g.ndim
        h = tuple(g.h[a] for a in range(nd))
        shape = tuple(g.n[a] + 2 * g.nbl for a in range(nd))
        og = oracle.Grid(shape, h, g.space_order)
        eta = oracle.damping_eta(tuple(g.n[a] for a in range(nd)), g.nbl, h, g.c_ref)
        ps = oracle.sparse_points(r.src_xyz, h, g.nbl, shape)
        pr = oracle.sparse_points(r.rec_xyz, h, g.nbl, shape)
        d_ref = oracle.forward(og, r.m.cpu().numpy().astype(np.float64), eta, r.dt, r.nt, ps,
                               r.src_wav.cpu().numpy().astype(np.float64), pr)
        check_record(teams[i].cpu().numpy(), d_ref, label="resident team %dD order %d" % (nd, g.space_order))


def _with_points(r, src_xyz, rec_xyz, seed):
    """Replace a request's sources (Ricker wavelets with per-source scales)
    and receivers."""
    from synthetic import ricker
    r.src_xyz = np.asarray(src_xyz, dtype=np.float64)
    w = ricker(r.nt, r.dt, 10.0)[:, None] * np.linspace(1.0, 0.5, r.src_xyz.shape[0])[None, :]
    r.src_wav = torch.from_numpy(w.astype(np.float32)).cuda()
    r.rec_xyz = np.asarray(rec_xyz, dtype=np.float64)
    r.rec_out = torch.empty((r.nt, r.rec_xyz.shape[0]), dtype=torch.float32, device="cuda")
    return r


def test_resident_team_edge_cases_equal_other_paths():
    """Resident teams at the edges of what they take: 3D order 4 (512
    threads) and order 16 (256 threads), 2D order 16, one- and two-sample
    shots, three sources (one in the absorbing layer, one on the grid's last
    node) with a receiver on that node; and a grid one node past the LDS limit
    (142^2), which must go to the batched launches. Every record equals the
    run with resident teams switched off and the plain propagator bit for bit;
    the multi-source one also matches the oracle."""
    import os
    import oracle
    from _harness import check_record
    from paper_1808_01995_amd.serve import Server, build_request, run_one_shot_baseline, run_stream
    specs = [({"ndim": 3, "n": 14, "space_order": 4, "steps": 80, "kind": "forward", "seed": 120}, 6),
             ({"ndim": 3, "n": 6, "space_order": 16, "steps": 60, "kind": "forward", "seed": 121}, 8),
             ({"ndim": 2, "n": 60, "space_order": 16, "steps": 90, "kind": "forward", "seed": 122}, 10),
             ({"ndim": 2, "n": 101, "space_order": 4, "steps": 0, "kind": "forward", "seed": 123}, 20),
             ({"ndim": 2, "n": 101, "space_order": 4, "steps": 1, "kind": "forward", "seed": 124}, 20),
             ({"ndim": 2, "n": 70, "space_order": 8, "steps": 150, "kind": "forward", "seed": 125}, 10),
             ({"ndim": 2, "n": 102, "space_order": 4, "steps": 60, "kind": "forward", "seed": 126}, 20)]
    reqs = [build_request(sp, nbl=nbl) for sp, nbl in specs]
    multi = reqs[5]
    h, nbl = 10.0, 10
    last = (70 - 1 + nbl) * h
    _with_points(multi, [[345.0, 20.0], [-7.5 * h, 123.0], [last, last]],
                 np.vstack([np.stack([np.linspace(0.0, 690.0, 40), np.full(40, 30.0)], 1), [[last, last]]]), 125)
    srv = Server(hbm_budget_bytes=2 << 30, max_slots=16)
    st = run_stream(srv, reqs)
    paths = srv.paths()
    srv.close()
    assert st["failed"] == 0, [r.status for r in reqs]
    assert paths == {"teams": len(reqs) - 1, "batched": 1, "workers": 0}, paths
    teams = [r.rec_out.clone() for r in reqs]
    os.environ["WAVEFD_TEAMS"] = "0"
    try:
        srv = Server(hbm_budget_bytes=2 << 30, max_slots=16)
        for r in reqs:
            r.rec_out.fill_(float("nan"))
        st = run_stream(srv, reqs)
        srv.close()
    finally:
        del os.environ["WAVEFD_TEAMS"]
    assert st["failed"] == 0
    base = run_one_shot_baseline(reqs)
    for i, (r, (d, _)) in enumerate(zip(reqs, base["outputs"])):
        assert torch.equal(teams[i], r.rec_out), i
        assert torch.equal(teams[i], d), i
    assert torch.count_nonzero(teams[3]) == 0 and teams[3].shape[0] == 1
    g = multi.geom
    shape = (g.n[0] + 2 * g.nbl, g.n[1] + 2 * g.nbl)
    hh = (g.h[0], g.h[1])
    d_ref = oracle.forward(oracle.Grid(shape, hh, g.space_order), multi.m.cpu().numpy().astype(np.float64),
                           oracle.damping_eta((g.n[0], g.n[1]), g.nbl, hh, g.c_ref), multi.dt, multi.nt,
                           oracle.sparse_points(multi.src_xyz, hh, g.nbl, shape),
                           multi.src_wav.cpu().numpy().astype(np.float64),
                           oracle.sparse_points(multi.rec_xyz, hh, g.nbl, shape))
    check_record(teams[5].cpu().numpy(), d_ref, label="resident team, three sources")


def test_every_path_at_once_equals_one_at_a_time():
    """All three engine paths busy together: 48 tiny shots of 2D orders 4 /
    8 / 12 and 3D order 8 on resident teams (several launches in flight), six
    mid-size 2D grids on the batched launches, a 3D grid above the batching
    limit and two gradients on the workers, submitted at once and then in a
    second burst while the first still runs. Every record and gradient equals
    the one-shot run bit for bit, and each path served what it should."""
    from paper_1808_01995_amd.serve import Server, run_one_shot_baseline, run_stream
    tiny = [{"ndim": 2, "n": 60 + 7 * (i % 5), "space_order": (4, 8, 12)[i % 3], "steps": 40 + 9 * (i % 7),
             "kind": "forward", "seed": 400 + i} for i in range(40)]
    tiny += [{"ndim": 3, "n": 4 + (i % 3), "space_order": 8, "steps": 30 + 5 * i, "kind": "forward",
              "seed": 440 + i} for i in range(8)]
    mid = [{"ndim": 2, "n": 180 + 40 * i, "space_order": (4, 8, 12)[i % 3], "steps": 50, "kind": "forward",
            "seed": 460 + i} for i in range(6)]
    heavy = [{"ndim": 3, "n": 176, "space_order": 8, "steps": 20, "kind": "forward", "seed": 470},
             {"ndim": 2, "n": 90, "space_order": 8, "steps": 40, "kind": "gradient", "seed": 471, "perturb": 0.05},
             {"ndim": 3, "n": 24, "space_order": 4, "steps": 30, "kind": "gradient", "seed": 472, "perturb": 0.05}]
    specs = tiny[:24] + mid[:3] + heavy + tiny[24:] + mid[3:]
    reqs = _build(specs, nbl=10)
    arrivals = [0.0] * (24 + 3 + 3) + [0.004] * (24 + 3)
    srv = Server(hbm_budget_bytes=24 << 30, max_slots=96)
    st = run_stream(srv, reqs, arrivals)
    paths = srv.paths()
    srv.close()
    assert st["failed"] == 0, [r.status for r in reqs]
    assert paths == {"teams": 48, "batched": 6, "workers": 3}, paths
    base = run_one_shot_baseline(reqs, 24 << 30)
    for i, (r, (d, g)) in enumerate(zip(reqs, base["outputs"])):
        assert torch.equal(r.rec_out, d), (i, specs[i])
        if g is not None:
            assert torch.equal(r.grad_out, g), (i, specs[i])


def test_split_teams_equal_batched_launches_for_every_width_and_period():
    """Shots split over teams of W work-groups that exchange boundary planes
    every K updates (W = 2 / 4 / 8, K = 1 / 3 / as long as the parts allow,
    forced through WAVEFD_TEAM_WIDTH / WAVEFD_TEAM_PERIOD): 2D orders 4 and 8
    with sources and receivers across the part boundaries and 3D order 8
    records equal the batched launches bit for bit."""
    import os
    from paper_1808_01995_amd.serve import Server, build_request, run_stream
    specs = [({"ndim": 2, "n": 101, "space_order": 4, "steps": 70, "kind": "forward", "seed": 500}, 20),
             ({"ndim": 2, "n": 90, "space_order": 8, "steps": 55, "kind": "forward", "seed": 501}, 12),
             ({"ndim": 3, "n": 6, "space_order": 8, "steps": 40, "kind": "forward", "seed": 502}, 10)]
    reqs = [build_request(sp, nbl=nbl) for sp, nbl in specs]
    # sources on either side of the part boundaries of the 2D grids
    h = 10.0
    for r, (sp, nbl) in zip(reqs[:2], specs[:2]):
        n = sp["n"]
        last = (n - 1) * h
        xs = np.array([0.13, 0.249, 0.376, 0.5, 0.626, 0.751, 0.874]) * (n + 2 * nbl) * h - nbl * h
        _with_points(r, np.stack([xs, np.full(xs.size, 35.0)], 1),
                     np.stack([np.linspace(-nbl * h, last + nbl * h, 97), np.full(97, 25.0)], 1), 0)
    os.environ["WAVEFD_TEAMS"] = "0"
    try:
        srv = Server(hbm_budget_bytes=2 << 30, max_slots=8)
        st = run_stream(srv, reqs)
        srv.close()
    finally:
        del os.environ["WAVEFD_TEAMS"]
    assert st["failed"] == 0
    ref = [r.rec_out.clone() for r in reqs]
    for w in ("2", "4", "8"):
        for k in ("1", "3", "64"):
            os.environ["WAVEFD_TEAM_WIDTH"], os.environ["WAVEFD_TEAM_PERIOD"] = w, k
            try:
                srv = Server(hbm_budget_bytes=2 << 30, max_slots=8)
                for r in reqs:
                    r.rec_out.fill_(float("nan"))
                for r in reqs:   # one at a time: each launch may split
                    st = run_stream(srv, [r])
                    assert st["failed"] == 0, (w, k)
                paths = srv.paths()
                srv.close()
            finally:
                del os.environ["WAVEFD_TEAM_WIDTH"], os.environ["WAVEFD_TEAM_PERIOD"]
            assert paths["teams"] == len(reqs), paths
            for i, r in enumerate(reqs):
                assert torch.equal(r.rec_out, ref[i]), (w, k, i)
