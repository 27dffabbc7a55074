#!/usr/bin/env python3
"""Benchmark of the gfx950 acoustic propagator.

One "step" of this benchmark is one complete forward shot of the 3D order-8
workload: 256^3 physical grid (336^3 with the 40-node damping layer), h = 10 m,
smooth random velocity 1.5-4.5 km/s, 1000 time updates at dt = 0.5 dt_crit,
one 15 Hz Ricker source at 20 m depth and 128 x 128 receivers at 20 m depth:
every update runs the fused stencil/damping/time-update kernel, the source
injection and the receiver interpolation. Inputs are resident in HBM before
the timed region.

Printed: one JSON line with the headline metric (grid-point updates per second
on the computational grid), the roofline of the dominant kernel (HBM bound,
16 algorithmic bytes per point per update against 8 TB/s) measured with HIP
events inside the timed region, the serving stream, short shots of the
workloads that run two updates per launch by default (592^3 and 8272^2 at
order 4, each also with one update per launch), and the FP64 oracle timed on
the host cores on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--extras]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_POINT = 16.0     # read u^n, u^{n-1}, kappa; write u^{n+1}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(os.path.join(ROOT, "paper_1808_01995_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profile(name: str, n_points: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def setup_c2(torch, space_order=8, steps=None):
    from paper_1808_01995_amd import Propagator
    from synthetic import config, ricker
    c = config("c2_3d_so8", space_order=space_order, steps=steps)
    v = c.velocity()
    prop = Propagator(v, spacing=c.spacing, nbl=c.nbl, space_order=c.space_order)
    dt = c.dt_factor * prop.critical_dt()
    q = torch.from_numpy(ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32)).cuda()
    rec_out = torch.empty((c.nt, c.rec.shape[0]), dtype=torch.float32, device="cuda")
    return c, v, prop, dt, q, rec_out


def cpu_baseline(c, v, dt, sample_steps: int):
    """The FP64 oracle (plain C + OpenMP, untuned) on the same grid and
    acquisition, first `sample_steps` updates of the shot."""
    import oracle
    from synthetic import ricker
    oracle.build()
    nt = sample_steps + 1
    m = 1.0 / oracle.pad_edge(v, c.nbl) ** 2
    g = oracle.Grid(m.shape, c.spacing, c.space_order)
    eta = oracle.damping_eta(c.shape, c.nbl, c.spacing, float(v.max()))
    src = oracle.sparse_points(c.src, c.spacing, c.nbl, m.shape)
    rec = oracle.sparse_points(c.rec, c.spacing, c.nbl, m.shape)
    q = ricker(nt, dt, c.f0_hz)[:, None]
    t = time.perf_counter()
    oracle.forward(g, m, eta, dt, nt, src, q, rec)
    el = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", 0) or os.cpu_count() or 1)
    out = {"value": m.size * sample_steps / el / 1e9, "unit": "GPts/s", "cores": cores,
           "kind": "oracle",
           "sample": "FP64 oracle, %d of %d updates of the same %s-point shot (%.1f s)"
                     % (sample_steps, c.steps, "x".join(map(str, m.shape)), el)}
    if sample_steps >= 10:
        # the same oracle on one core (a child process with one OpenMP thread)
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-one-core", "8"],
                           env=env, capture_output=True, text=True, timeout=300)
        lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
        if r.returncode == 0 and lines:
            one = json.loads(lines[-1])
            out["value_one_core"] = one["value"]
            out["sample_one_core"] = one["sample"]
    return out


def oracle_one_core(steps: int):
    """Child of cpu_baseline: the oracle with one OpenMP thread on the first
    `steps` updates of the 3D order-8 shot (no GPU use)."""
    from synthetic import config
    import oracle
    c = config("c2_3d_so8")
    v = c.velocity()
    dt = c.dt_factor * oracle.critical_dt(3, c.spacing, c.space_order, float(v.max()))
    r = cpu_baseline(c, v, dt, min(steps, 9))
    print(json.dumps({"value": r["value"], "sample": r["sample"].replace("FP64 oracle", "FP64 oracle, 1 thread")}),
          flush=True)


def _timed(torch, fn, reps=1):
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps, out


def graph_c1(torch, shots=20):
    """141^2 computational (101^2 + 20-node layer), order 4, 500 updates:
    the time loop launched kernel by kernel against the same loop replayed
    from its captured HIP graph (launch cost dominates at this size)."""
    from paper_1808_01995_amd import Propagator, _abi
    from synthetic import config, ricker
    c = config("c1_2d")
    v = c.velocity()
    prop = Propagator(v, spacing=c.spacing, nbl=c.nbl, space_order=c.space_order)
    dt = c.dt_factor * prop.critical_dt()
    q = torch.from_numpy(ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32)).cuda()
    rec = torch.empty((c.nt, c.rec.shape[0]), device="cuda")

    def shot():
        prop.forward(dt, c.nt, c.src, q, c.rec, rec_out=rec)

    res = {"workload": "C1: 141^2 computational, order 4, %d updates, 101 receivers" % c.steps,
           "note": "eager and graph: two updates per launch (the default for 2D order 4); "
                   "eager_one_update_per_launch: the same shots with one"}
    for mode, two in (("eager", 1), ("graph", 1), ("eager_one_update_per_launch", 0)):
        _abi.wf_two_step_enable(two)
        _abi.wf_graph_enable(mode == "graph")
        shot()
        shot()     # graph mode: captured here
        g0 = _abi.wf_model_graph_launches(prop.handle)
        el, _ = _timed(torch, shot, reps=shots)
        res[mode] = {"ms_per_shot": round(el * 1e3, 3), "us_per_update": round(el / c.steps * 1e6, 2),
                     "gpts": round(prop.npoints * c.steps / el / 1e9, 3),
                     "graph_launches": _abi.wf_model_graph_launches(prop.handle) - g0}
    _abi.wf_graph_enable(False)
    _abi.wf_two_step_enable(1)
    res["graph_speedup"] = round(res["eager"]["ms_per_shot"] / res["graph"]["ms_per_shot"], 2)
    prop.close()
    log("c1: %s" % res)
    return res


def c1_batch(torch, counts=(1, 8, 32, 256), steps=500):
    """C1-size forward shots (101^2 physical + 20-node layer = 141^2, order 4,
    500 updates, 101 receivers at 20 m, smooth random velocity) through the
    serving engine, N requests submitted together: on resident teams (each
    shot's fields held in one work-group's LDS for the whole shot) and, with
    those switched off, on batched step launches (all grids share every step
    launch); wall time from submission to the last completion, per grid and
    update, against the same shots one at a time on the plain propagator
    (one launch per update)."""
    import os
    from paper_1808_01995_amd.serve import Server, build_request, run_one_shot_baseline, run_stream
    specs = [{"ndim": 2, "n": 101, "space_order": 4, "steps": steps, "kind": "forward", "seed": 300 + i}
             for i in range(max(counts))]
    reqs = [build_request(s, nbl=20) for s in specs]
    torch.cuda.synchronize()
    base = run_one_shot_baseline(reqs[:8], 4 << 30)
    one = base["seconds"] / (8 * steps) * 1e6
    paths = {}
    for label, teams in (("resident_teams", "1"), ("batched_launches", "0")):
        os.environ["WAVEFD_TEAMS"] = teams
        try:
            srv = Server(hbm_budget_bytes=8 << 30, max_slots=max(counts))
        finally:
            del os.environ["WAVEFD_TEAMS"]
        run_stream(srv, reqs[:2])   # warm-up
        rows = []
        for n in counts:
            st = run_stream(srv, reqs[:n])
            rows.append({"grids": n, "makespan_ms": round(st["makespan_s"] * 1e3, 2),
                         "us_per_grid_update": round(st["makespan_s"] * 1e6 / (n * steps), 3),
                         "failed": st["failed"]})
            log("c1 %s %d: %s" % (label, n, rows[-1]))
        paths[label] = {"rows": rows, "requests_by_path": srv.paths()}
        srv.close()
    return {"workload": "141^2 computational (101^2 + 20-node layer), order 4, %d updates, 101 receivers; "
                        "engine makespan (model set-up included) per grid-update" % steps,
            "one_at_a_time_us_per_update": round(one, 3), "engine": paths}


def large_2d(torch, n=8192, orders=(4, 8, 12), steps=300):
    """Large 2D grids: n^2 physical + 40-node layer, v = 2 km/s, one source,
    256 receivers at 20 m; GPts/s and the step kernel's algorithmic bandwidth
    per update (the shot's run of step launches timed by one pair of HIP
    events). Where the default runs two updates per launch the same shot
    also runs with one, for comparison."""
    from paper_1808_01995_amd import Propagator, _abi
    from synthetic import ricker
    res = []
    for so in orders:
        prop = Propagator(np.full((n, n), 2.0, dtype=np.float32), spacing=(10.0, 10.0), nbl=40,
                          space_order=so)
        dt = 0.5 * prop.critical_dt()
        nt = steps + 1
        ext = (n - 1) * 10.0
        src = np.array([[ext / 2, 20.0]])
        rec = np.stack([np.linspace(0, ext, 256), np.full(256, 20.0)], 1)
        q = torch.from_numpy(ricker(nt, dt, 10.0)[:, None].astype(np.float32)).cuda()
        out = torch.empty((nt, 256), device="cuda")
        for mode in (1, 0):
            _abi.wf_two_step_enable(mode)
            prop.forward(dt, 21, src, q[:21].contiguous(), rec, rec_out=out[:21])
            _abi.wf_profile_read(_abi.WF_KERNEL_STEP_RUN, reset=True)
            _abi.wf_profile_runs_enable(True)
            el, _ = _timed(torch, lambda: prop.forward(dt, nt, src, q, rec, rec_out=out))
            _abi.wf_profile_runs_enable(False)
            ms1, n1 = _abi.wf_profile_read(_abi.WF_KERNEL_STEP_RUN)
            ms2, n2 = _abi.wf_profile_read(_abi.WF_KERNEL_STEP2_RUN, reset=True)
            us = (ms1 + ms2) / max(n1 + 2 * n2, 1) * 1e3
            gbs = BYTES_PER_POINT * prop.npoints / (us * 1e-6) / 1e9
            r = {"space_order": so, "gpts": round(prop.npoints * steps / el / 1e9, 1),
                 "updates_per_launch": 2 if n2 else 1,
                 "step_kernel_us": round(us, 1), "algorithmic_GBs": round(gbs),
                 "frac_8TBs": round(gbs / PEAK_HBM_GBS, 3)}
            if n2:
                two_us = ms2 / n2 * 1e3
                r.update({"step_kernel_us_note": "per update; 16 B per node per update",
                          "two_update_launch_us": round(two_us, 1),
                          "two_update_frac_8TBs": round(20.0 * prop.npoints / (two_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 3)})
            res.append(r)
            log("2d %d so%d: %s" % (n, so, res[-1]))
            if not n2:
                break
        _abi.wf_two_step_enable(1)
        prop.close()
    return {"workload": "%d^2 physical (%d^2 computational), %d updates" % (n, n + 80, steps), "orders": res}


def slab_share(torch, ngpu=8, steps=300, so=8):
    """One GPU's share of the 592^3 grid split into x-slabs over `ngpu` GPUs:
    592/ngpu planes plus M halo planes on each side (the planes a neighbour
    would send each update), at the real shape; the step kernel's time per
    update against the time the halo faces would take over one xGMI link."""
    from paper_1808_01995_amd import Propagator, _abi
    from synthetic import ricker
    half = so // 2
    nx = 592 // ngpu + 2 * half
    shape = (nx, 592, 592)
    prop = Propagator(np.full(shape, 2.0, dtype=np.float32), spacing=(10.0,) * 3, nbl=0, space_order=so)
    dt = 0.5 * prop.critical_dt()
    nt = steps + 1
    src = np.array([[nx * 5.0, 2955.0, 20.0]])
    rec = np.stack([np.full(512, nx * 5.0), np.linspace(0, 5910, 512), np.full(512, 20.0)], 1)
    q = torch.from_numpy(ricker(nt, dt, 15.0)[:, None].astype(np.float32)).cuda()
    out = torch.empty((nt, 512), device="cuda")
    prop.forward(dt, 21, src, q[:21].contiguous(), rec, rec_out=out[:21])
    _abi.wf_profile_read(0, reset=True)
    _abi.wf_profile_enable(4)
    el, _ = _timed(torch, lambda: prop.forward(dt, nt, src, q, rec, rec_out=out))
    _abi.wf_profile_enable(False)
    ms, k = _abi.wf_profile_read(0, reset=True)
    us = ms / max(k, 1) * 1e3
    face = half * 592 * 592 * 4
    res = {"workload": "x-slab of 592^3 for %d GPUs: %dx592x592 nodes (%d planes + 2 x %d halo planes), order %d"
                       % (ngpu, nx, 592 // ngpu, half, so),
           "step_kernel_us": round(us, 1), "us_per_update": round(el / steps * 1e6, 1),
           "frac_8TBs": round(BYTES_PER_POINT * prop.npoints / (us * 1e-6) / 1e9 / PEAK_HBM_GBS, 3),
           "halo_face_MB": round(face / 1e6, 2),
           "face_transfer_us_at_153GBs": round(face / 153e9 * 1e6, 1)}
    prop.close()
    log("slab: %s" % res)
    return res


def sweep_c3(torch, orders=(4, 8, 12, 16), steps=500):
    """512^3 physical (592^3 computational), two-layer 1.5/2.5 km/s, one
    shot per order: GPts/s and the step kernel's algorithmic bandwidth (the
    shot's run of step launches timed by one pair of HIP events). Where the
    default runs two updates per launch (order 4 at this size) the same shot
    also runs with one update per launch, for comparison."""
    from paper_1808_01995_amd import Propagator, _abi
    from synthetic import config, ricker
    res = []
    v = None
    stream = None
    for so in orders:
        c = config("c3_sweep", space_order=so, steps=steps)
        if v is None:
            v = c.velocity()
        prop = Propagator(v, spacing=c.spacing, nbl=c.nbl, space_order=so)
        dt = 0.5 * prop.critical_dt()
        q = torch.from_numpy(ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32)).cuda()
        rec = torch.empty((c.nt, c.rec.shape[0]), device="cuda")
        for mode in (1, 0):
            _abi.wf_two_step_enable(mode)
            prop.forward(dt, 21, c.src, q[:21].contiguous(), c.rec, rec_out=rec[:21])   # warm-up
            _abi.wf_profile_read(_abi.WF_KERNEL_STEP_RUN, reset=True)
            _abi.wf_profile_runs_enable(True)
            el, _ = _timed(torch, lambda: prop.forward(dt, c.nt, c.src, q, c.rec, rec_out=rec))
            _abi.wf_profile_runs_enable(False)
            ms1, n1 = _abi.wf_profile_read(_abi.WF_KERNEL_STEP_RUN)
            ms2, n2 = _abi.wf_profile_read(_abi.WF_KERNEL_STEP2_RUN, reset=True)
            # per update: the summed spans over the updates they cover
            us = (ms1 + ms2) / max(n1 + 2 * n2, 1) * 1e3
            gbs = BYTES_PER_POINT * prop.npoints / (us * 1e-6) / 1e9
            if stream is None:
                stream = _abi.wf_stream_bandwidth(prop.npoints, 10)
            r = {"space_order": so, "dt_ms": round(dt, 4), "gpts": round(prop.npoints * c.steps / el / 1e9, 1),
                 "updates_per_launch": 2 if n2 else 1,
                 "step_kernel_us": round(us, 1), "algorithmic_GBs": round(gbs), "frac_8TBs": round(gbs / PEAK_HBM_GBS, 3),
                 "frac_of_stream": round(gbs / stream, 3)}
            if n2:
                two_us = ms2 / n2 * 1e3
                r.update({"step_kernel_us_note": "per update; 16 B per node per update",
                          "two_update_launch_us": round(two_us, 1),
                          "two_update_frac_8TBs": round(20.0 * prop.npoints / (two_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 3),
                          "two_update_note": "its own 20 B per node per launch (read u^n, u^{n-1}, kappa; "
                                             "write u^{n+1}, u^{n+2})"})
            res.append(r)
            log("c3 so%d: %s" % (so, res[-1]))
            if not n2:
                break   # one update per launch by default: nothing to compare
        _abi.wf_two_step_enable(1)
        prop.close()
    return {"workload": "592^3 computational (512^3 + 40-node layer), two-layer 1.5/2.5 km/s, %d updates" % steps,
            "stream_GBs": round(stream, 1), "orders": res}


def gradient_c4(torch, steps=2000, snaps=(-1, 50, 20, -2)):
    """200^3 physical (280^3), order 8, Gaussian anomaly; residual of the
    background model against data of the true model; gradient with store-all
    and revolve checkpointing, and through torch.autograd."""
    from paper_1808_01995_amd import Propagator, model_data, pad_replicate, slowness_sq
    from synthetic import config, ricker
    c = config("c4_gradient", steps=steps)
    v_true = c.velocity()
    v0 = np.full(c.shape, 2.0)
    pt = Propagator(v_true, spacing=c.spacing, nbl=c.nbl, space_order=8, c_ref=2.5)
    dt = 0.5 * pt.critical_dt(2.5)
    q = torch.from_numpy(ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32)).cuda()
    d_obs = pt.forward(dt, c.nt, c.src, q, c.rec)
    pt.close()
    p0 = Propagator(v0, spacing=c.spacing, nbl=c.nbl, space_order=8, c_ref=2.5)
    t_fwd, d = _timed(torch, lambda: p0.forward(dt, c.nt, c.src, q, c.rec))
    r = (d - d_obs).contiguous()
    out = {"workload": "280^3 computational, order 8, %d updates, 1 source, 100x100 receivers" % steps,
           "forward_s": round(t_fwd, 3), "misfit": 0.5 * float((r.double() ** 2).sum())}
    ref = None
    runs = []
    from paper_1808_01995_amd import _abi
    # store-all runs first: its workspace (the largest) is then reused by the
    # other modes, so no timed call reallocates device memory
    fb = p0.npoints * 4
    slabs = sum(2 * 4 * int(np.prod([c.shape[b] for b in range(3) if b != a])) for a in range(3))
    l = c.nt - 1
    for s in snaps:
        _abi.wf_profile_step_launches(0, reset=True)
        el, g = _timed(torch, lambda: p0.gradient(dt, c.nt, c.src, q, c.rec, r, n_checkpoints=s))
        fwd_counted = _abi.wf_profile_step_launches(0)
        rev_counted = _abi.wf_profile_step_launches(1)
        if s == -2:
            fwd_model = 2 * l - 2     # forward sweep + backward rebuild
            name = "boundary"
            need = 4 * fb + c.nt * slabs * 4
        else:
            # state 0 needs one step; revolve then advances its optimum
            fwd_model = l if s == -1 else 1 + _abi.wf_revolve_forward_steps(l, s)
            name = "all" if s == -1 else s
            need = (c.nt + 2 if s == -1 else 2 * s + 5) * fb
        runs.append({"checkpoints": name, "seconds": round(el, 3),
                     "forward_steps_counted": fwd_counted, "reverse_steps_counted": rev_counted,
                     "forward_steps_model": fwd_model, "workspace_GB": round(need / 1e9, 1),
                     "gpts_effective": round(p0.npoints * c.steps / el / 1e9, 1)})
        if ref is None:
            ref = g
        if s == -2:
            inner = tuple(slice(c.nbl, c.nbl + n) for n in c.shape)
            runs[-1]["rel_l2_vs_store_all_on_physical_grid"] = float(
                (g[inner] - ref[inner]).double().norm() / ref[inner].double().norm())
        else:
            runs[-1]["bitwise_equal_to_store_all"] = bool(torch.equal(g, ref))
        log("c4 gradient s=%s: %s" % (s, runs[-1]))
        del g
    out["gradient"] = runs
    out["accuracy"] = c4_gradient_accuracy(torch, p0, c, dt, q, steps)
    # torch.autograd path on the physical grid (replicate-pad adjoint folds the layer)
    m_phys = torch.from_numpy((1.0 / v0 ** 2).astype(np.float32)).cuda().requires_grad_(True)
    def ag():
        dd = model_data(pad_replicate(m_phys, c.nbl), p0, dt, c.nt, c.src, q, c.rec, 50)
        loss = 0.5 * ((dd - d_obs) ** 2).sum()
        loss.backward()
        return loss
    el, _ = _timed(torch, ag)
    out["autograd_forward_plus_backward_s"] = round(el, 3)
    p0.close()
    return out


def c4_gradient_accuracy(torch, p0, c, dt, q, steps):
    """J^T r of the initial model for the seeded band-limited residual stored
    with the FP64 oracle's result on the plane y = 140 (tests/golden,
    written by a script that calls only the oracle): rel. L2 over the plane,
    over its nodes more than 4 cells from every source and receiver node, and
    the largest element error against the plane's peak."""
    from synthetic import band_limited_noise
    path = os.path.join(ROOT, "tests", "golden", "c4_gradient_slice.npz")
    if steps != 2000 or not os.path.exists(path):
        return {"note": "stored oracle result not available for %d updates" % steps}
    gs = np.load(path)
    y, st = int(gs["y_index"]), int(gs["step"])
    rn = band_limited_noise(c.nt, c.rec.shape[0], dt, float(gs["noise_f0_hz"]), int(gs["noise_seed"]))
    gn = p0.gradient(dt, c.nt, c.src, q, c.rec, torch.from_numpy(rn.astype(np.float32)).cuda(),
                     n_checkpoints=-1)[::st, y, ::st].double().cpu().numpy()
    ref = gs["gradient"].astype(np.float64)
    comp = p0.comp_shape
    near = np.zeros(comp, dtype=bool)
    for xyz in (c.src, c.rec):
        s_ = np.floor(np.asarray(xyz) / np.asarray(c.spacing) + c.nbl).astype(int)
        for i in s_:
            near[tuple(slice(max(0, a - 4), a + 6) for a in i)] = True
    away = ~near[::st, y, ::st]
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))   # noqa: E731
    return {"jt_r_plane_rel_l2": rel(gn, ref), "jt_r_plane_away_rel_l2": rel(gn[away], ref[away]),
            "jt_r_plane_max_element": float(np.abs(gn - ref).max() / np.abs(ref).max()),
            "bar": "rel. L2 <= 1e-3 vs the FP64 oracle",
            "note": "a residual both sides share; the workload's own residual (initial minus true "
                    "model record) is 7e-5 of the records, whose FP32 error (8e-6 of the records) "
                    "leaves it about 3 % uncertain, so the gradient of the workload's own misfit is "
                    "only that close to the oracle's (measured 2.8 % on this plane)"}


def born_c4(torch, steps=2000):
    """Linearised modelling J dm on the 280^3 order-8 workload (background
    v = 2 km/s, dm = the Gaussian anomaly's squared-slowness change): two
    launches per update, 44 algorithmic bytes per node (background step with
    the scattered source: 24; scattered step: 20)."""
    from paper_1808_01995_amd import Propagator, _abi
    from synthetic import config, ricker
    c = config("c4_gradient", steps=steps)
    v_true = c.velocity()
    p0 = Propagator(np.full(c.shape, 2.0), spacing=c.spacing, nbl=c.nbl, space_order=8, c_ref=2.5)
    dt = 0.5 * p0.critical_dt(2.5)
    q = torch.from_numpy(ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32)).cuda()
    from paper_1808_01995_amd import slowness_sq
    dm = (slowness_sq(v_true, c.nbl, "cuda") - p0.m).contiguous()
    p0.born(dt, 21, c.src, q[:21].contiguous(), dm, c.rec)     # warm-up
    el, dd = _timed(torch, lambda: p0.born(dt, c.nt, c.src, q, dm, c.rec))
    gbs = 44.0 * p0.npoints * c.steps / el / 1e9
    out = {"workload": "280^3 computational, order 8, %d updates, 1 source, 100x100 receivers" % steps,
           "seconds": round(el, 3), "gpts": round(p0.npoints * c.steps / el / 1e9, 1),
           "algorithmic_GBs": round(gbs), "frac_8TBs": round(gbs / PEAK_HBM_GBS, 3)}
    p0.close()
    log("born: %s" % out)
    return out


def fwi_multishot(torch, steps=2000, iters=3):
    """Multi-shot FWI on the 280^3 order-8 gradient workload: 4 sources at
    20 m depth on a 2 x 2 pattern, the 100 x 100 receiver grid for each;
    per iteration the summed gradient (two wave solves per shot, store-all or
    revolve as memory allows) and one fixed-step update. The observed data
    are modelled on the true model with the same forward (a timing row)."""
    from paper_1808_01995_amd import Propagator
    from synthetic import config, ricker
    c = config("c4_gradient", steps=steps)
    v_true = c.velocity()
    pt = Propagator(v_true, spacing=c.spacing, nbl=c.nbl, space_order=8, c_ref=2.5)
    dt = 0.5 * pt.critical_dt(2.5)
    q = torch.from_numpy(ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32)).cuda()
    ext = (c.shape[0] - 1) * c.spacing[0]
    srcs = [np.array([[fx * ext, fy * ext, 20.0]]) for fx in (0.25, 0.75) for fy in (0.25, 0.75)]
    shots = [(sx, q, c.rec, pt.forward(dt, c.nt, sx, q, c.rec)) for sx in srcs]
    pt.close()
    p0 = Propagator(np.full(c.shape, 2.0), spacing=c.spacing, nbl=c.nbl, space_order=8, c_ref=2.5)
    its = []
    for it in range(iters):
        torch.cuda.synchronize()
        t = time.perf_counter()
        phi, g = p0.fwi_gradient(dt, c.nt, shots)
        # fixed step (Cauchy): 0.001 % of max m at the gradient's peak, which
        # sits on a source node; 0.01 % already overshoots there and raises
        # the misfit, 0.001 % lowers it by the first-order prediction
        alpha = 1e-5 * float(p0.m.abs().max()) / float(g.abs().max())
        p0.update(g, alpha, vmin=1.5, vmax=2.5)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        its.append({"seconds": round(el, 3), "misfit": phi,
                    "shots_per_s": round(len(shots) / el, 2),
                    "gpts_effective": round(2 * len(shots) * p0.npoints * c.steps / el / 1e9, 1)})
        log("fwi iteration %d: %s" % (it, its[-1]))
    p0.close()
    return {"workload": "280^3 computational, order 8, %d updates, 4 shots x 100x100 receivers, "
                        "fixed-step update (0.001 %% of max m at the gradient's peak) with 1.5-2.5 km/s "
                        "bounds" % steps,
            "iterations": its,
            "note": "gpts_effective counts two wave solves per shot; the first iteration also "
                    "allocates the model's gradient workspace (store-all: 2001 fields, 176 GB)"}


def serving_c5(torch, n_requests=256, seed=5):
    """The serving stream at full size (the seeded mix of 256 requests, or its
    first `n_requests`: 2D 256^2-2048^2 or 3D 128^3-384^3 physical, orders
    4/8/12, 500-2000 updates, 1 in 4 a gradient): one-shot-per-launch baseline
    mu_0, saturated throughput, Poisson arrivals at 0.5/0.8/1.2 mu_0."""
    from paper_1808_01995_amd.serve import (GRADIENT_SHARE, Server, build_request, run_one_shot_baseline,
                                            run_stream)
    from synthetic import serving_requests
    specs = serving_requests(n_requests, seed=seed)
    t_build = time.perf_counter()
    reqs = [build_request(sp) for sp in specs]
    torch.cuda.synchronize()
    log("serving: %d requests built in %.1f s" % (len(reqs), time.perf_counter() - t_build))
    # one budget for both paths (0.9 of what is free once the baseline's
    # outputs are held): the engine's arena, and the gradient checkpoint
    # memory the baseline mirrors
    outs_bytes = sum(r.rec_out.numel() * 4 + (r.m.numel() * 4 if r.grad_out is not None else 0) for r in reqs)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.9 * (free - outs_bytes - (1 << 30)))
    base = run_one_shot_baseline(reqs, budget, time_reuse=True)
    mu0 = base["shots_per_s"]
    mu0_noalloc = len(reqs) / base["seconds_without_workspace_allocation"]
    log("serving: one-shot baseline %.2f shots/s (%.2f without gradient workspace allocation)" % (mu0, mu0_noalloc))
    srv = Server(hbm_budget_bytes=budget, max_slots=64)
    sat = run_stream(srv, reqs)
    log("serving: saturated %.2f shots/s" % sat["shots_per_s"])
    rel = 0.0
    for r, (d, g) in zip(reqs, base["outputs"]):
        rel = max(rel, float((r.rec_out - d).norm() / max(float(d.norm()), 1e-30)))
        if g is not None:
            rel = max(rel, float((r.grad_out - g).norm() / max(float(g.norm()), 1e-30)))
    base = None
    rng = np.random.default_rng(seed)
    poisson = []
    for f in (0.5, 0.8, 1.2):
        lam = f * mu0
        arr = np.cumsum(rng.exponential(1.0 / lam, size=len(reqs))).tolist()
        st = run_stream(srv, reqs, arr)
        poisson.append({"lambda_over_mu0": f, "arrival_rate_per_s": round(lam, 2),
                        "p50_ms": round(st["p50_ms"], 1), "p99_ms": round(st["p99_ms"], 1),
                        "shots_per_s": round(st["shots_per_s"], 2), "failed": st["failed"]})
        log("serving poisson %.1f: %s" % (f, poisson[-1]))
    srv.close()
    n2 = sum(1 for s_ in specs if s_["ndim"] == 2)
    ng = sum(1 for s_ in specs if s_["kind"] == "gradient")
    return {"workload": "%d requests (%d 2D / %d 3D, %d gradients) of the seeded serving mix at full size: "
                        "2D 256^2-2048^2 or 3D 128^3-384^3 physical + 40-node layer, orders 4/8/12, "
                        "500-2000 updates, smooth random v 1.5-4.5 km/s; a gradient's checkpoints in "
                        "1/%d of the budget (store-all if they fit, else revolve) on both paths"
                        % (len(specs), n2, len(specs) - n2, ng, GRADIENT_SHARE),
            "one_shot_baseline_shots_per_s": round(mu0, 2),
            "one_shot_baseline_without_workspace_allocation_shots_per_s": round(mu0_noalloc, 2),
            "engine_budget_bytes": budget,
            "saturated": {"shots_per_s": round(sat["shots_per_s"], 2), "p50_ms": round(sat["p50_ms"], 1),
                          "p99_ms": round(sat["p99_ms"], 1), "failed": sat["failed"]},
            "speedup_vs_one_shot": round(sat["shots_per_s"] / mu0, 2),
            "speedup_vs_one_shot_without_workspace_allocation": round(sat["shots_per_s"] / mu0_noalloc, 2),
            "poisson": poisson,
            "max_rel_l2_vs_one_shot": rel}


def profile_kernels(torch, steps=400):
    """A short run of every step-kernel mode for rocprofv3: 280^3 order 8,
    v = 2 km/s, 100 x 100 receivers; two store-all gradients (plain and
    imaging modes) for a random residual and two Born modellings (Born-source
    and volume-source modes) for a random perturbation."""
    from paper_1808_01995_amd import Propagator
    from synthetic import config, ricker
    c = config("c4_gradient", steps=steps)
    p0 = Propagator(np.full(c.shape, 2.0), spacing=c.spacing, nbl=c.nbl, space_order=8, c_ref=2.5)
    dt = 0.5 * p0.critical_dt(2.5)
    q = torch.from_numpy(ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32)).cuda()
    gen = torch.Generator(device="cuda").manual_seed(0)
    r = torch.randn((c.nt, c.rec.shape[0]), device="cuda", generator=gen)
    dm = torch.randn(p0.comp_shape, device="cuda", generator=gen) * 1e-3
    for _ in range(2):
        p0.gradient(dt, c.nt, c.src, q, c.rec, r, n_checkpoints=-1)
        p0.born(dt, c.nt, c.src, q, dm, c.rec)
    torch.cuda.synchronize()
    p0.close()
    print(json.dumps({"profile_kernels": "done", "grid": list(p0.comp_shape), "updates": steps}), flush=True)


def profile_two_update(torch, so, steps=20):
    """A short run of the two-update kernel for rocprofv3: the C2 grid (336^3,
    smooth random velocity) at space order `so`, `steps` updates with two
    updates per launch forced (wf_two_step_enable(2))."""
    from paper_1808_01995_amd import Propagator, _abi
    from synthetic import config, ricker
    c = config("c2_3d_so8", space_order=so, steps=steps)
    prop = Propagator(c.velocity(), spacing=c.spacing, nbl=c.nbl, space_order=so)
    dt = 0.5 * prop.critical_dt()
    q = torch.from_numpy(ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32)).cuda()
    _abi.wf_two_step_enable(2)
    rec = prop.forward(dt, c.nt, c.src, q, c.rec)
    torch.cuda.synchronize()
    _abi.wf_two_step_enable(1)
    prop.close()
    print(json.dumps({"profile_two_update": "done", "space_order": so, "updates": steps,
                      "record_max": float(rec.abs().max())}), flush=True)


def profile_team_shots(torch, shots=3):
    """C1-size forward shots (101^2 physical + 20-node layer, order 4, 500
    updates) submitted to the serving engine one after another, each run on
    resident teams (WAVEFD_TEAM_WIDTH in the environment sets the split), for
    rocprofv3 counters."""
    from paper_1808_01995_amd.serve import Server, build_request, run_stream
    reqs = [build_request({"ndim": 2, "n": 101, "space_order": 4, "steps": 500, "kind": "forward",
                           "seed": 300 + i}, nbl=20) for i in range(shots)]
    srv = Server(hbm_budget_bytes=4 << 30, max_slots=16)
    for r in reqs:
        run_stream(srv, [r])
    srv.close()
    print(json.dumps({"profile_team_shots": "done", "shots": shots,
                      "team_width": os.environ.get("WAVEFD_TEAM_WIDTH")}), flush=True)


def copy_bandwidth(torch, nbytes=1 << 30, reps=10) -> float:
    """Read + write GB/s of a plain device-to-device copy (the STREAM-copy
    analogue the step kernel's bandwidth is compared with)."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t) / reps
    del a, b
    return 2.0 * nbytes / el / 1e9


def run_rows(torch, args, orders, out):
    """The further rows named by --rows, added to `out`; returns the set."""
    rows = set(x for x in args.rows.split(",") if x)
    if "all" in rows:
        rows = {"c1", "2d", "c3", "slab", "c4", "born", "fwi", "serve"}
    if "c1" in rows:
        out["c1_graph"] = graph_c1(torch)
        out["c1_batch"] = c1_batch(torch)
    if "2d" in rows:
        out["large_2d"] = large_2d(torch)
    if "c3" in rows:
        out["c3_sweep"] = sweep_c3(torch, orders=orders, steps=args.updates or 500)
    if "slab" in rows:
        out["slab_share"] = slab_share(torch)
    if "c4" in rows:
        out["c4_gradient"] = gradient_c4(torch)
    if "born" in rows:
        out["born"] = born_c4(torch)
    if "fwi" in rows:
        out["fwi_multishot"] = fwi_multishot(torch)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed shots")
    ap.add_argument("--warmup", type=int, default=1, help="untimed shots")
    ap.add_argument("--space-order", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-two-update", action="store_true",
                    help="skip the short shots that compare two updates per launch with one "
                         "(also skipped with --serve-requests 0)")
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--extras", action="store_true", help="also time the adjoint shot")
    ap.add_argument("--rows", default="",
                    help="comma list of further rows to measure: c1,2d,c3,slab,c4,born,fwi,serve (or all)")
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests of the full-size serving stream measured with the headline "
                         "(default: the whole seeded mix of 256; 0 skips it)")
    ap.add_argument("--updates", type=int, default=None,
                    help="shorter shots (profiling runs only; the benchmark uses 1000): the headline "
                         "shot and, with --rows c3, the sweep's shots")
    ap.add_argument("--orders", default="4,8,12,16", help="space orders of the c3 sweep")
    ap.add_argument("--rows-only", action="store_true",
                    help="only the rows of --rows (no headline shot, serving or oracle baseline): "
                         "short profiling runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--profile-two-update", type=int, default=0, metavar="ORDER",
                    help="short run of the two-update kernel at this space order on the C2 grid, for rocprofv3")
    ap.add_argument("--profile-team-shots", action="store_true",
                    help="three C1-size shots on the engine's resident teams, for rocprofv3")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only run the gradient and Born kernels for a profiler: 280^3 order 8, "
                         "400 updates, two store-all gradients and two Born modellings")
    ap.add_argument("--oracle-one-core", type=int, default=0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_one_core:
        oracle_one_core(args.oracle_one_core)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(shots are independent; see the design notes for how it would shard)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "no GPU"
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": a.numel() * 4}), flush=True)
        return
    from paper_1808_01995_amd import _abi
    if args.profile_kernels:
        profile_kernels(torch)
        return
    if args.profile_two_update:
        profile_two_update(torch, args.profile_two_update)
        return
    if args.profile_team_shots:
        profile_team_shots(torch)
        return
    orders = tuple(int(x) for x in args.orders.split(",") if x)
    if args.rows_only:
        out = {}
        run_rows(torch, args, orders, out)
        print(json.dumps(out), flush=True)
        return

    c, v, prop, dt, q, rec_out = setup_c2(torch, args.space_order, args.updates)
    npts = prop.npoints
    log("workload: %s Nc=%s nt=%d dt=%.4f ms" % (c.name, prop.comp_shape, c.nt, dt))

    def shot():
        prop.forward(dt, c.nt, c.src, q, c.rec, rec_out=rec_out)

    for _ in range(args.warmup):
        shot()
    torch.cuda.synchronize()

    # each shot's run of step launches is bracketed by one pair of HIP events
    # on the stream the steps are launched on (two events per shot): the
    # spans summed over the timed shots, divided by their step launches, give
    # the average step-launch duration, gaps between the back-to-back
    # launches included, so that it times every launch of the timed region
    _abi.wf_profile_read(_abi.WF_KERNEL_STEP_RUN, reset=True)
    _abi.wf_profile_runs_enable(True)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i].record()   # on the stream the shot is enqueued on
        shot()
    evs[-1].record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    shot_ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)]
    _abi.wf_profile_runs_enable(False)
    k_ms, k_n = _abi.wf_profile_read(_abi.WF_KERNEL_STEP_RUN, reset=True)

    # the same shots launched as a captured HIP graph (kernel timing off, so
    # the loop is captured on the first call with an unchanged signature)
    _abi.wf_graph_enable(True)
    g0 = _abi.wf_model_graph_launches(prop.handle)
    shot()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        shot()
    torch.cuda.synchronize()
    el_graph = time.perf_counter() - t0
    g_launches = _abi.wf_model_graph_launches(prop.handle) - g0
    _abi.wf_graph_enable(False)

    copy_gbs = copy_bandwidth(torch)
    # the same 16 bytes per node as a plain stream over arrays of the grid's size
    stream_gbs = _abi.wf_stream_bandwidth(npts, 20)

    ms_per_shot = el / args.steps * 1e3
    updates = npts * c.steps
    gpts = updates / (ms_per_shot * 1e-3) / 1e9
    phys = int(np.prod(c.shape)) * c.steps / (ms_per_shot * 1e-3) / 1e9
    avg_kernel_ms = k_ms / max(k_n, 1)
    achieved = BYTES_PER_POINT * npts / (avg_kernel_ms * 1e-3) / 1e9
    tb = traffic_from_profile("step3d_so8_c2_traffic.json", npts)

    out = {
        "metric": "GPts/s (3D SO8 forward, computational grid incl. damping layer)",
        "value": round(gpts, 3),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_shot, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D acoustic SO8 forward shot: 256^3 physical (%s computational), "
                               "h=10 m, nbl=40, smooth random v 1.5-4.5 km/s, %d updates, "
                               "15 Hz Ricker at 20 m, 128x128 receivers"
                               % ("x".join(map(str, prop.comp_shape)), c.steps),
                   "grid": list(prop.comp_shape), "updates": c.steps, "space_order": c.space_order},
        "physical_gpts": round(phys, 3),
        "shot_device_ms": {"median": round(float(np.median(shot_ms)), 3), "min": round(min(shot_ms), 3),
                           "max": round(max(shot_ms), 3),
                           "note": "each timed shot bracketed by events on its stream"},
        "graph_replay": {"ms_per_step": round(el_graph / args.steps * 1e3, 3),
                         "value": round(updates / (el_graph / args.steps) / 1e9, 3),
                         "graph_launches": g_launches,
                         "note": "same shots replayed from one captured HIP graph, no kernel events"},
        "hbm_fraction_of_8TBs": round(BYTES_PER_POINT * updates / (ms_per_shot * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": tb,
                     "kernel": "k_step3d<M=4> (fused stencil + damping + time update)",
                     "avg_kernel_ms": round(avg_kernel_ms, 5), "timed_launches": k_n,
                     "launches_in_timed_region": args.steps * c.steps,
                     "timing_note": "average step launch = the summed spans from before the first to "
                                    "after the last step launch of each timed shot (two events per shot "
                                    "on the launch stream) over the launches they cover",
                     "algorithmic_bytes_per_launch": BYTES_PER_POINT * npts,
                     "measured_copy_GBs": round(copy_gbs, 1),
                     "frac_of_measured_copy": round(achieved / copy_gbs, 4),
                     "measured_stream_GBs": round(stream_gbs, 1),
                     "frac_of_measured_stream": round(achieved / stream_gbs, 4),
                     "stream_note": "wf_stream_bandwidth: 3 float reads + 1 float write per node "
                                    "(the step kernel's algorithmic bytes) over %d-float arrays, no stencil"
                                    % npts},
    }

    if args.extras:
        y = rec_out.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        prop.adjoint(dt, c.nt, c.rec, y, c.src)
        torch.cuda.synchronize()
        out["adjoint_gpts"] = round(updates / (time.perf_counter() - t) / 1e9, 3)

    prop.close()
    rows = run_rows(torch, args, orders, out)
    if not args.no_two_update and args.serve_requests > 0 and "c3" not in rows and "2d" not in rows:
        # the shots that run two updates per launch by default, each also
        # with one: 592^3 order 4 and 8272^2 order 4 (short shots; part of
        # the full default line, like the serving rows, so skipped with
        # --serve-requests 0, the headline-only run the profiles are taken on)
        try:
            out["two_update"] = {"c3_order4": sweep_c3(torch, orders=(4,), steps=100),
                                 "large_2d_order4": large_2d(torch, orders=(4,), steps=100)}
        except Exception as e:  # must not hide the headline
            out["two_update"] = {"error": str(e)}
    if "serve" in rows and args.serve_requests < 256:
        args.serve_requests = 256
    if args.serve_requests > 0:
        try:
            out["c5_serving"] = serving_c5(torch, args.serve_requests)
        except Exception as e:  # the serving row must not hide the headline
            out["c5_serving"] = {"error": str(e)}
    if not args.no_cpu:
        try:
            out["cpu_baseline"] = cpu_baseline(c, v, dt, args.cpu_steps)
        except Exception as e:  # the baseline must not hide the GPU number
            out["cpu_baseline"] = {"error": str(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
