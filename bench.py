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
events inside the timed region, and the FP64 oracle timed on the host cores on
a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--extras]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
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
    return {"value": m.size * sample_steps / el / 1e9, "unit": "GPts/s", "cores": cores,
            "kind": "oracle",
            "sample": "FP64 oracle, %d of %d updates of the same %s-point shot (%.1f s)"
                      % (sample_steps, c.steps, "x".join(map(str, m.shape)), el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed shots")
    ap.add_argument("--warmup", type=int, default=1, help="untimed shots")
    ap.add_argument("--space-order", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--extras", action="store_true", help="also time adjoint and gradient")
    ap.add_argument("--updates", type=int, default=None,
                    help="shorter shots (profiling runs only; the benchmark uses 1000)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
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

    c, v, prop, dt, q, rec_out = setup_c2(torch, args.space_order, args.updates)
    npts = prop.npoints
    log("workload: %s Nc=%s nt=%d dt=%.4f ms" % (c.name, prop.comp_shape, c.nt, dt))

    def shot():
        prop.forward(dt, c.nt, c.src, q, c.rec, rec_out=rec_out)

    for _ in range(args.warmup):
        shot()
    torch.cuda.synchronize()

    _abi.wf_profile_read(_abi.WF_KERNEL_STEP, reset=True)
    _abi.wf_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        shot()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    _abi.wf_profile_enable(False)
    k_ms, k_n = _abi.wf_profile_read(_abi.WF_KERNEL_STEP)
    i_ms, i_n = _abi.wf_profile_read(_abi.WF_KERNEL_INJECT)
    s_ms, s_n = _abi.wf_profile_read(_abi.WF_KERNEL_SAMPLE, reset=True)

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
        "hbm_fraction_of_8TBs": round(BYTES_PER_POINT * updates / (ms_per_shot * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": tb,
                     "kernel": "k_step3d<M=4> (fused stencil + damping + time update)",
                     "avg_kernel_ms": round(avg_kernel_ms, 5), "launches": k_n,
                     "algorithmic_bytes_per_launch": BYTES_PER_POINT * npts},
        "sparse_kernels_ms_per_shot": {"inject": round(i_ms / args.steps, 3),
                                       "sample": round(s_ms / args.steps, 3)},
    }

    if args.extras:
        y = rec_out.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        prop.adjoint(dt, c.nt, c.rec, y, c.src)
        torch.cuda.synchronize()
        out["adjoint_gpts"] = round(updates / (time.perf_counter() - t) / 1e9, 3)

    prop.close()
    if not args.no_cpu:
        try:
            out["cpu_baseline"] = cpu_baseline(c, v, dt, args.cpu_steps)
        except Exception as e:  # the baseline must not hide the GPU number
            out["cpu_baseline"] = {"error": str(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
