"""Serving front-end over the library's continuous-batching engine.

`Server` submits shot-modelling and gradient requests to the native engine
(wf_engine_*), which admits them by HBM budget, batches small grids into
shared launches and runs the rest concurrently; the front-end only keeps the
request tensors alive, timestamps arrivals and completions, and reports
latency percentiles and throughput.

`build_request` turns a request description (dimension, grid size, space
order, steps, kind, seed) into device tensors: a smooth random velocity model
(generated on the device: the mix reaches 384^3), a 10 Hz Ricker source at the
centre at 20 m depth, receivers at 20 m depth (a line in 2D, 64 x 64 in 3D);
gradient requests carry observed data modelled on a model perturbed by a few
percent.
"""
from __future__ import annotations

import ctypes
import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _abi
from .propagator import Propagator, pad_replicate


@dataclasses.dataclass
class Request:
    kind: int                      # _abi.WF_REQ_FORWARD or _abi.WF_REQ_GRADIENT
    geom: _abi.wf_geom
    m: torch.Tensor                # computational-grid squared slowness (device)
    dt: float
    nt: int
    src_xyz: np.ndarray
    src_wav: torch.Tensor
    rec_xyz: np.ndarray
    rec_out: torch.Tensor
    d_obs: Optional[torch.Tensor] = None
    grad_out: Optional[torch.Tensor] = None
    misfit: Optional[float] = None
    arrival: float = 0.0           # seconds (wall clock) when the request arrived
    done: float = 0.0
    status: int = 0
    tag: Dict = dataclasses.field(default_factory=dict)
    _misfit_buf: Optional[ctypes.c_double] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def updates(self) -> int:
        n = 1
        for a in range(self.geom.ndim):
            n *= self.geom.n[a] + 2 * self.geom.nbl
        return n * (self.nt - 1) * (2 if self.kind == _abi.WF_REQ_GRADIENT else 1)   # a gradient is two solves


def build_request(spec: Dict, device="cuda", vmin: float = 1.5, vmax: float = 4.5,
                  h: float = 10.0, nbl: int = 40, f0_hz: float = 10.0) -> Request:
    """Device tensors for one serving request (see module docstring)."""
    from synthetic import grid_receivers, line_receivers, ricker, smooth_random_velocity_device
    nd, n, so, steps = spec["ndim"], spec["n"], spec["space_order"], spec["steps"]
    shape = (n,) * nd
    v = smooth_random_velocity_device(shape, spec["seed"], sigma=max(2.0, n / 32.0), vmin=vmin, vmax=vmax,
                                      device=device)
    v_top = float(v.max())
    ext = (n - 1) * h
    if nd == 2:
        src = np.array([[ext / 2, 20.0]])
        rec = line_receivers(n, 0.0, ext, 20.0, ndim=2)
    else:
        src = np.array([[ext / 2, ext / 2, 20.0]])
        rec = grid_receivers(64, 64, ext, ext, 20.0)
    geom = _abi.make_geom(shape, (h,) * nd, nbl, so, v_top)
    m = pad_replicate(1.0 / (v * v), nbl).float().contiguous()
    nt = steps + 1
    dt = 0.5 * _abi.wf_critical_dt(geom, v_top * 1.06)
    wav = torch.from_numpy(ricker(nt, dt, f0_hz)[:, None].astype(np.float32)).to(device)
    rec_out = torch.empty((nt, rec.shape[0]), dtype=torch.float32, device=device)
    kind = _abi.WF_REQ_FORWARD if spec["kind"] == "forward" else _abi.WF_REQ_GRADIENT
    r = Request(kind, geom, m, dt, nt, src, wav, rec, rec_out, tag=dict(spec))
    if kind == _abi.WF_REQ_GRADIENT:
        # observed data from the model perturbed by `perturb` (smoothly)
        pattern = smooth_random_velocity_device(shape, spec["seed"] + 7, sigma=max(2.0, n / 16.0),
                                                vmin=-1.0, vmax=1.0, device=device)
        v_true = v * (1.0 + spec.get("perturb", 0.05) * pattern)
        m_true = pad_replicate(1.0 / (v_true * v_true), nbl).float().contiguous()
        del pattern, v_true
        prop = Propagator(m=m_true, shape=shape, spacing=(h,) * nd, nbl=nbl, space_order=so, c_ref=v_top)
        r.d_obs = prop.forward(dt, nt, src, wav, rec)
        torch.cuda.synchronize()
        prop.close()
        del m_true
        r.grad_out = torch.empty(m.shape, dtype=torch.float32, device=device)
        r._misfit_buf = ctypes.c_double(0.0)
    return r


# the engine gives a gradient request budget / GRADIENT_SHARE bytes of
# checkpoint memory: every forward field if they fit, else a revolve pool
GRADIENT_SHARE = 4


def gradient_memory(budget: int, npoints: int, nt: int, nrec: int):
    """(n_checkpoints, hbm_budget_bytes) for the plain propagator's gradient
    call that give it the checkpoint memory the engine gives a gradient
    request under `budget`, so that both run the same schedule (up to the
    field padding, estimated here as 10 %)."""
    fb = npoints * 4
    share = budget // GRADIENT_SHARE
    if int(1.1 * nt * fb) <= share:
        return -1, 0
    return 0, max(5 * fb, share) + 3 * fb + 2 * nt * nrec * 4 + (1 << 20)


def request_struct(r: Request) -> "_abi.wf_request":
    """The C request for `r` (its host coordinate arrays are kept on r)."""
    q = _abi.wf_request()
    q.kind = r.kind
    q.geom = r.geom
    q.m_dev = r.m.data_ptr()
    q.dt = r.dt
    q.nt = r.nt
    r._src = np.ascontiguousarray(r.src_xyz, dtype=np.float64)
    r._rec = np.ascontiguousarray(r.rec_xyz, dtype=np.float64)
    q.nsrc = r._src.shape[0]
    q.src_xyz = r._src.ctypes.data
    q.src_wav = r.src_wav.data_ptr()
    q.nrec = r._rec.shape[0]
    q.rec_xyz = r._rec.ctypes.data
    q.rec_out = r.rec_out.data_ptr()
    if r.kind == _abi.WF_REQ_GRADIENT:
        q.d_obs = r.d_obs.data_ptr()
        q.grad_out = r.grad_out.data_ptr()
        q.misfit_out = ctypes.addressof(r._misfit_buf)
    return q


class Server:
    """Client of one native engine (HBM budget, slot limit)."""

    def __init__(self, hbm_budget_bytes: Optional[int] = None, max_slots: int = 64,
                 budget_fraction: float = 0.9):
        if hbm_budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget_bytes = int(budget_fraction * free)
        self.budget = int(hbm_budget_bytes)
        self.handle = _abi.wf_engine_create(self.budget, max_slots)
        self.inflight: Dict[int, Request] = {}
        self.completed: List[Request] = []

    def submit(self, r: Request) -> int:
        """Queue `r`; the engine's work on it is ordered after the work the
        caller has queued on torch's current stream (which produced its
        inputs): no synchronisation of the device or the stream."""
        q = request_struct(r)
        if not r.arrival:
            r.arrival = time.perf_counter()
        t = _abi.wf_engine_submit_on(self.handle, q)
        self.inflight[t] = r
        return t

    def poll(self, wait_ms: int = 0) -> List[Request]:
        out = []
        for t, st in _abi.wf_engine_poll(self.handle, 256, wait_ms):
            r = self.inflight.pop(t)
            r.done = time.perf_counter()
            r.status = st
            if r._misfit_buf is not None:
                r.misfit = r._misfit_buf.value
            out.append(r)
        self.completed.extend(out)
        return out

    def stats(self):
        return _abi.wf_engine_stats(self.handle)

    def paths(self):
        """Completed requests by path: resident teams, batched launches, workers."""
        return _abi.wf_engine_paths(self.handle)

    def drain(self):
        while self.inflight:
            self.poll(wait_ms=50)

    def close(self):
        if getattr(self, "handle", None):
            self.drain()
            _abi.wf_engine_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_stream(server: Server, requests: List[Request], arrivals: Optional[List[float]] = None) -> Dict:
    """Submit `requests` at the given arrival offsets (seconds from now; all at
    once if None), wait for all, and return throughput and latency figures."""
    t0 = time.perf_counter()
    order = sorted(range(len(requests)), key=lambda i: (arrivals[i] if arrivals else 0.0))
    k = 0
    while k < len(order) or server.inflight:
        now = time.perf_counter() - t0
        while k < len(order) and (arrivals is None or arrivals[order[k]] <= now):
            r = requests[order[k]]
            r.arrival = t0 + (arrivals[order[k]] if arrivals else 0.0)
            server.submit(r)
            k += 1
        wait = 1
        if k < len(order) and arrivals is not None:
            wait = max(1, min(20, int(1000 * (arrivals[order[k]] - (time.perf_counter() - t0)))))
        server.poll(wait_ms=wait if server.inflight else 0)
        if not server.inflight and k < len(order) and arrivals is not None:
            time.sleep(max(0.0, arrivals[order[k]] - (time.perf_counter() - t0)))
    t1 = time.perf_counter()
    lat = np.array([r.latency for r in requests])
    bad = [r for r in requests if r.status != 0]
    return {"requests": len(requests), "makespan_s": t1 - t0, "shots_per_s": len(requests) / (t1 - t0),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "failed": len(bad)}


def run_one_shot_baseline(requests: List[Request], budget: Optional[int] = None,
                          time_reuse: bool = False) -> Dict:
    """The plain propagator, one request at a time (model created per request,
    one kernel launch per time step; gradients by the two-solve multi-shot
    call with one shot and the checkpoint memory an engine with `budget`
    gives them, so the same work the engine does): the reference throughput
    mu_0. Each model allocates its fields and gradient workspace with
    hipMalloc, which the engine's arena avoids; with `time_reuse` every
    gradient runs a second time on the same model (its workspace reused) and
    `seconds_without_workspace_allocation` charges the second run instead of
    the first."""
    if budget is None:
        free, _ = torch.cuda.mem_get_info()
        budget = int(0.9 * free)
    t0 = time.perf_counter()
    outs = []
    alloc = 0.0
    extra = 0.0   # second gradient runs: not part of the one-shot time
    for r in requests:
        nd = r.geom.ndim
        shape = tuple(r.geom.n[a] for a in range(nd))
        prop = Propagator(m=r.m, shape=shape, spacing=tuple(r.geom.h[a] for a in range(nd)),
                          nbl=r.geom.nbl, space_order=r.geom.space_order, c_ref=r.geom.c_ref)
        if r.kind == _abi.WF_REQ_GRADIENT:
            nck, cap = gradient_memory(budget, prop.npoints, r.nt, r.rec_xyz.shape[0])
            shot = [(r.src_xyz, r.src_wav, r.rec_xyz, r.d_obs)]
            ta = time.perf_counter()
            _, g, (d,) = prop.fwi_gradient(r.dt, r.nt, shot, n_checkpoints=nck, hbm_budget_bytes=cap,
                                           return_pred=True)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            if time_reuse:
                prop.fwi_gradient(r.dt, r.nt, shot, n_checkpoints=nck, hbm_budget_bytes=cap)
                torch.cuda.synchronize()
                tc = time.perf_counter()
                alloc += (tb - ta) - (tc - tb)
                extra += tc - tb
            outs.append((d, g))
        else:
            d = prop.forward(r.dt, r.nt, r.src_xyz, r.src_wav, r.rec_xyz)
            outs.append((d, None))
        torch.cuda.synchronize()
        prop.close()
    el = time.perf_counter() - t0 - extra
    out = {"requests": len(requests), "seconds": el, "shots_per_s": len(requests) / el, "outputs": outs}
    if time_reuse:
        out["seconds_without_workspace_allocation"] = el - alloc
    return out
