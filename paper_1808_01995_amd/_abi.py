"""ctypes binding of include/wavefd.h (libwavefd.so, built for gfx950).

Argument marshalling only: every numerical step runs in the library's HIP
kernels. Device arrays are torch tensors on the GPU (float32, contiguous);
host coordinate arrays are float64 numpy arrays; streams default to torch's
current stream. The functions keep the C names.

Importing this module loads the library and raises if it is missing: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# WAVEFD_LIBRARY selects another build of the same library (tuning runs).
LIB_PATH = os.environ.get("WAVEFD_LIBRARY") or os.path.join(HERE, "libwavefd.so")

WF_OK = 0
WF_E_ARG = -1
WF_E_DOMAIN = -2
WF_E_CFL = -3
WF_E_NOMEM = -4
WF_E_BUDGET = -5
WF_E_HIP = -6
WF_E_NONFINITE = -7
WF_E_STATE = -8
_NAMES = {0: "WF_OK", -1: "WF_E_ARG", -2: "WF_E_DOMAIN", -3: "WF_E_CFL", -4: "WF_E_NOMEM",
          -5: "WF_E_BUDGET", -6: "WF_E_HIP", -7: "WF_E_NONFINITE", -8: "WF_E_STATE"}

WF_REQ_FORWARD = 0
WF_REQ_GRADIENT = 1


class WaveFDError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__("%s: %s" % (_NAMES.get(status, str(status)), message))


class wf_geom(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int),
                ("n", ctypes.c_int64 * 3),
                ("h", ctypes.c_double * 3),
                ("origin", ctypes.c_double * 3),
                ("nbl", ctypes.c_int),
                ("space_order", ctypes.c_int),
                ("c_ref", ctypes.c_double),
                ("R", ctypes.c_double),
                ("eta_power", ctypes.c_int)]


class wf_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int),
                ("geom", wf_geom),
                ("m_dev", ctypes.c_void_p),
                ("dt", ctypes.c_double),
                ("nt", ctypes.c_int),
                ("nsrc", ctypes.c_int),
                ("src_xyz", ctypes.c_void_p),
                ("src_wav", ctypes.c_void_p),
                ("nrec", ctypes.c_int),
                ("rec_xyz", ctypes.c_void_p),
                ("d_obs", ctypes.c_void_p),
                ("rec_out", ctypes.c_void_p),
                ("grad_out", ctypes.c_void_p),
                ("misfit_out", ctypes.c_void_p)]


class wf_shot(ctypes.Structure):
    _fields_ = [("nsrc", ctypes.c_int),
                ("src_xyz", ctypes.c_void_p),
                ("src_wav", ctypes.c_void_p),
                ("nrec", ctypes.c_int),
                ("rec_xyz", ctypes.c_void_p),
                ("d_obs", ctypes.c_void_p),
                ("d_pred", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libwavefd.so is not built (run __graft_entry__.build() or "
                          "python paper_1808_01995_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    I64 = ctypes.c_int64
    D = ctypes.c_double
    sig = {
        "wf_last_error": (ctypes.c_char_p, []),
        "wf_version": (I, []),
        "wf_critical_dt": (D, [ctypes.POINTER(wf_geom), D]),
        "wf_geom_shape": (I, [ctypes.POINTER(wf_geom), P, P]),
        "wf_model_create": (I, [ctypes.POINTER(wf_geom), P, P, P]),
        "wf_model_set_m": (I, [P, P, P]),
        "wf_model_bytes": (I64, [P]),
        "wf_model_graph_launches": (I64, [P]),
        "wf_model_trim": (I, [P]),
        "wf_graph_enable": (I, [I]),
        "wf_two_step_enable": (I, [I]),
        "wf_model_destroy": (I, [P]),
        "wf_forward": (I, [P, D, I, I, P, P, I, P, P, P, I, P]),
        "wf_forward_noalloc": (I, [P, D, I, I, P, P, I, P, P, P]),
        "wf_adjoint": (I, [P, D, I, I, P, P, I, P, P, P]),
        "wf_gradient": (I, [P, D, I, I, P, P, I, P, P, P, I, I64, P]),
        "wf_fwi_gradient": (I, [P, D, I, I, ctypes.POINTER(wf_shot), P, P, I, I64, P]),
        "wf_born": (I, [P, D, I, I, P, P, P, I, P, P, P, P]),
        "wf_model_update": (I, [P, P, D, D, D, P, P]),
        "wf_revolve_forward_steps": (I64, [I64, I]),
        "wf_revolve_schedule": (I64, [I64, I, P, P, P, I64]),
        "wf_profile_enable": (I, [I]),
        "wf_profile_runs_enable": (I, [I]),
        "wf_profile_read": (I, [I, P, P, I]),
        "wf_profile_step_launches": (I, [I, P, I]),
        "wf_stream_bandwidth": (I, [I64, I, P]),
        "wf_model_ghost_nonzero": (I, [P, P]),
        "wf_validate_enable": (I, [I]),
        "wf_engine_create": (I, [I64, I, P]),
        "wf_engine_submit": (I, [P, ctypes.POINTER(wf_request), P]),
        "wf_engine_submit_on": (I, [P, ctypes.POINTER(wf_request), P, I, P]),
        "wf_engine_poll": (I, [P, P, P, I, P, I]),
        "wf_engine_request_bytes": (I, [ctypes.POINTER(wf_request), I64, P]),
        "wf_engine_stats": (I, [P, P, P, P, P]),
        "wf_engine_paths": (I, [P, P, P, P]),
        "wf_engine_destroy": (I, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()

# every symbol declared in include/wavefd.h
EXPORTS = ("wf_last_error", "wf_version", "wf_critical_dt", "wf_geom_shape", "wf_model_create",
           "wf_model_set_m", "wf_model_bytes", "wf_model_graph_launches", "wf_graph_enable",
           "wf_two_step_enable",
           "wf_model_trim",
           "wf_model_destroy", "wf_forward", "wf_forward_noalloc", "wf_adjoint",
           "wf_gradient", "wf_born", "wf_fwi_gradient", "wf_model_update", "wf_revolve_forward_steps", "wf_revolve_schedule",
           "wf_profile_enable", "wf_profile_runs_enable", "wf_profile_read", "wf_profile_step_launches",
           "wf_stream_bandwidth", "wf_model_ghost_nonzero", "wf_validate_enable",
           "wf_engine_create", "wf_engine_submit", "wf_engine_submit_on", "wf_engine_request_bytes",
           "wf_engine_poll", "wf_engine_stats", "wf_engine_paths", "wf_engine_destroy")


def _check(st: int):
    if st != WF_OK:
        raise WaveFDError(st, lib.wf_last_error().decode(errors="replace"))


def make_geom(shape: Sequence[int], spacing: Sequence[float], nbl: int, space_order: int,
              c_ref: float, origin: Optional[Sequence[float]] = None, R: float = 0.0,
              eta_power: int = 0) -> wf_geom:
    """Geometry of a physical grid `shape` (2 or 3 axes) with an nbl-node
    damping layer outside it on every side."""
    g = wf_geom()
    nd = len(shape)
    g.ndim = nd
    for a in range(nd):
        g.n[a] = int(shape[a])
        g.h[a] = float(spacing[a])
        g.origin[a] = float(origin[a]) if origin is not None else 0.0
    for a in range(nd, 3):
        g.n[a] = 1
        g.h[a] = 1.0
    g.nbl = int(nbl)
    g.space_order = int(space_order)
    g.c_ref = float(c_ref)
    g.R = float(R)
    g.eta_power = int(eta_power)
    return g


def _ptr(t) -> Optional[int]:
    """Device pointer of a contiguous float32 CUDA tensor (None passes NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError("expected a contiguous float32 tensor")
    return t.data_ptr()


def _host(xyz) -> tuple:
    if xyz is None:
        return 0, None, None
    a = np.ascontiguousarray(np.atleast_2d(np.asarray(xyz, dtype=np.float64)))
    if a.size == 0:
        return 0, None, a
    return a.shape[0], a.ctypes.data_as(ctypes.c_void_p), a


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


def wf_version() -> int:
    return lib.wf_version()


def wf_last_error() -> str:
    return lib.wf_last_error().decode(errors="replace")


def wf_critical_dt(geom: wf_geom, vmax: float) -> float:
    v = lib.wf_critical_dt(ctypes.byref(geom), float(vmax))
    if v < 0:
        raise WaveFDError(WF_E_ARG, wf_last_error())
    return v


def wf_geom_shape(geom: wf_geom):
    shp = (ctypes.c_int64 * 3)()
    n = ctypes.c_int64()
    _check(lib.wf_geom_shape(ctypes.byref(geom), shp, ctypes.byref(n)))
    return tuple(int(shp[a]) for a in range(geom.ndim)), int(n.value)


def wf_model_create(geom: wf_geom, m, stream=None) -> ctypes.c_void_p:
    out = ctypes.c_void_p()
    _check(lib.wf_model_create(ctypes.byref(geom), _ptr(m), _stream(stream), ctypes.byref(out)))
    return out


def wf_model_set_m(model, m, stream=None):
    _check(lib.wf_model_set_m(model, _ptr(m), _stream(stream)))


def wf_model_bytes(model) -> int:
    return int(lib.wf_model_bytes(model))


def wf_model_graph_launches(model) -> int:
    return int(lib.wf_model_graph_launches(model))


def wf_model_trim(model):
    _check(lib.wf_model_trim(model))


def wf_graph_enable(on: bool):
    _check(lib.wf_graph_enable(1 if on else 0))


def wf_two_step_enable(mode: int):
    """Two updates per launch in forward and adjoint loops: 0 off, 1 where
    measured faster (the default), 2 for every compiled order (4 and 8, 2D
    and 3D)."""
    _check(lib.wf_two_step_enable(int(mode)))


def wf_model_destroy(model):
    _check(lib.wf_model_destroy(model))


def wf_forward(model, dt: float, nt: int, src_xyz, src_wav, rec_xyz, rec_out,
               u_save=None, save_every: int = 1, stream=None):
    ns, sp, _sa = _host(src_xyz)
    nr, rp, _ra = _host(rec_xyz)
    _check(lib.wf_forward(model, float(dt), int(nt), ns, sp, _ptr(src_wav) if ns else None,
                          nr, rp, _ptr(rec_out) if nr else None, _ptr(u_save), int(save_every),
                          _stream(stream)))


def wf_forward_noalloc(model, dt: float, nt: int, src_xyz, src_wav, rec_xyz, rec_out, stream=None):
    """wf_forward without device allocation (tables in the library's fixed
    per-GPU scratch; raises WaveFDError(WF_E_BUDGET) beyond it)."""
    ns, sp, _sa = _host(src_xyz)
    nr, rp, _ra = _host(rec_xyz)
    _check(lib.wf_forward_noalloc(model, float(dt), int(nt), ns, sp, _ptr(src_wav) if ns else None,
                                  nr, rp, _ptr(rec_out) if nr else None, _stream(stream)))


def wf_adjoint(model, dt: float, nt: int, rec_xyz, rec_in, src_xyz, src_out, stream=None):
    nr, rp, _ra = _host(rec_xyz)
    ns, sp, _sa = _host(src_xyz)
    _check(lib.wf_adjoint(model, float(dt), int(nt), nr, rp, _ptr(rec_in) if nr else None,
                          ns, sp, _ptr(src_out) if ns else None, _stream(stream)))


def wf_gradient(model, dt: float, nt: int, src_xyz, src_wav, rec_xyz, residual, grad_out,
                n_checkpoints: int = 0, hbm_budget_bytes: int = 0, stream=None):
    ns, sp, _sa = _host(src_xyz)
    nr, rp, _ra = _host(rec_xyz)
    _check(lib.wf_gradient(model, float(dt), int(nt), ns, sp, _ptr(src_wav) if ns else None,
                           nr, rp, _ptr(residual) if nr else None, _ptr(grad_out),
                           int(n_checkpoints), int(hbm_budget_bytes), _stream(stream)))


def wf_born(model, dt: float, nt: int, src_xyz, src_wav, dm, rec_xyz, drec_out, rec_out=None,
            stream=None):
    ns, sp, _sa = _host(src_xyz)
    nr, rp, _ra = _host(rec_xyz)
    _check(lib.wf_born(model, float(dt), int(nt), ns, sp, _ptr(src_wav) if ns else None, _ptr(dm),
                       nr, rp, _ptr(drec_out) if nr else None,
                       _ptr(rec_out) if (rec_out is not None and nr) else None, _stream(stream)))


def wf_fwi_gradient(model, dt: float, nt: int, shots, grad_out, n_checkpoints: int = 0,
                    hbm_budget_bytes: int = 0, stream=None) -> float:
    """shots: sequence of (src_xyz, src_wav, rec_xyz, d_obs, d_pred or None).
    Returns the summed misfit; grad_out receives the summed gradient."""
    arr = (wf_shot * len(shots))()
    keep = []
    for i, (sxyz, wav, rxyz, dob, dpred) in enumerate(shots):
        ns, sp, sa = _host(sxyz)
        nr, rp, ra = _host(rxyz)
        keep += [sa, ra]
        arr[i] = wf_shot(ns, sp, _ptr(wav) if ns else None, nr, rp, _ptr(dob) if nr else None,
                         _ptr(dpred) if (dpred is not None and nr) else None)
    phi = ctypes.c_double()
    _check(lib.wf_fwi_gradient(model, float(dt), int(nt), len(shots), arr, _ptr(grad_out),
                               ctypes.byref(phi), int(n_checkpoints), int(hbm_budget_bytes),
                               _stream(stream)))
    del keep
    return float(phi.value)


def wf_model_update(model, grad, alpha: float, m_lo: float, m_hi: float = float("inf"),
                    m_out=None, stream=None):
    _check(lib.wf_model_update(model, _ptr(grad), float(alpha), float(m_lo), float(m_hi),
                               _ptr(m_out), _stream(stream)))


def wf_revolve_forward_steps(steps: int, snaps: int) -> int:
    return int(lib.wf_revolve_forward_steps(int(steps), int(snaps)))


WF_REVOLVE_ADVANCE, WF_REVOLVE_TAKESHOT, WF_REVOLVE_RESTORE, WF_REVOLVE_REVERSE, WF_REVOLVE_FREE = range(5)


def wf_revolve_schedule(steps: int, snaps: int):
    """The checkpoint schedule wf_gradient runs: a list of (kind, at, arg)."""
    n = int(lib.wf_revolve_schedule(int(steps), int(snaps), None, None, None, 0))
    if n < 0:
        raise WaveFDError(n, wf_last_error())
    kind = np.zeros(n, dtype=np.int32)
    at = np.zeros(n, dtype=np.int64)
    arg = np.zeros(n, dtype=np.int64)
    m = int(lib.wf_revolve_schedule(int(steps), int(snaps), kind.ctypes.data, at.ctypes.data,
                                    arg.ctypes.data, n))
    if m != n:
        raise WaveFDError(WF_E_STATE, "schedule length changed")
    return list(zip(kind.tolist(), at.tolist(), arg.tolist()))


WF_KERNEL_STEP = 0
WF_KERNEL_INJECT = 1
WF_KERNEL_SAMPLE = 2
WF_KERNEL_STEP_RUN = 3
WF_KERNEL_STEP2 = 4
WF_KERNEL_STEP2_RUN = 5
WF_STEP_LAUNCHES_TWO = 4   # wf_profile_step_launches: two-update launches


def wf_profile_enable(on):
    """True/1: time every launch; n > 1: every n-th launch of each kernel; 0: off."""
    _check(lib.wf_profile_enable(int(on)))


def wf_profile_runs_enable(on):
    """Time each forward/adjoint loop's run of step launches as one span."""
    _check(lib.wf_profile_runs_enable(1 if on else 0))


def wf_profile_step_launches(mode: int, reset: bool = False) -> int:
    """Step-kernel launches in `mode` (0 plain, 1 imaging, 2 Born source,
    3 volume source) since the last reset."""
    n = ctypes.c_int64()
    _check(lib.wf_profile_step_launches(int(mode), ctypes.byref(n), 1 if reset else 0))
    return n.value


def wf_profile_read(kind: int, reset: bool = False):
    """(summed device ms, launch count) of kernel `kind` since the last reset."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib.wf_profile_read(int(kind), ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
    return ms.value, n.value


def wf_validate_enable(on):
    """Post-run checks that every output value is finite (WF_E_NONFINITE)."""
    _check(lib.wf_validate_enable(1 if on else 0))


def wf_model_ghost_nonzero(model) -> int:
    """Nonzero values in the ghost planes and row padding of the model's
    fields (0 after any correct run)."""
    n = ctypes.c_int64()
    _check(lib.wf_model_ghost_nonzero(model, ctypes.byref(n)))
    return n.value


def wf_stream_bandwidth(n_floats: int, reps: int = 20) -> float:
    """GB/s of a plain 3-read + 1-write float4 stream over n_floats-float
    arrays (the step kernel's bytes per node, no stencil): the roofline's
    measured reference."""
    g = ctypes.c_double()
    _check(lib.wf_stream_bandwidth(int(n_floats), int(reps), ctypes.byref(g)))
    return g.value


def wf_engine_create(hbm_budget_bytes: int, max_slots: int):
    out = ctypes.c_void_p()
    _check(lib.wf_engine_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(out)))
    return out


def wf_engine_submit(engine, req: wf_request) -> int:
    t = ctypes.c_uint64()
    _check(lib.wf_engine_submit(engine, ctypes.byref(req), ctypes.byref(t)))
    return int(t.value)


def wf_engine_submit_on(engine, req: wf_request, stream=None) -> int:
    """Submit with the engine's work ordered after what the caller queued on
    `stream` (torch's current stream by default): no host synchronisation."""
    t = ctypes.c_uint64()
    _check(lib.wf_engine_submit_on(engine, ctypes.byref(req), _stream(stream), 1, ctypes.byref(t)))
    return int(t.value)


def wf_engine_request_bytes(req: wf_request, hbm_budget_bytes: int) -> int:
    """Bytes the engine reserves for `req` under that budget."""
    b = ctypes.c_int64()
    _check(lib.wf_engine_request_bytes(ctypes.byref(req), int(hbm_budget_bytes), ctypes.byref(b)))
    return b.value


def wf_engine_poll(engine, cap: int = 64, wait_ms: int = 0):
    tickets = (ctypes.c_uint64 * cap)()
    status = (ctypes.c_int * cap)()
    n = ctypes.c_int()
    _check(lib.wf_engine_poll(engine, tickets, status, int(cap), ctypes.byref(n), int(wait_ms)))
    return [(int(tickets[i]), int(status[i])) for i in range(n.value)]


def wf_engine_stats(engine):
    q, r, c, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib.wf_engine_stats(engine, ctypes.byref(q), ctypes.byref(r), ctypes.byref(c), ctypes.byref(b)))
    return {"queued": q.value, "running": r.value, "completed": c.value, "bytes_in_use": b.value}


def wf_engine_paths(engine):
    """Completed requests per path: resident teams, batched launches, workers."""
    t, b, w = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib.wf_engine_paths(engine, ctypes.byref(t), ctypes.byref(b), ctypes.byref(w)))
    return {"teams": t.value, "batched": b.value, "workers": w.value}


def wf_engine_destroy(engine):
    _check(lib.wf_engine_destroy(engine))
