"""Python front-end of the gfx950 propagator.

`Propagator` owns one device-resident model (squared slowness on the
computational grid plus the library's wavefields) and exposes forward
modelling, the adjoint and the gradient; `ModelingFunction` wraps forward and
gradient as a torch.autograd.Function (forward: m -> shot record; backward:
J^T applied to the record's gradient, Section "Full-Waveform Inversion",
eqs. AS and Grad).

Model set-up follows the paper's acoustic parameterisation (eq. acoustic):
m = 1 / v^2 on the physical grid, padded by nbl nodes of edge-replicated
values on every side to form the computational grid that carries the damping
layer (Section "Boundary conditions"). Everything after the set-up runs in the
library's kernels.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import _abi
from ._abi import make_geom


def pad_replicate(x: torch.Tensor, nbl: int) -> torch.Tensor:
    """Edge-replicating pad by nbl on every side of a 2D or 3D tensor
    (differentiable; its adjoint folds the layer back onto the edges)."""
    if nbl == 0:
        return x
    nd = x.dim()
    return torch.nn.functional.pad(x[None, None], (nbl,) * (2 * nd), mode="replicate")[0, 0]


def slowness_sq(v_phys, nbl: int, device="cuda") -> torch.Tensor:
    """m = 1/v^2 on the computational grid (float32, device)."""
    v = torch.as_tensor(np.asarray(v_phys), dtype=torch.float64)
    m = 1.0 / (v * v)
    return pad_replicate(m, nbl).to(device=device, dtype=torch.float32).contiguous()


class Propagator:
    """One model on the GPU.

    shape: physical grid (2 or 3 axes); spacing in metres; nbl damping-layer
    width; space_order k in 4..16; c_ref the damping reference velocity
    (default: the largest velocity of the model at creation, then frozen);
    origin the physical origin (m); R and eta_power the damping profile's
    nominal reflection coefficient and power (0: 1e-3 and 2).
    """

    def __init__(self, v_phys=None, spacing: Sequence[float] = (10.0, 10.0, 10.0), nbl: int = 40,
                 space_order: int = 8, c_ref: Optional[float] = None,
                 origin: Optional[Sequence[float]] = None, m: Optional[torch.Tensor] = None,
                 shape: Optional[Sequence[int]] = None, device="cuda", R: float = 0.0,
                 eta_power: int = 0):
        if m is None:
            if v_phys is None:
                raise ValueError("give v_phys or m")
            v = np.asarray(v_phys, dtype=np.float64)
            shape = v.shape
            if c_ref is None:
                c_ref = float(v.max())
            m = slowness_sq(v, nbl, device)
        else:
            if shape is None:
                shape = tuple(int(n) - 2 * nbl for n in m.shape)
            if c_ref is None:
                c_ref = float(1.0 / torch.sqrt(m.min()).item())
        self.shape = tuple(int(n) for n in shape)
        self.ndim = len(self.shape)
        self.spacing = tuple(float(h) for h in spacing[: self.ndim])
        self.nbl = int(nbl)
        self.space_order = int(space_order)
        self.c_ref = float(c_ref)
        self.geom = make_geom(self.shape, self.spacing, self.nbl, self.space_order, self.c_ref, origin,
                              R, eta_power)
        self.comp_shape, self.npoints = _abi.wf_geom_shape(self.geom)
        if tuple(m.shape) != self.comp_shape:
            raise ValueError("m has shape %s, expected %s" % (tuple(m.shape), self.comp_shape))
        self.device = m.device
        self.m = m.contiguous()
        self.handle = _abi.wf_model_create(self.geom, self.m)

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            _abi.wf_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def trim(self):
        """Free the gradient workspace the model keeps between calls."""
        _abi.wf_model_trim(self.handle)

    def set_m(self, m: torch.Tensor):
        m = m.to(device=self.device, dtype=torch.float32).contiguous()
        if tuple(m.shape) != self.comp_shape:
            raise ValueError("m has shape %s, expected %s" % (tuple(m.shape), self.comp_shape))
        _abi.wf_model_set_m(self.handle, m)
        self.m = m

    @property
    def vmax(self) -> float:
        return float(1.0 / torch.sqrt(self.m.min()).item())

    def critical_dt(self, vmax: Optional[float] = None) -> float:
        return _abi.wf_critical_dt(self.geom, vmax if vmax is not None else self.vmax)

    # ------------------------------------------------------------------
    def _series(self, a, nt, npts, name):
        t = torch.as_tensor(a, dtype=torch.float32, device=self.device).contiguous()
        if t.dim() == 1:
            t = t[:, None].contiguous()
        if tuple(t.shape) != (nt, npts):
            raise ValueError("%s must be [nt, %d]" % (name, npts))
        return t

    def forward(self, dt: float, nt: int, src_xyz, src_wav, rec_xyz, save_every: Optional[int] = None,
                rec_out: Optional[torch.Tensor] = None):
        """Shot record d = P_r A(m)^-1 P_s^T q, [nt, nrec] float32 on the GPU.
        With save_every, also returns the saved wavefields [k, *comp_shape]."""
        src_xyz = np.atleast_2d(np.asarray(src_xyz, dtype=np.float64))
        rec_xyz = np.atleast_2d(np.asarray(rec_xyz, dtype=np.float64))
        q = self._series(src_wav, nt, src_xyz.shape[0], "src_wav")
        if rec_out is None:
            rec_out = torch.empty((nt, rec_xyz.shape[0]), dtype=torch.float32, device=self.device)
        u = None
        if save_every:
            k = (nt - 1) // save_every + 1
            u = torch.empty((k,) + self.comp_shape, dtype=torch.float32, device=self.device)
        _abi.wf_forward(self.handle, dt, nt, src_xyz, q, rec_xyz, rec_out, u, save_every or 1)
        return (rec_out, u) if save_every else rec_out

    def adjoint(self, dt: float, nt: int, rec_xyz, rec_data, src_xyz):
        """x = P_s A(m)^-T P_r^T y, [nt, nsrc]."""
        src_xyz = np.atleast_2d(np.asarray(src_xyz, dtype=np.float64))
        rec_xyz = np.atleast_2d(np.asarray(rec_xyz, dtype=np.float64))
        y = self._series(rec_data, nt, rec_xyz.shape[0], "rec_data")
        out = torch.empty((nt, src_xyz.shape[0]), dtype=torch.float32, device=self.device)
        _abi.wf_adjoint(self.handle, dt, nt, rec_xyz, y, src_xyz, out)
        return out

    def gradient(self, dt: float, nt: int, src_xyz, src_wav, rec_xyz, residual,
                 n_checkpoints: int = 0, hbm_budget_bytes: int = 0):
        """J^T r on the computational grid for the residual r = P_r u - d_obs.
        n_checkpoints: s > 0 revolve states, -1 store all, 0 as many as the
        budget allows, -2 boundary-wavefield reconstruction (the gradient on
        the physical grid, 0 in the layer)."""
        src_xyz = np.atleast_2d(np.asarray(src_xyz, dtype=np.float64))
        rec_xyz = np.atleast_2d(np.asarray(rec_xyz, dtype=np.float64))
        q = self._series(src_wav, nt, src_xyz.shape[0], "src_wav")
        r = self._series(residual, nt, rec_xyz.shape[0], "residual")
        g = torch.empty(self.comp_shape, dtype=torch.float32, device=self.device)
        _abi.wf_gradient(self.handle, dt, nt, src_xyz, q, rec_xyz, r, g, n_checkpoints,
                         hbm_budget_bytes)
        return g


    def born(self, dt: float, nt: int, src_xyz, src_wav, dm: torch.Tensor, rec_xyz,
             return_background: bool = False):
        """Linearised modelling dd = J dm for a squared-slowness perturbation dm
        on the computational grid; with return_background also P_r u."""
        src_xyz = np.atleast_2d(np.asarray(src_xyz, dtype=np.float64))
        rec_xyz = np.atleast_2d(np.asarray(rec_xyz, dtype=np.float64))
        q = self._series(src_wav, nt, src_xyz.shape[0], "src_wav")
        dm = dm.to(device=self.device, dtype=torch.float32).contiguous()
        if tuple(dm.shape) != self.comp_shape:
            raise ValueError("dm has shape %s, expected %s" % (tuple(dm.shape), self.comp_shape))
        dd = torch.empty((nt, rec_xyz.shape[0]), dtype=torch.float32, device=self.device)
        d = torch.empty_like(dd) if return_background else None
        _abi.wf_born(self.handle, dt, nt, src_xyz, q, dm, rec_xyz, dd, d)
        return (dd, d) if return_background else dd

    def fwi_gradient(self, dt: float, nt: int, shots, n_checkpoints: int = 0,
                     hbm_budget_bytes: int = 0, return_pred: bool = False):
        """Multi-shot FWI objective and gradient at the current m: shots is a
        sequence of (src_xyz, src_wav [nt, nsrc], rec_xyz, d_obs [nt, nrec]).
        Returns (misfit, gradient on the computational grid) and, with
        return_pred, the predicted records."""
        marsh, preds = [], []
        for sxyz, wav, rxyz, dob in shots:
            sxyz = np.atleast_2d(np.asarray(sxyz, dtype=np.float64))
            rxyz = np.atleast_2d(np.asarray(rxyz, dtype=np.float64))
            q = self._series(wav, nt, sxyz.shape[0], "src_wav")
            d = self._series(dob, nt, rxyz.shape[0], "d_obs")
            dp = torch.empty_like(d) if return_pred else None
            preds.append(dp)
            marsh.append((sxyz, q, rxyz, d, dp))
        g = torch.empty(self.comp_shape, dtype=torch.float32, device=self.device)
        phi = _abi.wf_fwi_gradient(self.handle, dt, nt, marsh, g, n_checkpoints, hbm_budget_bytes)
        return (phi, g, preds) if return_pred else (phi, g)

    def update(self, grad: torch.Tensor, alpha: float, vmin: Optional[float] = None,
               vmax: Optional[float] = None):
        """Fixed-step update m <- m - alpha grad, with the velocity kept in
        [vmin, vmax] (as bounds 1/vmax^2 <= m <= 1/vmin^2)."""
        grad = grad.to(device=self.device, dtype=torch.float32).contiguous()
        if tuple(grad.shape) != self.comp_shape:
            raise ValueError("grad has shape %s, expected %s" % (tuple(grad.shape), self.comp_shape))
        m_lo = 1.0 / vmax ** 2 if vmax else float(np.finfo(np.float32).tiny)
        m_hi = 1.0 / vmin ** 2 if vmin else float("inf")
        m = torch.empty_like(self.m)
        _abi.wf_model_update(self.handle, grad, alpha, m_lo, m_hi, m)
        self.m = m


class ModelingFunction(torch.autograd.Function):
    """d = F(m): forward modelling as a differentiable function of the squared
    slowness on the computational grid. backward returns J^T (dL/dd), computed
    by the adjoint-state method with revolve checkpointing (n_checkpoints as in
    wf_gradient)."""

    @staticmethod
    def forward(ctx, m: torch.Tensor, prop: Propagator, dt: float, nt: int, src_xyz, src_wav,
                rec_xyz, n_checkpoints: int = 0):
        prop.set_m(m.detach())
        d = prop.forward(dt, nt, src_xyz, src_wav, rec_xyz)
        ctx.prop = prop
        ctx.args = (dt, nt, src_xyz, src_wav, rec_xyz, n_checkpoints)
        ctx.m = m.detach()
        return d

    @staticmethod
    def backward(ctx, grad_d: torch.Tensor):
        dt, nt, src_xyz, src_wav, rec_xyz, nck = ctx.args
        prop = ctx.prop
        if prop.m.data_ptr() != ctx.m.data_ptr():
            prop.set_m(ctx.m)
        g = prop.gradient(dt, nt, src_xyz, src_wav, rec_xyz, grad_d.contiguous().float(), nck)
        return g, None, None, None, None, None, None, None


def model_data(m: torch.Tensor, prop: Propagator, dt: float, nt: int, src_xyz, src_wav, rec_xyz,
               n_checkpoints: int = 0) -> torch.Tensor:
    return ModelingFunction.apply(m, prop, dt, nt, src_xyz, src_wav, rec_xyz, n_checkpoints)


class FWIObjective(torch.autograd.Function):
    """Phi(m) = sum_s 1/2 ||F_s(m) - d_obs,s||^2 as a differentiable scalar of
    the squared slowness on the computational grid (the multi-shot objective
    of Section "FWI using Devito operators"). The forward pass already forms
    the summed gradient (two wave solves per shot, wf_fwi_gradient); backward
    scales it by the incoming gradient. shots: sequence of (src_xyz, src_wav,
    rec_xyz, d_obs)."""

    @staticmethod
    def forward(ctx, m: torch.Tensor, prop: Propagator, dt: float, nt: int, shots,
                n_checkpoints: int = 0):
        prop.set_m(m.detach())
        phi, g = prop.fwi_gradient(dt, nt, shots, n_checkpoints)
        ctx.save_for_backward(g)
        return torch.tensor(phi, dtype=torch.float64, device=m.device)

    @staticmethod
    def backward(ctx, grad_phi: torch.Tensor):
        (g,) = ctx.saved_tensors
        return (grad_phi.to(torch.float32) * g), None, None, None, None, None


def fwi_objective(m: torch.Tensor, prop: Propagator, dt: float, nt: int, shots,
                  n_checkpoints: int = 0) -> torch.Tensor:
    return FWIObjective.apply(m, prop, dt, nt, shots, n_checkpoints)
