"""Seeded synthetic inputs for the acoustic propagator: velocity models, source
wavelets and acquisition geometry.

This module only *generates inputs*. It holds none of the method's arithmetic
(no stencil weights, no damping, no time stepping, no interpolation): both the
FP64 oracle and the GPU library receive what is generated here as plain arrays
and coordinates, and each side derives everything else on its own.

Units throughout: metres, milliseconds, km/s (= m/ms). Frequencies are given in
Hz and converted to 1/ms where a wavelet is sampled.

The workloads mirror the paper's setting: an acoustic medium described by its
velocity (Section "Symbolic definition of finite difference stencils",
eq. acoustic), a point source with a Ricker signature and receivers near the
surface (Section "Acoustic forward modelling operator"); the concrete sizes are
those of the five benchmark configurations described in the repository's design
notes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

__all__ = [
    "ricker",
    "Config",
    "config",
    "CONFIG_NAMES",
    "smooth_random_velocity",
    "smooth_random_velocity_device",
    "two_layer_velocity",
    "gaussian_anomaly_velocity",
    "line_receivers",
    "grid_receivers",
    "band_limited_noise",
    "serving_requests",
]


def ricker(nt: int, dt: float, f0_hz: float, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet sampled at t_n = n*dt (ms), amplitude 1 at the delay t0.

    r(t) = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2), tau = t - t0,
    with f0 in 1/ms and, by default, t0 = 1.5 / f0 (the textbook delay that makes
    the wavelet start at ~1e-10 of its peak).
    """
    f0 = f0_hz * 1e-3
    if t0 is None:
        t0 = 1.5 / f0
    t = np.arange(nt, dtype=np.float64) * dt
    a = (math.pi * f0 * (t - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def smooth_random_velocity(shape, seed: int, sigma: float = 8.0,
                           vmin: float = 1.5, vmax: float = 4.5) -> np.ndarray:
    """Gaussian-filtered N(0,1) noise rescaled to [vmin, vmax] km/s."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(tuple(shape))
    s = gaussian_filter(noise, sigma=sigma, mode="reflect", truncate=4.0)
    lo, hi = float(s.min()), float(s.max())
    if hi <= lo:
        return np.full(shape, 0.5 * (vmin + vmax))
    return vmin + (vmax - vmin) * (s - lo) / (hi - lo)


def smooth_random_velocity_device(shape, seed: int, sigma: float = 8.0, vmin: float = 1.5,
                                  vmax: float = 4.5, device="cuda"):
    """The recipe of smooth_random_velocity generated on a torch device, for
    workloads whose host-side filtering would take minutes (the serving mix
    reaches 384^3): N(0,1) noise from a device generator seeded with `seed`
    (a different random stream from the host recipe), smoothed by the same
    separable Gaussian truncated at 4 sigma with half-sample-symmetric edges
    (scipy's mode 'reflect'), min-max rescaled to [vmin, vmax] km/s.
    Returns a float64 tensor on `device`."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    x = torch.randn(tuple(int(n) for n in shape), generator=gen, device=device, dtype=torch.float32)
    r = int(4.0 * float(sigma) + 0.5)
    taps = np.exp(-0.5 * (np.arange(-r, r + 1) / float(sigma)) ** 2)
    taps /= taps.sum()
    for ax in range(x.dim()):
        n = x.shape[ax]
        k = np.arange(-r, n + r) % (2 * n)
        k = np.where(k >= n, 2 * n - 1 - k, k)
        xp = x.index_select(ax, torch.from_numpy(k).to(device))
        y = torch.zeros_like(x)
        for t in range(2 * r + 1):
            y.add_(xp.narrow(ax, t, n), alpha=float(taps[t]))
        x = y
    x = x.double()
    lo, hi = float(x.min()), float(x.max())
    if hi <= lo:
        return torch.full_like(x, 0.5 * (vmin + vmax))
    return vmin + (vmax - vmin) * (x - lo) / (hi - lo)


def two_layer_velocity(shape, v_top: float = 1.5, v_bottom: float = 2.5,
                       interface: Optional[int] = None) -> np.ndarray:
    """Flat interface normal to the last (depth) axis at index `interface`
    (default: mid-depth). Cells with depth index < interface get v_top."""
    shape = tuple(shape)
    nz = shape[-1]
    if interface is None:
        interface = nz // 2
    v = np.full(shape, v_bottom, dtype=np.float64)
    v[..., :interface] = v_top
    return v


def gaussian_anomaly_velocity(shape, background: float = 2.0, peak: float = 2.5,
                              radius_cells: float = 30.0,
                              centre: Optional[Tuple[float, ...]] = None) -> np.ndarray:
    """background + (peak - background) * exp(-r^2 / radius^2), r in cells."""
    shape = tuple(shape)
    if centre is None:
        centre = tuple((n - 1) / 2.0 for n in shape)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    r2 = sum((g - c) ** 2 for g, c in zip(grids, centre))
    return background + (peak - background) * np.exp(-r2 / radius_cells ** 2)


def line_receivers(n: int, x0: float, x1: float, depth: float, ndim: int = 2,
                   y: Optional[float] = None) -> np.ndarray:
    """n receivers evenly spaced in x from x0 to x1 at a fixed depth.
    Returns (n, ndim) coordinates in metres ordered (x, z) or (x, y, z)."""
    xs = np.linspace(x0, x1, n) if n > 1 else np.array([x0], dtype=np.float64)
    if ndim == 2:
        return np.stack([xs, np.full(n, depth)], axis=1)
    return np.stack([xs, np.full(n, y if y is not None else 0.0), np.full(n, depth)], axis=1)


def grid_receivers(nx: int, ny: int, extent_x: float, extent_y: float,
                   depth: float) -> np.ndarray:
    """nx*ny receivers on a regular areal grid, x_i = i*extent_x/(nx-1)."""
    xs = np.arange(nx, dtype=np.float64) * (extent_x / (nx - 1))
    ys = np.arange(ny, dtype=np.float64) * (extent_y / (ny - 1))
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, depth)], axis=1)


def band_limited_noise(nt: int, ntr: int, dt: float, f0_hz: float, seed: int) -> np.ndarray:
    """N(0,1) noise of shape (nt, ntr) convolved in time with a zero-delay Ricker
    of peak frequency f0: random traces with a seismic-like spectrum (used as
    the random vectors of dot tests)."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((nt, ntr))
    f0 = f0_hz * 1e-3
    half = int(math.ceil(1.5 / (f0 * dt)))
    t = np.arange(-half, half + 1) * dt
    a = (math.pi * f0 * t) ** 2
    w = (1.0 - 2.0 * a) * np.exp(-a)
    out = np.empty_like(noise)
    for r in range(ntr):
        out[:, r] = np.convolve(noise[:, r], w, mode="full")[half:half + nt]
    return out


@dataclasses.dataclass
class Config:
    """One workload: physical grid, spacing, layer width, order, steps and the
    acquisition. `velocity()` returns the physical-grid velocity (km/s)."""
    name: str
    shape: Tuple[int, ...]
    spacing: Tuple[float, ...]
    nbl: int
    space_order: int
    steps: int
    f0_hz: float
    src: np.ndarray
    rec: np.ndarray
    kind: str = "smooth"
    seed: int = 0
    dt_factor: float = 0.5
    velocity_args: dict = dataclasses.field(default_factory=dict)

    @property
    def ndim(self) -> int:
        return len(self.shape)

    @property
    def nt(self) -> int:
        # N updates produce N+1 samples t_0 .. t_N
        return self.steps + 1

    @property
    def extent(self) -> Tuple[float, ...]:
        return tuple((n - 1) * h for n, h in zip(self.shape, self.spacing))

    def velocity(self) -> np.ndarray:
        if self.kind == "constant":
            return np.full(self.shape, float(self.velocity_args.get("v", 1.5)))
        if self.kind == "smooth":
            return smooth_random_velocity(self.shape, self.seed, **self.velocity_args)
        if self.kind == "two_layer":
            return two_layer_velocity(self.shape, **self.velocity_args)
        if self.kind == "anomaly":
            return gaussian_anomaly_velocity(self.shape, **self.velocity_args)
        raise ValueError(self.kind)


CONFIG_NAMES = ("c1_2d", "c2_3d_so8", "c3_sweep", "c4_gradient", "c5_small")


def config(name: str, space_order: Optional[int] = None, scale: Optional[int] = None,
           steps: Optional[int] = None) -> Config:
    """The benchmark workloads. `scale` replaces the physical grid size N (all
    axes) keeping the physical layout proportional; `steps` replaces the step
    count; both exist for reduced-size parity runs."""
    if name == "c1_2d":
        n = scale or 101
        h = 10.0
        ext = (n - 1) * h
        return Config(name, (n, n), (h, h), nbl=20, space_order=space_order or 4,
                      steps=steps or 500, f0_hz=10.0,
                      src=np.array([[ext / 2, ext / 2]]),
                      rec=line_receivers(n, 0.0, ext, 20.0, ndim=2),
                      kind="constant", velocity_args={"v": 1.5})
    if name == "c2_3d_so8":
        n = scale or 256
        h = 10.0
        ext = (n - 1) * h
        nr = 128 if scale is None else max(2, min(128, n // 2))
        # source half a cell off the grid in x and y, on a node in z
        return Config(name, (n, n, n), (h, h, h), nbl=40, space_order=space_order or 8,
                      steps=steps or 1000, f0_hz=15.0,
                      src=np.array([[ext / 2.0, ext / 2.0, 20.0]]),
                      rec=grid_receivers(nr, nr, ext, ext, 20.0),
                      kind="smooth", seed=2, velocity_args={"sigma": 8.0 * n / 256.0})
    if name == "c3_sweep":
        n = scale or 512
        h = 10.0
        ext = (n - 1) * h
        return Config(name, (n, n, n), (h, h, h), nbl=40, space_order=space_order or 8,
                      steps=steps or 500, f0_hz=15.0,
                      src=np.array([[ext / 2.0, ext / 2.0, 20.0]]),
                      rec=line_receivers(n, 0.0, ext, 20.0, ndim=3, y=ext / 2.0),
                      kind="two_layer", velocity_args={"interface": n // 2})
    if name == "c4_gradient":
        n = scale or 200
        h = 10.0
        ext = (n - 1) * h
        nr = 100 if scale is None else max(2, min(100, n // 2))
        c = (n - 1) / 2.0
        return Config(name, (n, n, n), (h, h, h), nbl=40 if scale is None else min(40, max(8, n // 5)),
                      space_order=space_order or 8, steps=steps or 2000, f0_hz=10.0,
                      src=np.array([[ext / 2.0, ext / 2.0, 20.0]]),
                      rec=grid_receivers(nr, nr, ext, ext, 20.0),
                      kind="anomaly",
                      velocity_args={"radius_cells": 30.0 * n / 200.0, "centre": (c, c, c)})
    if name == "c5_small":
        # a small 2D request of the serving mix
        n = scale or 256
        h = 10.0
        ext = (n - 1) * h
        return Config(name, (n, n), (h, h), nbl=40, space_order=space_order or 8,
                      steps=steps or 500, f0_hz=10.0,
                      src=np.array([[ext / 2.0, 20.0]]),
                      rec=line_receivers(n, 0.0, ext, 20.0, ndim=2),
                      kind="smooth", seed=5)
    raise KeyError(name)


def serving_requests(n_requests: int = 256, seed: int = 5, scale_down: int = 1,
                     max_steps: Optional[int] = None):
    """Draw the mixed serving workload: a list of dicts with keys
    ndim, n (physical points per axis), space_order, steps, kind ('forward' or
    'gradient'), seed (for the velocity), perturb (model perturbation for the
    observed data of gradient requests). `scale_down` divides grid sizes for
    reduced runs."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_requests):
        ndim = 2 if rng.random() < 0.5 else 3
        if ndim == 2:
            n = int(rng.integers(256, 2049))
        else:
            n = int(rng.integers(128, 385))
        n = max(16, n // scale_down)
        so = int(rng.choice([4, 8, 12]))
        steps = int(rng.integers(500, 2001))
        if max_steps is not None:
            steps = min(steps, max_steps)
        kind = "forward" if rng.random() < 0.75 else "gradient"
        out.append({"id": i, "ndim": ndim, "n": n, "space_order": so, "steps": steps,
                    "kind": kind, "seed": 1000 + i, "perturb": 0.05})
    return out
