"""FP64 CPU oracle for the explicit finite-difference acoustic propagator.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package. It shares no code with the GPU
library (paper_1808_01995_amd) and never imports it.

What it computes follows the paper (arxiv 1808.01995, Devito v3.1.0):

* the acoustic wave equation in squared slowness with a damping term
  (eq. acoustic, eq. fdWE-abc),
* the order-k centred second difference per axis (eq. fdSpace) summed into the
  Laplacian, the second-order time difference (eq. fdTime) and the explicit
  update (eq. eulerfwd),
* multilinear sparse injection and interpolation inside the containing cell
  (Section "Sparse point interpolation"),
* the exact discrete adjoint A(m)^T (Section "Temporal discretization", the
  matrix view; Section "Discrete adjoint wave-equation and FWI gradient"),
* the adjoint-state gradient of the least-squares misfit (eqs. AS, Grad, Adj).

The heavy loops are plain C (wave.c / wave_core.inc, FP64, OpenMP); this module
holds the exact weights, the damping profile, the sparse-point weights, the
CFL limit and the ctypes glue.

Readings where the paper is silent or garbled (all listed in the design notes):
centre weight taken once (eq. fdSpace j = 0 term); centred first difference for
the damping term; damping profile eta = sum_a eta_max (d_a/nbl)^p with
eta_max = 3 ln(1/R) / (2 nbl h c_ref) (the paper only says 0 inside, growing
outward); injection weight dt^2/a, a = m + eta dt/2 (dt^2/m where eta = 0);
the layer lies outside the physical grid, which is edge-padded; multilinear
interpolation with the last-node tie-break; nt = steps + 1 samples.

Parity: the weights, the Laplacian, the time stepping, the adjoint and the
gradient are pinned by the tests (exact rationals and polynomial exactness,
Kronecker-sum Laplacian, dense brute-force solve, energy conservation,
dot test, complex-step derivative, Taylor slopes, analytic Green's function).
The damping constants are pinned only by the reading above (the paper prints
no formula): parity unpinned against the paper for eta_max itself.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from fractions import Fraction
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

__all__ = [
    "build", "fd_weights", "fd_weights_float", "abs_weight_sum", "critical_dt",
    "pad_edge", "damping_eta", "sparse_points", "Grid", "laplacian", "step",
    "forward", "adjoint", "gradient", "energy", "misfit", "fwi_objective", "fwi_update",
    "born",
]


# --------------------------------------------------------------------------
# build / load
# --------------------------------------------------------------------------
def build(force: bool = False) -> str:
    """Compile wave.c into liboracle.so next to this file (gcc, FP64, OpenMP)."""
    src = [os.path.join(_HERE, "wave.c"), os.path.join(_HERE, "wave_core.inc")]
    if not force and os.path.exists(_SO):
        if os.path.getmtime(_SO) >= max(os.path.getmtime(s) for s in src):
            return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-o", tmp, os.path.join(_HERE, "wave.c")]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        build()
        _lib_handle = ctypes.CDLL(_SO)
    return _lib_handle


class _GridC(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("M", ctypes.c_int),
                ("nx", ctypes.c_long), ("ny", ctypes.c_long), ("nz", ctypes.c_long),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("alpha", ctypes.c_double * 17)]


# --------------------------------------------------------------------------
# finite-difference weights (eq. fdSpace)
# --------------------------------------------------------------------------
def fd_weights(space_order: int) -> list:
    """Exact centred second-derivative weights [alpha_0, alpha_1..alpha_M] of
    accuracy order k = space_order (eq. fdSpace; taps +j and -j share alpha_j,
    the centre weight alpha_0 is applied once).

    Closed form of the standard centred weights:
        alpha_j = 2 (-1)^{j+1} (M!)^2 / (j^2 (M-j)! (M+j)!),  j = 1..M,
        alpha_0 = -2 sum_j alpha_j.
    """
    if space_order < 2 or space_order % 2:
        raise ValueError("space order must be even and >= 2")
    M = space_order // 2
    fM = math.factorial(M)
    a = [Fraction(0)] * (M + 1)
    for j in range(1, M + 1):
        a[j] = Fraction(2 * (-1) ** (j + 1) * fM * fM,
                        j * j * math.factorial(M - j) * math.factorial(M + j))
    a[0] = -2 * sum(a[1:])
    return a


def fd_weights_float(space_order: int) -> np.ndarray:
    return np.array([float(x) for x in fd_weights(space_order)], dtype=np.float64)


def abs_weight_sum(space_order: int) -> Fraction:
    """sum of |w| over all 2M+1 taps of the 1D stencil."""
    a = fd_weights(space_order)
    return abs(a[0]) + 2 * sum(abs(x) for x in a[1:])


def critical_dt(ndim: int, spacing: Sequence[float], space_order: int, vmax: float) -> float:
    """Von Neumann limit of the leapfrog update (eq. eulerfwd):
    dt^2 v^2 rho(-L) <= 4 with rho(-L) <= sum_a h_a^-2 sum|w|, i.e.
    dt_crit = 2 / (vmax sqrt(sum|w| * sum_a h_a^-2)). For equal spacing this is
    2 h / (vmax sqrt(D sum|w|))."""
    s = float(abs_weight_sum(space_order))
    inv = sum(1.0 / (h * h) for h in spacing[:ndim])
    return 2.0 / (vmax * math.sqrt(s * inv))


# --------------------------------------------------------------------------
# model set-up: padding, damping layer (Section "Boundary conditions")
# --------------------------------------------------------------------------
def pad_edge(v_phys: np.ndarray, nbl: int) -> np.ndarray:
    """The damping layer lies outside the physical grid (reading): every axis
    is padded by nbl nodes on both sides, replicating the edge value."""
    return np.pad(np.asarray(v_phys, dtype=np.float64), nbl, mode="edge")


def damping_eta(shape_phys: Sequence[int], nbl: int, spacing: Sequence[float],
                c_ref: float, R: float = 1e-3, power: int = 2) -> np.ndarray:
    """Damping coefficient eta on the computational grid (eq. fdWE-abc): zero on
    the physical grid and growing toward the outer edge (Section "Boundary
    conditions"). Profile (reading): eta = sum_a eta_max_a (d_a / nbl)^power,
    d_a = distance in nodes from the physical grid along axis a,
    eta_max_a = 3 ln(1/R) / (2 nbl h_a c_ref)."""
    shape_phys = tuple(int(n) for n in shape_phys)
    nd = len(shape_phys)
    eta = np.zeros(tuple(n + 2 * nbl for n in shape_phys), dtype=np.float64)
    if nbl == 0:
        return eta
    for a in range(nd):
        Nc = shape_phys[a] + 2 * nbl
        c = np.arange(Nc, dtype=np.float64)
        d = np.maximum(np.maximum(nbl - c, c - (nbl + shape_phys[a] - 1)), 0.0)
        emax = 3.0 * math.log(1.0 / R) / (2.0 * nbl * spacing[a] * c_ref)
        prof = emax * (d / nbl) ** power
        shp = [1] * nd
        shp[a] = Nc
        eta = eta + prof.reshape(shp)
    return eta


# --------------------------------------------------------------------------
# sparse points (Section "Sparse point interpolation")
# --------------------------------------------------------------------------
def sparse_points(coords: np.ndarray, spacing: Sequence[float], nbl: int,
                  shape_comp: Sequence[int], origin: Optional[Sequence[float]] = None
                  ) -> Tuple[np.ndarray, np.ndarray]:
    """Multilinear interpolation inside the containing cell.

    For a point with coordinates x_a (metres, relative to the physical origin)
    s_a = (x_a - o_a)/h_a + nbl, i_a = floor(s_a), f_a = s_a - i_a; on the last
    node (i_a = Nc_a - 1) the cell to its left is used with f_a = 1. The 2^D
    corner nodes delta in {0,1}^D get weights prod_a (delta_a ? f_a : 1 - f_a).
    Corner k has delta_a = bit (D-1-a) of k (x is the most significant bit).
    Returns (node linear indices int64 [n, 2^D], weights float64 [n, 2^D]).
    A point outside [0, Nc_a - 1] raises ValueError."""
    coords = np.atleast_2d(np.asarray(coords, dtype=np.float64))
    nd = len(shape_comp)
    if coords.shape[1] != nd:
        raise ValueError("coordinates must have %d columns" % nd)
    if origin is None:
        origin = [0.0] * nd
    n = coords.shape[0]
    K = 1 << nd
    base = np.zeros((n, nd), dtype=np.int64)
    frac = np.zeros((n, nd), dtype=np.float64)
    for a in range(nd):
        s = (coords[:, a] - origin[a]) / spacing[a] + nbl
        if np.any(s < 0) or np.any(s > shape_comp[a] - 1):
            raise ValueError("sparse point outside the computational grid")
        i = np.floor(s).astype(np.int64)
        f = s - i
        last = i >= shape_comp[a] - 1
        i[last] = shape_comp[a] - 2
        f[last] = 1.0
        base[:, a] = i
        frac[:, a] = f
    strides = [int(np.prod(shape_comp[a + 1:])) for a in range(nd)]
    node = np.zeros((n, K), dtype=np.int64)
    w = np.ones((n, K), dtype=np.float64)
    for k in range(K):
        for a in range(nd):
            bit = (k >> (nd - 1 - a)) & 1
            node[:, k] += (base[:, a] + bit) * strides[a]
            w[:, k] *= frac[:, a] if bit else (1.0 - frac[:, a])
    return node, w


# --------------------------------------------------------------------------
# grid description and the C kernels
# --------------------------------------------------------------------------
class Grid:
    """Computational grid: shape (Nc per axis, 2 or 3 axes), spacing (m) and
    space order."""

    def __init__(self, shape: Sequence[int], spacing: Sequence[float], space_order: int):
        self.shape = tuple(int(n) for n in shape)
        self.ndim = len(self.shape)
        if self.ndim not in (2, 3):
            raise ValueError("2D or 3D only")
        self.spacing = tuple(float(h) for h in spacing)
        self.space_order = int(space_order)
        self.M = self.space_order // 2
        if self.M > 16:
            raise ValueError("space order up to 32")
        self.alpha = fd_weights_float(self.space_order)
        self.size = int(np.prod(self.shape))

    def cstruct(self) -> _GridC:
        g = _GridC()
        g.ndim = self.ndim
        g.M = self.M
        if self.ndim == 3:
            g.nx, g.ny, g.nz = self.shape
            g.hx, g.hy, g.hz = self.spacing
        else:
            g.nx, g.nz = self.shape
            g.ny = 1
            g.hx, g.hz = self.spacing
            g.hy = 1.0
        for j in range(self.M + 1):
            g.alpha[j] = self.alpha[j]
        return g


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.c_void_p)


def _real(x, cplx: bool) -> np.ndarray:
    dt = np.complex128 if cplx else np.float64
    return np.ascontiguousarray(x, dtype=dt)


def _fn(name: str, cplx: bool):
    f = getattr(_lib(), name + ("_z" if cplx else "_d"))
    f.restype = ctypes.c_int if name in ("oracle_forward", "oracle_adjoint", "oracle_gradient") else None
    return f


def laplacian(grid: Grid, u: np.ndarray) -> np.ndarray:
    """L u with zero values beyond the grid (eq. fdSpace summed over axes)."""
    cplx = np.iscomplexobj(u)
    u = _real(u, cplx)
    out = np.empty_like(u)
    g = grid.cstruct()
    _fn("oracle_laplacian", cplx)(ctypes.byref(g), _ptr(u), _ptr(out))
    return out


def step(grid: Grid, m: np.ndarray, eta: np.ndarray, dt: float,
         u_prev: np.ndarray, u: np.ndarray) -> np.ndarray:
    """One source-free update u^{n+1} = (2 m u^n - b u^{n-1} + dt^2 L u^n)/a
    (eqs. fdWE-abc, fdTime, eulerfwd)."""
    cplx = np.iscomplexobj(m) or np.iscomplexobj(u) or np.iscomplexobj(u_prev)
    m = _real(m, cplx)
    u = _real(u, cplx)
    u_prev = _real(u_prev, cplx)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    out = np.empty_like(u)
    work = np.empty_like(u)
    g = grid.cstruct()
    _fn("oracle_step", cplx)(ctypes.byref(g), _ptr(m), _ptr(eta), ctypes.c_double(dt),
                             _ptr(u_prev), _ptr(u), _ptr(out), _ptr(work))
    return out


def _pts(p):
    """(node, weight) arrays [npts, K] -> (npts, K, node, weight)."""
    if p is None:
        return 0, 1, None, None
    node, w = p
    node = np.ascontiguousarray(np.atleast_2d(node), dtype=np.int64)
    w = np.ascontiguousarray(np.atleast_2d(w), dtype=np.float64)
    if node.shape != w.shape:
        raise ValueError("node and weight arrays must have the same shape")
    return node.shape[0], node.shape[1], node, w


def forward(grid: Grid, m: np.ndarray, eta: np.ndarray, dt: float, nt: int,
            src, q: Optional[np.ndarray], rec, save: bool = False,
            u_init: Optional[np.ndarray] = None, u_prev_init: Optional[np.ndarray] = None):
    """Forward modelling d = F q (Section "Acoustic forward modelling
    operator"): nt samples, u^0 = u^{-1} = 0 unless initial fields are given,
    q^n injected into u^{n+1} with weight dt^2/a, d^n = P_r u^n.

    src, rec: (node, weight) pairs from sparse_points (or None).
    q: [nt, nsrc]. Returns d [nt, nrec] (and u [nt, *shape] if save)."""
    cplx = np.iscomplexobj(m) or (q is not None and np.iscomplexobj(q))
    m = _real(m, cplx)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    ns, ks, sn, sw = _pts(src)
    nr, kr, rn, rw = _pts(rec)
    qq = _real(q, cplx) if q is not None else None
    if qq is not None and qq.shape != (nt, ns):
        raise ValueError("q must be [nt, nsrc]")
    d = np.zeros((nt, nr), dtype=m.dtype)
    us = np.zeros((nt,) + grid.shape, dtype=m.dtype) if save else None
    ui = _real(u_init, cplx) if u_init is not None else None
    upi = _real(u_prev_init, cplx) if u_prev_init is not None else None
    g = grid.cstruct()
    rc = _fn("oracle_forward", cplx)(
        ctypes.byref(g), _ptr(m), _ptr(eta), ctypes.c_double(dt), ctypes.c_long(nt),
        ctypes.c_long(ns), ctypes.c_int(ks), _ptr(sn), _ptr(sw), _ptr(qq),
        ctypes.c_long(nr), ctypes.c_int(kr), _ptr(rn), _ptr(rw), _ptr(d), _ptr(us), _ptr(ui), _ptr(upi))
    if rc != 0:
        raise MemoryError("oracle_forward")
    return (d, us) if save else d


def adjoint(grid: Grid, m: np.ndarray, eta: np.ndarray, dt: float, nt: int,
            rec, y: np.ndarray, src, save: bool = False):
    """Adjoint x = F^T y (eq. Adj; backward substitution on A(m)^T): y^{n+1}
    enters v^n with weight dt^2/a, x^n = P_s v^n, v^{nt} = v^{nt-1} = 0.
    y: [nt, nrec]. Returns x [nt, nsrc] (and v [nt, *shape] if save)."""
    cplx = np.iscomplexobj(m) or np.iscomplexobj(y)
    m = _real(m, cplx)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    nr, kr, rn, rw = _pts(rec)
    ns, ks, sn, sw = _pts(src)
    yy = _real(y, cplx)
    if yy.shape != (nt, nr):
        raise ValueError("y must be [nt, nrec]")
    x = np.zeros((nt, ns), dtype=m.dtype)
    vs = np.zeros((nt,) + grid.shape, dtype=m.dtype) if save else None
    g = grid.cstruct()
    rc = _fn("oracle_adjoint", cplx)(
        ctypes.byref(g), _ptr(m), _ptr(eta), ctypes.c_double(dt), ctypes.c_long(nt),
        ctypes.c_long(nr), ctypes.c_int(kr), _ptr(rn), _ptr(rw), _ptr(yy),
        ctypes.c_long(ns), ctypes.c_int(ks), _ptr(sn), _ptr(sw), _ptr(x), _ptr(vs))
    if rc != 0:
        raise MemoryError("oracle_adjoint")
    return (x, vs) if save else x


def misfit(d: np.ndarray, d_obs: np.ndarray) -> float:
    """Phi = 1/2 sum (d - d_obs)^2 over samples and receivers (eq. AS)."""
    r = np.asarray(d) - np.asarray(d_obs)
    return 0.5 * float(np.sum(r * r)) if not np.iscomplexobj(r) else 0.5 * np.sum(r * r)


def gradient(grid: Grid, m: np.ndarray, eta: np.ndarray, dt: float, nt: int,
             src, q: np.ndarray, rec, residual: np.ndarray, seg: Optional[int] = None,
             both: bool = False):
    """Adjoint-state gradient of Phi with respect to m on the computational
    grid (eqs. Grad, Adj), for the residual y = P_r u - d_obs:
        g = - sum_{j=1}^{nt-1} u^j (v^{j-1} - 2 v^j + v^{j+1}) / dt^2,
    v = the adjoint wavefield driven by y. With both=True also returns the
    summation-by-parts form - sum_n v^n (u^{n+1} - 2u^n + u^{n-1}) / dt^2.
    The forward wavefield is kept by two-level checkpointing every `seg` steps
    (default ceil(sqrt(nt)))."""
    cplx = np.iscomplexobj(m) or np.iscomplexobj(residual) or np.iscomplexobj(q)
    m = _real(m, cplx)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    ns, ks, sn, sw = _pts(src)
    nr, kr, rn, rw = _pts(rec)
    qq = _real(q, cplx)
    yy = _real(residual, cplx)
    if seg is None:
        seg = max(1, int(math.ceil(math.sqrt(nt))))
    g1 = np.zeros(grid.shape, dtype=m.dtype)
    g2 = np.zeros(grid.shape, dtype=m.dtype)
    g = grid.cstruct()
    rc = _fn("oracle_gradient", cplx)(
        ctypes.byref(g), _ptr(m), _ptr(eta), ctypes.c_double(dt), ctypes.c_long(nt),
        ctypes.c_long(ns), ctypes.c_int(ks), _ptr(sn), _ptr(sw), _ptr(qq),
        ctypes.c_long(nr), ctypes.c_int(kr), _ptr(rn), _ptr(rw), _ptr(yy), ctypes.c_long(seg),
        _ptr(g1), _ptr(g2))
    if rc != 0:
        raise MemoryError("oracle_gradient")
    return (g1, g2) if both else g1


def born(grid: Grid, m: np.ndarray, eta: np.ndarray, dt: float, nt: int,
         src, q: np.ndarray, rec, dm: np.ndarray) -> np.ndarray:
    """Linearised (Born) modelling dd = J dm, J the Jacobian of the discrete
    forward map m -> P_r u(m) whose transpose the adjoint-state gradient
    applies (eq. Grad). Differentiating the update
        a u^{n+1} = 2 m u^n - b u^{n-1} + dt^2 L u^n + dt^2 P_s^T q^n,
        a = m + eta dt/2, b = m - eta dt/2 (eta independent of m),
    in direction dm gives the scattered field
        a du^{n+1} = 2 m du^n - b du^{n-1} + dt^2 L du^n - dm (u^{n+1} - 2 u^n + u^{n-1}),
    du^0 = du^{-1} = 0, dd^n = P_r du^n, u the background field of forward().
    Returns dd [nt, nrec]."""
    m = np.asarray(m, dtype=np.float64)
    dm = np.asarray(dm, dtype=np.float64)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    _, us = forward(grid, m, eta, dt, nt, src, q, rec, save=True)
    a = m + 0.5 * eta * dt
    node, w = rec
    node = np.atleast_2d(np.asarray(node, dtype=np.int64))
    w = np.atleast_2d(np.asarray(w, dtype=np.float64))
    dd = np.zeros((nt, node.shape[0]))
    du_prev = np.zeros(grid.shape)
    du = np.zeros(grid.shape)
    zero = np.zeros(grid.shape)
    for n in range(nt - 1):
        u_prev = us[n - 1] if n >= 1 else zero
        du_next = step(grid, m, eta, dt, du_prev, du) - (dm / a) * (us[n + 1] - 2.0 * us[n] + u_prev)
        dd[n + 1] = np.sum(w * du_next.ravel()[node], axis=1)
        du_prev, du = du, du_next
    return dd


def fwi_objective(grid: Grid, m: np.ndarray, eta: np.ndarray, dt: float, nt: int,
                  shots, d_obs):
    """Multi-shot FWI objective and gradient (eq. AS summed over the source
    experiments; Section "FWI using Devito operators": a loop over the shots
    whose gradients are added). For shot s = (src, q, rec):
        d_s = P_r A(m)^{-1} P_s^T q_s,  r_s = d_s - d_obs[s],
        Phi = sum_s 1/2 ||r_s||^2,     g = sum_s J_s^T r_s  (eq. Grad per shot).
    Returns (Phi, g, [d_s])."""
    phi = 0.0
    g = None
    preds = []
    for (src, q, rec), dob in zip(shots, d_obs):
        d = forward(grid, m, eta, dt, nt, src, q, rec)
        r = d - dob
        phi = phi + misfit(d, dob)
        gs = gradient(grid, m, eta, dt, nt, src, q, rec, r)
        g = gs if g is None else g + gs
        preds.append(d)
    return phi, g, preds


def fwi_update(m: np.ndarray, g: np.ndarray, alpha: float,
               m_lo: Optional[float] = None, m_hi: Optional[float] = None) -> np.ndarray:
    """One fixed-step gradient update of the squared slowness, m - alpha g
    (the steepest-descent step of Section "FWI using Devito operators"),
    projected onto the box [m_lo, m_hi] (velocity bounds 1/vmax^2 <= m <=
    1/vmin^2, the bound constraints of the inversion example)."""
    out = np.asarray(m, dtype=np.float64) - alpha * np.asarray(g, dtype=np.float64)
    if m_lo is not None:
        out = np.maximum(out, m_lo)
    if m_hi is not None:
        out = np.minimum(out, m_hi)
    return out


def energy(grid: Grid, m: np.ndarray, dt: float, u_n: np.ndarray, u_np1: np.ndarray) -> float:
    """Discrete energy of the undamped leapfrog between t_n and t_{n+1}:
    E = 1/2 <m (u^{n+1} - u^n), u^{n+1} - u^n> / dt^2 - 1/2 <u^{n+1}, L u^n>.
    Conserved exactly (up to rounding) by the update of eq. eulerfwd when
    eta = 0 and there is no source, because L is symmetric."""
    du = u_np1 - u_n
    return 0.5 * float(np.sum(m * du * du)) / (dt * dt) - 0.5 * float(np.sum(u_np1 * laplacian(grid, u_n)))
