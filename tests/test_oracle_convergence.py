"""Accuracy pins for the oracle's forward operator (Section "Numerical
accuracy"): a 2D constant-velocity medium with an on-grid point source
compared with the analytic Green's-function solution (eq. analytical, read as
the textbook 2D solution; the printed prefactor is garbled), plus the orders of
convergence in time (eq. fdTime, second order) and in space (eq. fdSpace,
order k).

The 2D solution of m u_tt - Lap u = f(t) delta(x), m = 1/c^2, is
    u(r, t) = 1/(2 pi) * int_{-inf}^{t - r/c} f(tau) / sqrt((t - tau)^2 - r^2/c^2) dtau
            = 1/(2 pi) * int_0^{acosh(c t / r)} f(t - (r/c) cosh(theta)) dtheta
(substituting t - tau = (r/c) cosh(theta) removes the endpoint singularity).
A discrete point source approximates f delta(x) when its samples are scaled by
1/h^2.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

from synthetic import ricker

HERE = os.path.dirname(os.path.abspath(__file__))
PAPER = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))

C = 1.5          # km/s
F0 = 15.0        # Hz
T0 = 100.0       # ms, wavelet delay
L = 400.0        # m, square domain, source at the centre
R_OFF = 60.0     # m, receiver offset along x
T_END = 200.0    # ms: the edge reflection reaches the receiver only after ~227 ms


def _analytic(times):
    f0 = F0 * 1e-3

    def f(tau):
        a = (math.pi * f0 * (tau - T0)) ** 2
        return (1 - 2 * a) * math.exp(-a) if tau >= 0 else 0.0

    out = np.zeros_like(times)
    for i, t in enumerate(times):
        if C * t <= R_OFF:
            continue
        th = math.acosh(C * t / R_OFF)
        out[i] = quad(lambda s: f(t - (R_OFF / C) * math.cosh(s)), 0.0, th, limit=400)[0] / (2 * math.pi)
    return out


def _numerical(o, h, k, dt):
    n = int(round(L / h)) + 1
    g = o.Grid((n, n), (h, h), k)
    m = np.full((n, n), 1.0 / C ** 2)
    eta = np.zeros((n, n))
    nt = int(round(T_END / dt)) + 1
    ctr = (n - 1) // 2
    src = (np.array([[ctr * n + ctr]], dtype=np.int64), np.ones((1, 1)))
    ir = ctr + int(round(R_OFF / h))
    rec = (np.array([[ir * n + ctr]], dtype=np.int64), np.ones((1, 1)))
    q = ricker(nt, dt, F0, t0=T0)[:, None] / (h * h)
    d = o.forward(g, m, eta, dt, nt, src, q, rec)
    return d[:, 0], np.arange(nt) * dt


def test_matches_analytic_solution(oracle_mod):
    d, t = _numerical(oracle_mod, 2.5, 8, 0.05)
    ref = _analytic(t)
    err = np.linalg.norm(d - ref) / np.linalg.norm(ref)
    assert err < 2e-3, err


def test_time_convergence_second_order(oracle_mod):
    """Against the analytic solution at fixed fine grid (k = 8, h = 2.5 m):
    the error falls as dt^2 (the paper measures slope 1.94)."""
    o = oracle_mod
    dts = [0.4, 0.2, 0.1]
    errs = []
    for dt in dts:
        d, t = _numerical(o, 2.5, 8, dt)
        stride = int(round(0.4 / dt))
        ref = _analytic(t[::stride])
        errs.append(np.linalg.norm(d[::stride] - ref) / np.linalg.norm(ref))
    slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    assert abs(slope - 2.0) < 0.15, (slope, errs, PAPER["time_convergence_slope"])


@pytest.mark.parametrize("k", [2, 4, 6, 8])
def test_space_convergence_order_k(oracle_mod, k):
    """Self-convergence at a fixed small dt: ||u_h - u_{h/2}|| / ||u_{h/2} - u_{h/4}||
    -> 2^k (the time error is common to all grids and cancels)."""
    o = oracle_mod
    dt = 0.1
    hs = [10.0, 5.0, 2.5] if k <= 4 else [5.0, 2.5, 1.25]
    traces = [_numerical(o, h, k, dt)[0] for h in hs]
    e1 = np.linalg.norm(traces[0] - traces[1])
    e2 = np.linalg.norm(traces[1] - traces[2])
    rate = math.log2(e1 / e2)
    assert abs(rate - k) < 0.3, (k, rate)
