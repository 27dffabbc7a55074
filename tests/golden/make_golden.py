"""Write the stored expected values of the full-size parity checks.

Calls only the FP64 oracle and the seeded input generators. For the 3D
order-8 workload (256^3 physical, h = 10 m, 40-node layer, 1000 steps, 15 Hz
Ricker at (1275, 1275, 20) m, 128 x 128 receivers at 20 m depth) the oracle
record is kept at every 8th receiver in x and y (256 traces x 1001 samples,
stored as float32).

The model and wavelet are rounded to float32 first and widened back, exactly
as they reach the GPU, so the stored record is the FP64 solution of the same
discrete problem.

For the 512^3 sweep grid (592^3 computational, two layers 1.5 / 2.5 km/s)
at every space order 4 / 8 / 12 / 16, 60 updates of a 40 Hz Ricker delayed
by only 10 ms (the sweep's 15 Hz wavelet would still be silent after 60
updates) at the sweep's source: the oracle wavefield on a window of nodes
around the source (receivers placed on nodes: x indices 279..312, y 295..296,
z 40..74 in steps of 2), every 4th sample.

For the gradient workload (200^3 physical, 280^3 computational, order 8,
2000 steps, 10 Hz Ricker at (995, 995, 20) m): the oracle records of the true
model (the observed data) and of the 2 km/s initial model at every 10th
receiver in x and y (100 traces), every 4th sample.

For the same gradient workload, the oracle's J^T r of the initial model for
a seeded band-limited residual r at all 100 x 100 receivers (two-level
checkpointing), on the plane y = 140 through the source and the anomaly,
every 2nd node in x and z. (The workload's own residual, the initial minus
the true model's record, is 7e-5 of the records, so the records' float32
rounding leaves it a few percent uncertain: a shared residual compares the
gradient operators themselves.)

Usage: python tests/golden/make_golden.py [c2] [c3] [c4] [c4g]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synthetic import config, ricker  # noqa: E402


def c2_record(path):
    c = config("c2_3d_so8")
    v = c.velocity()
    vmax = float(v.max())
    m32 = (1.0 / oracle.pad_edge(v, c.nbl) ** 2).astype(np.float32)
    dt = c.dt_factor * oracle.critical_dt(3, c.spacing, c.space_order, vmax)
    q32 = ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32)
    sel = np.array([ix * 128 + iy for ix in range(0, 128, 8) for iy in range(0, 128, 8)])
    rec = c.rec[sel]
    g = oracle.Grid(m32.shape, c.spacing, c.space_order)
    eta = oracle.damping_eta(c.shape, c.nbl, c.spacing, vmax)
    src_p = oracle.sparse_points(c.src, c.spacing, c.nbl, m32.shape)
    rec_p = oracle.sparse_points(rec, c.spacing, c.nbl, m32.shape)
    t = time.time()
    d = oracle.forward(g, m32.astype(np.float64), eta, dt, c.nt, src_p, q32.astype(np.float64), rec_p)
    print("oracle C2 forward: %.1f s" % (time.time() - t))
    np.savez_compressed(path, record=d.astype(np.float32), receiver_index=sel, dt=dt,
                        nt=c.nt, vmax=vmax)


C3_ORDERS = (4, 8, 12, 16)
C3_STEPS = 60


def c3_window_points(c):
    """Window nodes around the sweep's source as physical coordinates (m)."""
    h = c.spacing
    pts = [((ix - c.nbl) * h[0], (iy - c.nbl) * h[1], (iz - c.nbl) * h[2])
           for ix in range(279, 313) for iy in (295, 296) for iz in range(40, 75, 2)]
    return np.array(pts, dtype=np.float64)


def c3_windows(path):
    c = config("c3_sweep")
    v = c.velocity()
    vmax = float(v.max())
    m32 = (1.0 / oracle.pad_edge(v, c.nbl) ** 2).astype(np.float32)
    m64 = m32.astype(np.float64)
    del v
    rec = c3_window_points(c)
    eta = oracle.damping_eta(c.shape, c.nbl, c.spacing, vmax)
    out = {"rec_xyz": rec, "vmax": vmax, "orders": np.array(C3_ORDERS), "nt": C3_STEPS + 1}
    for k in C3_ORDERS:
        dt = 0.5 * oracle.critical_dt(3, c.spacing, k, vmax)
        nt = C3_STEPS + 1
        q32 = ricker(nt, dt, 40.0, t0=10.0)[:, None].astype(np.float32)
        g = oracle.Grid(m32.shape, c.spacing, k)
        src_p = oracle.sparse_points(c.src, c.spacing, c.nbl, m32.shape)
        rec_p = oracle.sparse_points(rec, c.spacing, c.nbl, m32.shape)
        t = time.time()
        d = oracle.forward(g, m64, eta, dt, nt, src_p, q32.astype(np.float64), rec_p)
        print("oracle C3 order %d, %d updates: %.1f s, max |u| %.3e" % (k, nt - 1, time.time() - t,
                                                                      np.abs(d).max()))
        out["dt_so%d" % k] = dt
        out["record_so%d" % k] = d[::4].astype(np.float32)
    np.savez_compressed(path, **out)


def c4_records(path):
    c = config("c4_gradient")
    v_true = c.velocity()
    v0 = np.full(c.shape, 2.0)
    dt = 0.5 * oracle.critical_dt(3, c.spacing, 8, 2.5)
    q32 = ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32)
    sel = np.array([ix * 100 + iy for ix in range(0, 100, 10) for iy in range(0, 100, 10)])
    rec = c.rec[sel]
    out = {"receiver_index": sel, "dt": dt, "nt": c.nt}
    for name, v in (("true", v_true), ("initial", v0)):
        m32 = (1.0 / oracle.pad_edge(v, c.nbl) ** 2).astype(np.float32)
        g = oracle.Grid(m32.shape, c.spacing, 8)
        eta = oracle.damping_eta(c.shape, c.nbl, c.spacing, 2.5)
        src_p = oracle.sparse_points(c.src, c.spacing, c.nbl, m32.shape)
        rec_p = oracle.sparse_points(rec, c.spacing, c.nbl, m32.shape)
        t = time.time()
        d = oracle.forward(g, m32.astype(np.float64), eta, dt, c.nt, src_p, q32.astype(np.float64), rec_p)
        print("oracle C4 %s model, %d updates: %.1f s" % (name, c.nt - 1, time.time() - t))
        out["record_" + name] = d[::4].astype(np.float32)
    np.savez_compressed(path, **out)


C4G_NOISE = {"f0_hz": 10.0, "seed": 44}


def c4_gradient_slice(path):
    """J^T r of the initial model for a seeded band-limited residual r at all
    100 x 100 receivers (the same float32 values the GPU gets), forward
    history by the oracle's two-level checkpointing."""
    from synthetic import band_limited_noise
    c = config("c4_gradient")
    dt = 0.5 * oracle.critical_dt(3, c.spacing, 8, 2.5)
    q64 = ricker(c.nt, dt, c.f0_hz)[:, None].astype(np.float32).astype(np.float64)
    m0 = (1.0 / oracle.pad_edge(np.full(c.shape, 2.0), c.nbl) ** 2).astype(np.float32).astype(np.float64)
    g = oracle.Grid(m0.shape, c.spacing, 8)
    eta = oracle.damping_eta(c.shape, c.nbl, c.spacing, 2.5)
    src_p = oracle.sparse_points(c.src, c.spacing, c.nbl, g.shape)
    rec_p = oracle.sparse_points(c.rec, c.spacing, c.nbl, g.shape)
    r = band_limited_noise(c.nt, c.rec.shape[0], dt, C4G_NOISE["f0_hz"], C4G_NOISE["seed"])
    r = r.astype(np.float32).astype(np.float64)
    t = time.time()
    grad = oracle.gradient(g, m0, eta, dt, c.nt, src_p, q64, rec_p, r)
    print("oracle C4 gradient: %.1f s" % (time.time() - t), flush=True)
    np.savez_compressed(path, gradient=grad[::2, 140, ::2].astype(np.float32), y_index=140, step=2,
                        noise_f0_hz=C4G_NOISE["f0_hz"], noise_seed=C4G_NOISE["seed"], dt=dt, nt=c.nt)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2"]
    if "c2" in which:
        c2_record(os.path.join(HERE, "c2_so8_record_sampled.npz"))
    if "c3" in which:
        c3_windows(os.path.join(HERE, "c3_window_records.npz"))
    if "c4" in which:
        c4_records(os.path.join(HERE, "c4_records_sampled.npz"))
    if "c4g" in which:
        c4_gradient_slice(os.path.join(HERE, "c4_gradient_slice.npz"))
