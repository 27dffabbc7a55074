"""Write the stored expected values of the full-size parity checks.

Calls only the FP64 oracle and the seeded input generators. For the 3D
order-8 workload (256^3 physical, h = 10 m, 40-node layer, 1000 steps, 15 Hz
Ricker at (1275, 1275, 20) m, 128 x 128 receivers at 20 m depth) the oracle
record is kept at every 8th receiver in x and y (256 traces x 1001 samples,
stored as float32).

The model and wavelet are rounded to float32 first and widened back, exactly
as they reach the GPU, so the stored record is the FP64 solution of the same
discrete problem.

Usage: python tests/golden/make_golden.py [c2]
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


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2"]
    if "c2" in which:
        c2_record(os.path.join(HERE, "c2_so8_record_sampled.npz"))
