"""The local parity checks used by every GPU-vs-oracle test catch errors that
a whole-array norm lets through: mistakes planted in oracle results on the
CPU (the weakest trace held to its own size off by 3e-4, one sample off
by 2e-4 of the peak, a gradient off by 0.5 % away from the sources and
receivers) pass the global rel. L2 bar and fail the local ones.
"""
import numpy as np
import pytest

from _harness import check_field, check_record, make_problem, noise, rel_l2


@pytest.fixture(scope="module")
def problem():
    return make_problem((40, 34), 8, 8, 140, seed=5, nrec=60)


def test_record_checks_catch_a_weak_trace(problem):
    P = problem
    d_ref = P.oracle_forward()
    check_record(d_ref, d_ref)
    nr = np.sqrt(np.sum(d_ref ** 2, axis=0))
    rms = np.sqrt(np.mean(nr ** 2))
    keep = np.flatnonzero(nr >= 0.1 * rms)
    weak = keep[np.argmin(nr[keep])]
    bad = d_ref.copy()
    bad[:, weak] *= 1.0 + 3e-4
    assert rel_l2(bad, d_ref) <= 1e-4          # the whole-record norm does not see it
    with pytest.raises(AssertionError):
        check_record(bad, d_ref)


def test_record_checks_catch_one_wrong_sample(problem):
    P = problem
    d_ref = P.oracle_forward()
    bad = d_ref.copy()
    i = np.unravel_index(np.argmax(np.abs(d_ref)), d_ref.shape)
    bad[i] += 2e-4 * np.abs(d_ref).max()
    assert rel_l2(bad, d_ref) <= 1e-4
    with pytest.raises(AssertionError):
        check_record(bad, d_ref)


def test_gradient_checks_catch_an_error_away_from_the_points(problem):
    P = problem
    r = noise(P.nt, P.rec_xyz.shape[0], P.dt, 15.0, 2)
    g = P.oracle_gradient(r)
    away = P.away()
    check_field(g, g, mask=away)
    frac = np.sum(g[away] ** 2) / np.sum(g ** 2)
    bad = g.copy()
    bad[away] *= 1.0 + 5e-3
    print("energy away from the points: %.2e of the gradient's" % frac)
    assert rel_l2(bad, g) <= 1e-3              # the whole-array norm does not see it
    with pytest.raises(AssertionError):
        check_field(bad, g, mask=away)
