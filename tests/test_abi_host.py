"""Host-only checks of the C ABI (no GPU needed): the library loads, exports
every function include/wavefd.h declares, and its pure host functions agree
with the oracle (stability limit) and with a brute-force dynamic programme
(revolve forward-step counts)."""
import ctypes
import functools
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "wavefd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wf_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_1808_01995_amd import _abi
    names = _declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(_abi.lib, n), n
    assert set(names) == set(_abi.EXPORTS)


def test_version_and_error_string():
    from paper_1808_01995_amd import _abi
    assert _abi.wf_version() >= 10000
    assert isinstance(_abi.wf_last_error(), str)


@pytest.mark.parametrize("ndim,k", [(2, 4), (2, 8), (3, 8), (3, 16), (3, 12)])
def test_critical_dt_matches_oracle(oracle_mod, ndim, k):
    from paper_1808_01995_amd import _abi
    h = (10.0, 7.5, 12.5)[:ndim]
    g = _abi.make_geom((50,) * ndim, h, 10, k, 3.0)
    for v in (1.5, 4.5):
        a = _abi.wf_critical_dt(g, v)
        b = oracle_mod.critical_dt(ndim, h, k, v)
        assert abs(a - b) <= 1e-14 * b


def test_geom_validation():
    from paper_1808_01995_amd import _abi
    g = _abi.make_geom((101, 101), (10.0, 10.0), 20, 4, 1.5)
    assert _abi.wf_geom_shape(g) == ((141, 141), 141 * 141)
    g3 = _abi.make_geom((10, 11, 12), (10.0, 10.0, 10.0), 3, 8, 2.0)
    assert _abi.wf_geom_shape(g3) == ((16, 17, 18), 16 * 17 * 18)
    for bad in [dict(space_order=5), dict(space_order=18), dict(space_order=2), dict(nbl=-1),
                dict(c_ref=0.0)]:
        args = dict(shape=(20, 20), spacing=(10.0, 10.0), nbl=4, space_order=4, c_ref=1.5)
        args.update(bad)
        gb = _abi.make_geom(**args)
        with pytest.raises(_abi.WaveFDError) as e:
            _abi.wf_geom_shape(gb)
        assert e.value.status == _abi.WF_E_ARG
        assert _abi.lib.wf_critical_dt(ctypes.byref(gb), 1.5) < 0
    gb = _abi.make_geom((20, 20), (0.0, 10.0), 4, 4, 1.5)
    with pytest.raises(_abi.WaveFDError):
        _abi.wf_geom_shape(gb)


def _dp_table(L, S):
    """Brute force: T(l, s) = min_m [m + T(l-m, s-1) + T(m, s)], T(1, s) = 0,
    T(l, 1) = l (l - 1) / 2, over every split."""
    T = [[0] * (S + 1) for _ in range(L + 1)]
    for s in range(1, S + 1):
        for l in range(1, L + 1):
            if l == 1:
                T[l][s] = 0
            elif s == 1:
                T[l][s] = l * (l - 1) // 2
            else:
                T[l][s] = min(m + T[l - m][s - 1] + T[m][s] for m in range(1, l))
    return T


def _closed_form(l, s):
    from math import comb
    r = 1
    while comb(s + r, s) < l:
        r += 1
    return r * l - comb(s + r, r - 1)


def test_revolve_counts_are_optimal():
    from paper_1808_01995_amd import _abi
    L, S = 60, 6
    T = _dp_table(L, S)
    for l in range(1, L + 1):
        for s in range(1, S + 1):
            assert T[l][s] == _closed_form(l, s), (l, s)
            assert _abi.wf_revolve_forward_steps(l, s) == T[l][s], (l, s)
    # the configurations of the gradient workload
    assert _abi.wf_revolve_forward_steps(2000, 20) == 5976
    assert _abi.wf_revolve_forward_steps(2000, 50) == 4622
    assert _abi.wf_revolve_forward_steps(2000, 2000) == 1999
    assert _abi.wf_revolve_forward_steps(0, 3) == -1
    assert _abi.wf_revolve_forward_steps(5, 0) == -1


def _run_schedule(acts, l, s):
    """Replay a schedule as a state machine (the state in memory, the states
    held in slots) and return its forward-step count; every action is checked
    against what the one before it left."""
    from paper_1808_01995_amd import _abi
    cur = 0                  # state 0 is in memory and in slot 0 at the start
    slots = {}
    advances = 0
    reversed_steps = []
    live = 0
    for kind, at, arg in acts:
        if kind == _abi.WF_REVOLVE_TAKESHOT:
            assert at == cur and arg not in slots and 0 <= arg < s
            slots[arg] = cur
        elif kind == _abi.WF_REVOLVE_ADVANCE:
            assert at == cur and arg > at
            advances += arg - at
            cur = arg
        elif kind == _abi.WF_REVOLVE_RESTORE:
            assert slots.get(arg) == at
            cur = at
        elif kind == _abi.WF_REVOLVE_REVERSE:
            assert at == cur          # the adjoint of step i needs state i
            reversed_steps.append(at)
        elif kind == _abi.WF_REVOLVE_FREE:
            assert arg in slots
            del slots[arg]
        else:
            raise AssertionError(kind)
        live = max(live, len(slots))
    assert reversed_steps == list(range(l - 1, -1, -1))   # every step once, last first
    assert not slots and live <= s
    return advances, live


def test_revolve_schedule_runs_the_optimal_count():
    """The schedule wf_gradient runs (not the closed form) reverses every
    step once, holds at most s states, and advances exactly the brute-force
    optimum T(l, s) for l <= 60 and s <= 6, and at the gradient workload's
    2000 steps with 20 and 50 states."""
    from paper_1808_01995_amd import _abi
    L, S = 60, 6
    T = _dp_table(L, S)
    for l in range(1, L + 1):
        for s in range(1, S + 1):
            adv, live = _run_schedule(_abi.wf_revolve_schedule(l, s), l, s)
            assert adv == T[l][s], (l, s, adv)
            assert live <= min(s, l)
    for s, t in ((20, 5976), (50, 4622)):
        adv, live = _run_schedule(_abi.wf_revolve_schedule(2000, s), 2000, s)
        assert adv == t and live <= s
    assert _abi.lib.wf_revolve_schedule(0, 3, None, None, None, 0) == _abi.WF_E_ARG
    assert _abi.lib.wf_revolve_schedule(5, 0, None, None, None, 0) == _abi.WF_E_ARG


def test_stream_bandwidth_argument_checks():
    """Argument errors are reported before any device work."""
    import ctypes
    from paper_1808_01995_amd import WaveFDError, _abi
    for n, reps in ((10, 5), (1 << 35, 5), (4096, 0)):
        with pytest.raises(WaveFDError) as e:
            _abi.wf_stream_bandwidth(n, reps)
        assert e.value.status == _abi.WF_E_ARG
    assert _abi.lib.wf_stream_bandwidth(4096, 1, None) == _abi.WF_E_ARG


def test_ghost_check_argument_checks():
    from paper_1808_01995_amd import _abi
    assert _abi.lib.wf_model_ghost_nonzero(None, None) == _abi.WF_E_ARG


def test_validation_switch():
    from paper_1808_01995_amd import _abi
    assert _abi.lib.wf_validate_enable(1) == _abi.WF_OK
    assert _abi.lib.wf_validate_enable(0) == _abi.WF_OK


def test_two_step_mode_switch():
    """The mode of two updates per launch takes 0, 1 or 2; anything else is
    an argument error that leaves the mode unchanged (pure host call)."""
    from paper_1808_01995_amd import _abi
    for bad in (-1, 3, 100):
        assert _abi.lib.wf_two_step_enable(bad) == _abi.WF_E_ARG
    for mode in (0, 2, 1):
        assert _abi.lib.wf_two_step_enable(mode) == _abi.WF_OK
