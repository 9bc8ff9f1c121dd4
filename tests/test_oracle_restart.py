"""Pins of the oracle's checkpoint/restart (Sec. Checkpoint and restart)."""
import numpy as np

import oracle
import workloads as wl


def small_bump_workload():
    """Config-2 recipe (ramped Gaussian well: the Hamiltonian depends on t) on 8^3."""
    w = wl.config2(M=16, n=8, steps=10)
    w.functional.ext_t_on = 0.05
    return w


def test_restart_with_history_is_exact():
    w = small_bump_workload()
    psi = w.qpwfs()
    a = oracle.Evolver(w.lattice, w.functional, psi)
    a.step(w.dt, 8)
    b = oracle.Evolver(w.lattice, w.functional, psi)
    b.step(w.dt, 3)
    r = oracle.Evolver.restore(w.lattice, w.functional, b.checkpoint())
    r.step(w.dt, 5)
    assert r.t == a.t and r.step_count == a.step_count
    assert np.array_equal(r.y, a.y)


def test_checkpoint_is_a_copy():
    w = small_bump_workload()
    ev = oracle.Evolver(w.lattice, w.functional, w.qpwfs())
    ev.step(w.dt, 2)
    ck = ev.checkpoint()
    y0 = ck["y"].copy()
    ev.step(w.dt, 2)
    assert np.array_equal(ck["y"], y0)


def restart_difference(w, psi, dt, T, lose_time=False):
    """Relative difference at time T between the continuous run and one restarted
    from the qpwfs alone a third of the way through."""
    n_total = round(T / dt) - 3           # ABM steps after the first start-up
    k = n_total // 3                      # checkpoint after k ABM steps
    a = oracle.Evolver(w.lattice, w.functional, psi)
    a.step(dt, n_total)
    b = oracle.Evolver(w.lattice, w.functional, psi)
    b.step(dt, k)
    ck = b.checkpoint(with_history=False)
    if lose_time:
        ck["t"] = 0.0
    r = oracle.Evolver.restore(w.lattice, w.functional, ck)
    assert r.hist is None
    r.step(dt, n_total - k - 3)           # start-up (3 steps) + the rest
    assert abs(a.t - T) < 1e-12
    return float(np.linalg.norm(r.y - a.y) / np.linalg.norm(a.y))


def test_restart_from_qpwfs_only_differs_at_third_order():
    """The paper's restart (latest qpwfs only, series start-up again) departs from the
    continuous run by the start-up's error: its self-consistent series step is second
    order (local error dt^3), so at a fixed final time the difference falls 8x per
    halving of dt (config-1 recipe: no time-dependent potential)."""
    w = wl.config1(M=32)
    psi = w.qpwfs()
    diffs = [restart_difference(w, psi, dt, 0.24) for dt in (0.02, 0.01, 0.005)]
    assert diffs[0] < 1e-6
    for d1, d2 in zip(diffs, diffs[1:]):
        assert 6.0 < d1 / d2 < 10.0, diffs


def test_restart_keeps_the_time():
    """With the ramped well, a restart that restores t stays within the start-up's
    error of the continuous run, one that lost t does not."""
    w = small_bump_workload()
    psi = w.qpwfs()
    good = restart_difference(w, psi, 0.01, 0.24)
    bad = restart_difference(w, psi, 0.01, 0.24, lose_time=True)
    assert good < 1e-6 and bad > 1e-5, (good, bad)
