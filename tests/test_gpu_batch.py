"""GPU parity of the batched form: systems grouped by lattice side advance with one
z-axis and one plane-kernel launch per ABM phase and group (device descriptor
tables), one fields launch for all systems, and four-step periods replayed from
one captured graph.  Every batched system must equal the same system stepped
alone bit for bit, and a grouped system must match the oracle.

Every case prints its name and shape before it touches the GPU.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lise():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    import paper_2009_00745_amd as lise_mod
    lise_mod.load_library()
    return lise_mod


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def mixed_systems():
    """Groups (FP64, 16), (FP32, 20), (FP64, 8) with uneven qpwf counts, functionals and
    C = 2 and 4 inside one group; plus one system with phase removal (stepped alone)."""
    a = wl.config2(M=24, n=16)
    b = wl.config2(M=10, n=16, seed=3)
    b.functional.g = 1.7
    b.functional.mu_up = b.functional.mu_dn = 0.45
    c = wl.config3(M=16, n=20, precision=wl.FP32)
    d = wl.config4(M=12, n=8, precision=wl.FP64)
    e = wl.config1(M=64)
    f = wl.config2(M=8, n=16, seed=5)
    f.functional.remove_phase = 1
    return [a, b, c, d, e, f]


def run_alone(lise, w, dt, calls):
    c = lise.Context(w.lattice, w.M, w.functional)
    c.set_qpwf(0, w.qpwfs())
    for n in calls:
        c.step(dt, n)
    out = (c.get_qpwf(0, w.M), c.densities()[0], c.time())
    c.close()
    return out


def run_batch(lise, ws, dt, calls, graph):
    ctxs = []
    for w in ws:
        c = lise.Context(w.lattice, w.M, w.functional)
        c.set_qpwf(0, w.qpwfs())
        ctxs.append(c)
    b = lise.Batch(ctxs)
    b.set_graph(graph)
    for n in calls:
        b.step(dt, n)
    info = b.info()
    out = [(c.get_qpwf(0, w.M), c.densities()[0], c.time()) for c, w in zip(ctxs, ws)]
    b.close()
    for c in ctxs:
        c.close()
    return out, info


_EAGER = {}


def test_batch_grouped_eager_matches_individual_bitwise(lise):
    """Grouped launches without graphs, 10 + 5 steps (the second call starts mid-period):
    every system equals itself stepped alone, bit for bit, densities and time included;
    the batch forms three groups and steps the phase-removal system alone."""
    ws = mixed_systems()
    dt = 0.002
    say("batch (eager, grouped): 6 systems in 3 groups + 1 alone, 10 + 5 steps")
    got, info = run_batch(lise, ws, dt, (10, 5), graph=0)
    _EAGER["mixed"] = got
    say(f"  groups, alone = {info}")
    assert info == (3, 1)
    for w, g in zip(ws, got):
        say(f"  alone: {w.name} precision {w.functional.precision} C {w.functional.ncomp}")
        ref = run_alone(lise, w, dt, (10, 5))
        assert g[2] == ref[2], w.name
        assert np.array_equal(g[0], ref[0]), w.name
        assert np.array_equal(g[1], ref[1]), w.name


def test_batch_grouped_system_matches_oracle(lise):
    """A system advanced inside a group (16^3 FP64, ramped well) against the oracle after
    3 start-up + 15 ABM steps: psi and densities within 1e-11."""
    if "mixed" not in _EAGER:
        pytest.skip("needs the eager batch run")
    w = mixed_systems()[0]
    say(f"oracle: {w.name} 15 steps")
    ev = oracle.Evolver(w.lattice, w.functional, w.qpwfs())
    ev.step(0.002, 15)
    n0, _ = oracle.densities(ev.y, w.functional)
    psi, n, _ = _EAGER["mixed"][0]
    e = (rel_l2(psi, ev.y), rel_l2(n, n0))
    say(f"  rel L2 psi {e[0]:.3e} n {e[1]:.3e}")
    assert max(e) < 1e-11


def test_batch_graph_replay_matches_eager_bitwise(lise):
    """The captured four-step graph of all groups (one internal stream, kernel nodes
    only), 11 + 9 steps (replays, then an eager tail; an eager head up to the next
    period, then replays): equal to the eager batch of the same calls, bit for bit."""
    ws = mixed_systems()
    dt = 0.002
    say("batch (graph, grouped): 6 systems, 11 + 9 steps")
    got, info = run_batch(lise, ws, dt, (11, 9), graph=1)
    assert info == (3, 1)
    say("batch (eager, grouped): same systems, 11 + 9 steps")
    ref, _ = run_batch(lise, ws, dt, (11, 9), graph=0)
    for w, g, r in zip(ws, got, ref):
        assert g[2] == r[2], w.name
        assert np.array_equal(g[0], r[0]), w.name
        assert np.array_equal(g[1], r[1]), w.name


def test_batch_with_options_matches_individual(lise):
    """A batch mixing phase removal (stepped alone), the regularised coupling and plain
    systems (grouped; graphs on) equals stepping each alone, bit for bit."""
    ws = [wl.config2(M=16, n=16), wl.config3(M=12, n=20, precision=wl.FP32), wl.config1(M=32)]
    ws[0].functional.remove_phase = 1
    ws[1].functional.regularize = 1
    dt = 0.002
    say("batch with options: 3 systems, 9 steps")
    got, info = run_batch(lise, ws, dt, (9,), graph=1)
    assert info == (2, 1)
    for w, g in zip(ws, got):
        ref = run_alone(lise, w, dt, (9,))
        assert np.array_equal(g[0], ref[0]), w.name


def test_batch_config5_sample_fp32(lise):
    """Eight systems of the 64-system recipe (16^3, 20^3, 24^3 FP32, scaled to 1/8 of
    their qpwfs) through the graph path for 3 start-up + 12 steps: each equals itself
    stepped alone bit for bit, and its densities stay within 1e-5 of the float64 run."""
    ws = wl.config5_systems(nsys=8, scale=0.125)
    dt = 0.002
    say("batch cfg5 sample: " + ", ".join(w.name for w in ws))
    got, info = run_batch(lise, ws, dt, (12,), graph=1)
    say(f"  groups, alone = {info}")
    assert info[1] == 0
    for w, g in zip(ws, got):
        ref = run_alone(lise, w, dt, (12,))
        assert np.array_equal(g[0], ref[0]), w.name
        w.functional.precision = wl.FP64
        r64 = run_alone(lise, w, dt, (12,))
        e = rel_l2(g[1], r64[1])
        say(f"  {w.name}: n rel L2 vs float64 {e:.3e}")
        assert e < 1e-5


def test_batch_errors(lise):
    """Unset qpwfs give STATE, a bad dt gives ARG, a duplicated context is refused."""
    w = wl.config1(M=8)
    say("batch errors")
    c1 = lise.Context(w.lattice, w.M, w.functional)
    c2 = lise.Context(w.lattice, w.M, w.functional)
    c1.set_qpwf(0, w.qpwfs())
    b = lise.Batch([c1, c2])
    with pytest.raises(lise.LiseError, match="STATE"):
        b.step(w.dt, 1)
    c2.set_qpwf(0, w.qpwfs())
    with pytest.raises(lise.LiseError, match="ARG"):
        b.step(0.0, 1)
    b.step(w.dt, 2)
    b.close()
    with pytest.raises(lise.LiseError, match="ARG"):
        lise.Batch([c1, c1])
    c1.close()
    c2.close()


def test_batch_single_pass_groups_match_individual(lise):
    """Systems on the single-pass kernel (16^3 FP64, 20^3 FP32, 8^3 C = 4) grouped with the
    batched single-pass launch, graph replays on, 9 steps: each equals itself alone with the
    same tuning, bit for bit."""
    ws = [wl.config2(M=12, n=16), wl.config2(M=7, n=16, seed=2), wl.config3(M=10, n=20, precision=wl.FP32),
          wl.config4(M=6, n=8, precision=wl.FP64)]
    dt = 0.002
    say("batch, single-pass groups: 4 systems, 9 steps")
    ctxs = []
    for w in ws:
        c = lise.Context(w.lattice, w.M, w.functional)
        c.set_tuning(single_pass=1)
        c.set_qpwf(0, w.qpwfs())
        ctxs.append(c)
    b = lise.Batch(ctxs)
    b.step(dt, 9)
    assert b.info() == (3, 0)
    got = [c.get_qpwf(0, w.M) for c, w in zip(ctxs, ws)]
    b.close()
    for c in ctxs:
        c.close()
    for w, g in zip(ws, got):
        c = lise.Context(w.lattice, w.M, w.functional)
        c.set_tuning(single_pass=1)
        c.set_qpwf(0, w.qpwfs())
        c.step(dt, 9)
        ref = c.get_qpwf(0, w.M)
        c.close()
        assert np.array_equal(g, ref), w.name
