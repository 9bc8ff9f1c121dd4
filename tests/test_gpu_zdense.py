"""GPU parity of the ABM phases with the z-term inside the plane kernel (tuning z_dense):
the kinetic operator along z applied as the dense matrix T_z to the z-columns of the input,
no z-axis kernel and no z-term scratch.  Checked against the float64 oracle, against the
two-kernel path on the GPU, under graph replay, and in a batch.

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


def gpu_run(lise, w, nsteps, tuning):
    ctx = lise.Context(w.lattice, w.M, w.functional)
    ctx.set_tuning(**tuning)
    ctx.set_qpwf(0, w.qpwfs())
    ctx.step(w.dt, nsteps)
    out = dict(psi=ctx.get_qpwf(0, w.M), dens=ctx.densities(), time=ctx.time())
    ctx.close()
    return out


def cfg2(M, n, p):
    w = wl.config2(M=M, n=n)
    w.functional.precision = p
    return w


# (id, workload factory of a precision, tuning, density tolerance); the path covers
# whole-line plane rows of at most two points per lane: float64 16^3 and 32^3, float32 32^3
#   32^3 float64: 9 rows of one qpwf = 8 rows on the XCD map + 1 in plain order
#   16^3 float64, C = 4: two pairs; 20 rows (16 mapped + 4), two chunks
#   32^3 float32: 3 rows, two chunks
#   32^3 float64, one qpwf, default tuning (128 qpwfs per row): a single row
CASES = [
    ("32c_fp64", lambda p: cfg2(9, 32, p), {"jgroup": 1}, 1e-11),
    ("16c_fp64_c4", lambda p: wl.config4(M=40, n=16, precision=p), {"jgroup": 2, "chunk_qpwf": 24,
                                                                     "single_pass": -1}, 1e-11),
    ("32c_fp32", lambda p: cfg2(6, 32, p), {"jgroup": 2, "chunk_qpwf": 4}, 1e-5),
    ("32c_fp64_m1", lambda p: cfg2(1, 32, p), {}, 1e-11),     # one qpwf: one row, in plain order
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_z_dense_matches_oracle_and_two_kernel_path(lise, case):
    """3 start-up + 8 ABM steps with z_dense = 1: float64 psi and densities within 1e-11 of
    the oracle (float32 densities within 1e-5 of the float64 oracle), and within rounding
    of the two-kernel path (z_dense = -1) on the GPU."""
    name, make, tuning, tol = case
    w = make(wl.FP32 if tol > 1e-9 else wl.FP64)
    say(f"z_dense {name}: {w.name} M={w.M} 8 steps, tuning {tuning}")
    g = gpu_run(lise, w, 8, dict(tuning, z_dense=1))
    r = gpu_run(lise, w, 8, dict(tuning, z_dense=-1))
    w64 = make(wl.FP64)
    say(f"  oracle {w64.name}: 8 ABM steps")
    ev = oracle.Evolver(w64.lattice, w64.functional, w64.qpwfs())
    ev.step(w64.dt, 8)
    n0, k0 = oracle.densities(ev.y, w64.functional)
    e = (rel_l2(g["dens"][0], n0), rel_l2(g["dens"][1], k0))
    d = rel_l2(g["psi"], r["psi"])
    say(f"  density rel L2 n {e[0]:.3e} kappa {e[1]:.3e}; psi vs two-kernel path {d:.3e}")
    assert g["time"] == r["time"]
    assert max(e) < tol
    if w.functional.precision == wl.FP64:
        assert rel_l2(g["psi"], ev.y) < 1e-11
        assert d < 1e-12
    else:
        assert d < 1e-5


def test_z_dense_graph_replay_and_batch_bitwise(lise):
    """z_dense under graph replay (4-step periods, 10 steps) equals eager stepping bit for
    bit; in a batch, the z_dense context is stepped alone and equals itself run alone."""
    w = wl.config2(M=7, n=32)
    say(f"z_dense graph: {w.name} 10 steps")
    eager = gpu_run(lise, w, 10, {"z_dense": 1, "jgroup": 2})
    graph = gpu_run(lise, w, 10, {"z_dense": 1, "jgroup": 2, "graph": 1})
    assert np.array_equal(eager["psi"], graph["psi"])
    assert np.array_equal(eager["dens"][0], graph["dens"][0])
    other = wl.config2(M=6, n=16, seed=4)
    say("z_dense batch: the 32^3 context (z_dense) with a 16^3 context, 10 steps")
    ctxs = []
    for ww, t in ((w, {"z_dense": 1, "jgroup": 2}), (other, {})):
        c = lise.Context(ww.lattice, ww.M, ww.functional)
        c.set_tuning(**t)
        c.set_qpwf(0, ww.qpwfs())
        ctxs.append(c)
    b = lise.Batch(ctxs)
    b.step(w.dt, 10)
    assert b.info() == (1, 1)
    got = ctxs[0].get_qpwf(0, w.M)
    b.close()
    for c in ctxs:
        c.close()
    assert np.array_equal(got, eager["psi"])


def test_z_dense_rejects_bad_values(lise):
    w = wl.config1(M=2)
    say("z_dense argument check")
    ctx = lise.Context(w.lattice, w.M, w.functional)
    with pytest.raises(lise.LiseError, match="ARG"):
        ctx.set_tuning(z_dense=2)
    ctx.close()
