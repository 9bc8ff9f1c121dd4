"""GPU parity of the single-pass ABM kernel (the whole component pair of a qpwf in LDS,
kinetic term as a 3D transform, no z-term scratch) against the CPU float64 oracle and
against the two-kernel path, for every lattice side and precision it covers.

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


def run(lise, w, nsteps, single_pass, jgroup=0):
    ctx = lise.Context(w.lattice, w.M, w.functional)
    ctx.set_tuning(single_pass=single_pass, jgroup=jgroup)
    ctx.set_qpwf(0, w.qpwfs())
    ctx.step(w.dt, nsteps)
    out = (ctx.get_qpwf(0, w.M), ctx.densities(), ctx.time())
    ctx.close()
    return out


# (name, workload, steps, tolerance of psi and densities against the float64 oracle)
CASES = [
    ("8c_fp64_cfg1", lambda: wl.config1(M=40), 12, 1e-11),
    ("16c_fp64_well", lambda: wl.config2(M=13, n=16), 12, 1e-11),
    ("16c_fp64_c4", lambda: wl.config4(M=6, n=16, precision=wl.FP64), 10, 1e-11),
    ("8c_fp32", lambda: wl.config3(M=10, n=8, precision=wl.FP32), 12, 1e-5),
    ("16c_fp32_vortex", lambda: wl.config3(M=11, n=16, precision=wl.FP32), 12, 1e-5),
    ("20c_fp32_vortex", lambda: wl.config3(M=9, n=20, precision=wl.FP32), 12, 1e-5),
    ("20c_fp32_c4", lambda: wl.config4(M=6, n=20, precision=wl.FP32), 10, 1e-5),
]


@pytest.mark.parametrize("name, make, nsteps, tol", CASES, ids=[c[0] for c in CASES])
def test_single_pass_matches_oracle_and_two_kernel_path(lise, name, make, nsteps, tol):
    w = make()
    say(f"single pass {name}: {w.name}, {nsteps} ABM steps (ragged jgroup 3)")
    one = run(lise, w, nsteps, single_pass=1, jgroup=3)
    two = run(lise, w, nsteps, single_pass=-1)
    w64 = make()
    w64.functional.precision = wl.FP64
    ev = oracle.Evolver(w64.lattice, w64.functional, w64.qpwfs())
    ev.step(w.dt, nsteps)
    n0, k0 = oracle.densities(ev.y, w64.functional)
    e_one = (rel_l2(one[1][0], n0), rel_l2(one[1][1], k0), rel_l2(one[0], ev.y))
    e_two = (rel_l2(two[1][0], n0), rel_l2(two[1][1], k0))
    say(f"  single pass: n {e_one[0]:.2e} kappa {e_one[1]:.2e} psi {e_one[2]:.2e}; two kernels: n {e_two[0]:.2e} kappa {e_two[1]:.2e}")
    assert one[2] == two[2]
    assert max(e_one[:2]) < tol
    if w.functional.precision == wl.FP64:
        assert e_one[2] < tol
    # the two paths differ only by rounding
    assert rel_l2(one[1][0], two[1][0]) < (1e-12 if w.functional.precision == wl.FP64 else 1e-5)
