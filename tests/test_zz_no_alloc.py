"""GPU check of lise_apply_h_noalloc, the entry point for callers that cannot allocate:
through the C-ABI, on two calls in a row (the second with fewer qpwfs), its output equals
lise_apply_h's bit for bit, in float64 (several staging pieces per call) and float32.

Every case prints its name and shape before it touches the GPU.
"""
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    import paper_2009_00745_amd as lise_mod
    lise_mod.load_library()
    return lise_mod, torch


# (workload, calls as (first, count)): 32^3 float64 qpwfs are 1 MiB, so 64 fill one
# 64 MiB piece and the first call takes three pieces; the second call is smaller
CASES = [
    ("fp64_32c", lambda: wl.config2(M=150, n=32), [(0, 150), (37, 20)]),
    ("fp32_24c", lambda: wl.config3(M=40, n=24, precision=wl.FP32), [(0, 40), (5, 3)]),
]


@pytest.mark.parametrize("name, make, calls", CASES, ids=[c[0] for c in CASES])
def test_apply_h_noalloc_equals_apply_h(env, name, make, calls):
    lise, torch = env
    w = make()
    say(f"apply_h_noalloc {w.name}: calls {calls}")
    ctx = lise.Context(w.lattice, w.M, w.functional)
    ctx.set_qpwf(0, w.qpwfs())
    ctx.step(w.dt, 2)                 # an evolved state, fields at t > 0
    shape = (w.functional.ncomp, w.lattice.nz, w.lattice.ny, w.lattice.nx)
    for first, count in calls:
        say(f"  first {first} count {count}")
        out = torch.full((count,) + shape, complex("nan"), dtype=torch.complex128, device="cuda")
        ctx.apply_h_noalloc(first, count, out)
        ref = torch.empty_like(out)
        ctx.apply_h(first, count, ref)
        torch.cuda.synchronize()
        got, exp = out.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(got).all()
        assert np.array_equal(got, exp), (name, first, count)
    ctx.close()


def test_apply_h_noalloc_rejects_bad_calls(env):
    lise, torch = env
    w = wl.config1(M=8)
    say("apply_h_noalloc argument checks")
    ctx = lise.Context(w.lattice, w.M, w.functional)
    out = torch.empty((2, 2, 8, 8, 8), dtype=torch.complex128, device="cuda")
    with pytest.raises(lise.LiseError, match="STATE"):
        ctx.apply_h_noalloc(0, 2, out)          # qpwfs not set
    ctx.set_qpwf(0, w.qpwfs())
    with pytest.raises(lise.LiseError, match="ARG"):
        ctx.apply_h_noalloc(7, 2, out)          # range beyond M
    with pytest.raises(ValueError):
        ctx.apply_h_noalloc(0, 2, np.empty((2, 2, 8, 8, 8), dtype=complex))
    ctx.close()
