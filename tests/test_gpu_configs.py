"""GPU parity at the lattices of the benchmark configurations: the ABM step kernels of
each form (float64, float32, split-bf16 MFMA) at 32^3, 48^3 and 64^3 against the CPU
float64 oracle, plus the boundary rules on qpwf coverage and the spin-resolved
particle numbers.

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


def gpu_run(lise, w, nsteps, tuning=None):
    ctx = lise.Context(w.lattice, w.M, w.functional)
    if tuning:
        ctx.set_tuning(**tuning)
    ctx.set_qpwf(0, w.qpwfs())
    ctx.step(w.dt, nsteps)
    out = dict(psi=ctx.get_qpwf(0, w.M), dens=ctx.densities(), time=ctx.time(), obs=ctx.observables())
    ctx.close()
    return out


_ORACLE = {}


def oracle_run(w, nsteps):
    """The float64 oracle on the same inputs (cached per workload and step count)."""
    key = (w.name, nsteps)
    if key not in _ORACLE:
        say(f"  oracle {w.name}: {nsteps} ABM steps")
        ev = oracle.Evolver(w.lattice, w.functional, w.qpwfs())
        ev.step(w.dt, nsteps)
        _ORACLE[key] = ev
    return _ORACLE[key]


@pytest.mark.parametrize("z_dense", [0, -1], ids=["default_in_kernel_z", "two_kernels"])
def test_config2_lattice_fp64_100_steps_past_the_ramp(lise, z_dense):
    """32^3 config-2 recipe (lowest-|k| BCS, ramped Gaussian well), M = 16, 3 start-up +
    100 ABM steps (t = 103 dt, past the ramp's end at 100 dt): psi and densities within
    1e-11 relative L2 of the oracle, observables within 1e-10.  Both ABM paths: the
    default (the z-term inside the plane kernel at this lattice) and the z-axis kernel
    with the plane kernel."""
    w = wl.config2(M=16)
    say(f"step {w.name} FP64 100 steps, z_dense {z_dense} (chunk 6, 4 qpwfs per workgroup: ragged chunks and groups)")
    g = gpu_run(lise, w, 100, tuning={"chunk_qpwf": 6, "jgroup": 4, "z_dense": z_dense})
    ev = oracle_run(w, 100)
    n0, k0 = oracle.densities(ev.y, w.functional)
    e = (rel_l2(g["psi"], ev.y), rel_l2(g["dens"][0], n0), rel_l2(g["dens"][1], k0))
    say(f"  rel L2 psi {e[0]:.3e} n {e[1]:.3e} kappa {e[2]:.3e}")
    assert g["time"][1] == 103 and abs(g["time"][0] - ev.t) < 1e-13
    assert max(e) < 1e-11
    o = oracle.observables(ev.y, w.lattice, w.functional, ev.t)
    for key in ("N", "N_up", "N_dn", "E", "E_kin", "E_int", "E_pair", "E_ext", "mean_abs_delta"):
        assert abs(g["obs"][key] - o[key]) < 1e-10 * max(1.0, abs(o[key])), key


def test_config3_lattice_fp32_step(lise):
    """48^3 config-3 recipe (vortex line, phase noise) in float32 with float64 sums,
    M = 4, 3 start-up + 30 ABM steps: densities within 1e-5 relative L2 of the float64
    oracle; the float64 form of the same run within 1e-11."""
    w64 = wl.config3(M=4, n=48, precision=wl.FP64)
    ev = oracle_run(w64, 30)
    n0, k0 = oracle.densities(ev.y, w64.functional)
    for prec, tol in ((wl.FP32, 1e-5), (wl.FP64, 1e-11)):
        w = wl.config3(M=4, n=48, precision=prec)
        say(f"step {w.name} precision {prec} 30 steps")
        g = gpu_run(lise, w, 30)
        e = (rel_l2(g["dens"][0], n0), rel_l2(g["dens"][1], k0))
        say(f"  density rel L2 n {e[0]:.3e} kappa {e[1]:.3e}, psi {rel_l2(g['psi'], ev.y):.3e}")
        assert g["time"][1] == 33
        assert max(e) < tol
        if prec == wl.FP64:
            assert rel_l2(g["psi"], ev.y) < 1e-11


@pytest.mark.parametrize("prec", [wl.FP32, wl.FP32_MFMA], ids=["fp32_register_fft", "mfma_bf16x3"])
def test_config4_lattice_four_component_step(lise, prec):
    """64^3 config-4 recipe (C = 4, spin-imbalanced), M = 2, 3 start-up + 20 ABM steps in
    float32 (register FFTs) and with the split-bf16 MFMA xy-kinetic term: densities
    within 1e-5 relative L2 of the float64 oracle; spin numbers within 1e-5."""
    w = wl.config4(M=2, n=64, precision=prec)
    w64 = wl.config4(M=2, n=64, precision=wl.FP64)
    ev = oracle_run(w64, 20)
    say(f"step {w.name} precision {prec} 20 steps")
    g = gpu_run(lise, w, 20)
    n0, k0 = oracle.densities(ev.y, w64.functional)
    e = (rel_l2(g["dens"][0], n0), rel_l2(g["dens"][1], k0))
    say(f"  density rel L2 n {e[0]:.3e} kappa {e[1]:.3e}, psi {rel_l2(g['psi'], ev.y):.3e}")
    assert g["time"][1] == 23
    assert max(e) < 1e-5
    o = oracle.observables(ev.y, w64.lattice, w64.functional, ev.t)
    for key in ("N", "N_up", "N_dn"):
        assert abs(g["obs"][key] - o[key]) < 1e-5 * o["N"], key


def test_spin_numbers_four_components_fp64(lise):
    """N_up, N_dn of a spin-imbalanced C = 4 set (8^3, FP64) after 10 ABM steps equal
    the oracle's to 1e-12 and differ from each other (the blocks have unequal sizes)."""
    w = wl.config4(M=40, n=8, precision=wl.FP64)
    say(f"step {w.name} 10 steps: spin-resolved numbers")
    g = gpu_run(lise, w, 10)
    ev = oracle_run(w, 10)
    o = oracle.observables(ev.y, w.lattice, w.functional, ev.t)
    say(f"  N_up {g['obs']['N_up']:.12f} (oracle {o['N_up']:.12f}), N_dn {g['obs']['N_dn']:.12f}")
    assert abs(g["obs"]["N_up"] - o["N_up"]) < 1e-12 * o["N"]
    assert abs(g["obs"]["N_dn"] - o["N_dn"]) < 1e-12 * o["N"]
    assert abs(g["obs"]["N_up"] + g["obs"]["N_dn"] - g["obs"]["N"]) < 1e-12 * o["N"]
    assert abs(o["N_up"] - o["N_dn"]) > 1e-3


def test_set_qpwf_requires_every_qpwf(lise):
    """lise_set_qpwf tracks which qpwfs were written: setting only the last one, or all
    but one, leaves every whole-state call at LISE_E_STATE; the missing one completes the
    set.  After an evolution a partial set starts the coverage over."""
    w = wl.config1(M=8)
    psi = w.qpwfs()
    say(f"coverage {w.name}")
    ctx = lise.Context(w.lattice, w.M, w.functional)
    ctx.set_qpwf(w.M - 1, psi[w.M - 1:])
    for call in (lambda: ctx.step(w.dt, 1), lambda: ctx.densities(), lambda: ctx.observables(),
                 lambda: ctx.apply_h(0, 1), lambda: ctx.startup(w.dt), lambda: ctx.current()):
        with pytest.raises(lise.LiseError, match="STATE"):
            call()
    ctx.set_qpwf(0, psi[:3])
    ctx.set_qpwf(4, psi[4:7])
    with pytest.raises(lise.LiseError, match="STATE"):
        ctx.step(w.dt, 1)
    ctx.set_qpwf(3, psi[3:4])          # the last missing qpwf
    ctx.step(w.dt, 1)
    ctx.set_qpwf(2, psi[2:3])          # partial set after an evolution: coverage restarts
    with pytest.raises(lise.LiseError, match="STATE"):
        ctx.step(w.dt, 1)
    ctx.set_qpwf(0, psi)
    ctx.set_time(0.0)
    ctx.step(w.dt, 1)
    ev = oracle.Evolver(w.lattice, w.functional, psi)
    ev.step(w.dt, 1)
    assert rel_l2(ctx.get_qpwf(0, w.M), ev.y) < 1e-12
    ctx.close()


@pytest.mark.parametrize("zl", [2, 4])
def test_z_lanes_steps_match_oracle(lise, zl):
    """The z-axis kernel with 2 or 4 lanes per column (the autotuner's z_lanes choice):
    32^3 FP64 and 24^3 FP32 steps against the oracle (1e-11, 1e-5), and a batch of both
    equal to the systems alone bit for bit."""
    cases = [(wl.config2(M=5, n=32), 1e-11), (wl.config3(M=6, n=24, precision=wl.FP32), 1e-5)]
    outs = []
    for w, tol in cases:
        say(f"z lanes {zl}: {w.name} 8 steps")
        g = gpu_run(lise, w, 8, tuning={"z_lanes": zl})
        w64 = wl.config2(M=5, n=32) if w.functional.precision == wl.FP64 else wl.config3(M=6, n=24, precision=wl.FP64)
        ev = oracle_run(w64, 8)
        n0, k0 = oracle.densities(ev.y, w64.functional)
        e = (rel_l2(g["dens"][0], n0), rel_l2(g["dens"][1], k0))
        say(f"  density rel L2 n {e[0]:.3e} kappa {e[1]:.3e}")
        assert max(e) < tol
        outs.append(g["psi"])
    ctxs = []
    for w, _ in cases:
        c = lise.Context(w.lattice, w.M, w.functional)
        c.set_tuning(z_lanes=zl)
        c.set_qpwf(0, w.qpwfs())
        ctxs.append(c)
    b = lise.Batch(ctxs)
    b.step(cases[0][0].dt, 8)
    got = [c.get_qpwf(0, w.M) for c, (w, _) in zip(ctxs, cases)]
    b.close()
    for c in ctxs:
        c.close()
    for g, ref in zip(got, outs):
        assert np.array_equal(g, ref)
