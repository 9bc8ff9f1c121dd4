"""GPU parity: the HIP library (through its C-ABI) against the CPU FP64 oracle.

Every case prints its name and shape before touching the GPU.
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


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def random_state(lat, M, C, seed):
    rng = np.random.default_rng(seed)
    shp = (M, C, lat.nz, lat.ny, lat.nx)
    psi = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    psi /= np.sqrt(np.sum(np.abs(psi) ** 2, axis=(1, 2, 3, 4), keepdims=True) * lat.a ** 3)
    return psi


APPLY_CASES = [
    # (nx, ny, nz, a, C, M, precision, tuning)
    (4, 4, 4, 1.0, 2, 5, 0, {}),
    (8, 8, 8, 1.0, 2, 7, 0, {}),
    (8, 8, 8, 1.0, 2, 7, 0, {"fused": 1}),
    (8, 8, 8, 1.0, 2, 7, 0, {"fused": -1}),
    (6, 10, 8, 0.8, 2, 4, 0, {}),
    (6, 10, 8, 0.8, 2, 9, 0, {"fused": -1, "chunk_qpwf": 4, "jgroup": 3}),
    (5, 3, 4, 1.2, 2, 3, 0, {}),
    (12, 12, 12, 1.0, 4, 3, 0, {}),
    (20, 20, 20, 1.0, 2, 3, 0, {}),
    (24, 16, 20, 1.0, 4, 2, 0, {}),
    (32, 32, 32, 1.0, 2, 3, 0, {}),
    (32, 32, 32, 1.0, 2, 3, 0, {"generic": 1}),
    (24, 24, 24, 1.0, 4, 2, 0, {}),
    (20, 20, 16, 1.0, 2, 3, 0, {"chunk_qpwf": 2, "jgroup": 1}),
    (16, 16, 16, 1.0, 2, 6, 1, {}),
    (16, 16, 16, 1.0, 2, 6, 1, {"fused": 1}),
    (16, 16, 16, 1.0, 2, 6, 1, {"fused": -1}),
    (48, 48, 48, 1.0, 2, 2, 1, {}),
    (48, 48, 48, 1.0, 2, 2, 1, {"generic": 1}),
    (64, 64, 64, 1.0, 4, 1, 1, {}),
    (8, 8, 8, 1.0, 2, 4, 0, {"fused": -1, "generic": 0}),
    (32, 32, 32, 1.0, 2, 5, 0, {"chunk_qpwf": 2, "jgroup": 1}),
    (32, 32, 32, 1.0, 2, 5, 0, {"chunk_qpwf": 2, "jgroup": 1, "no_overlap": 1}),
    (16, 16, 16, 1.0, 2, 3, 2, {}),
    (32, 32, 32, 1.0, 2, 3, 2, {}),
    (48, 48, 48, 1.0, 2, 2, 2, {}),
    (64, 64, 64, 1.0, 4, 1, 2, {}),
    (32, 32, 24, 0.9, 4, 2, 2, {"chunk_qpwf": 1, "jgroup": 1}),
    # float32 planes whose rows are partial cache lines (natural-order path), ragged qpwf groups
    (8, 8, 8, 1.0, 2, 5, 1, {"fused": -1}),
    (20, 20, 20, 1.0, 2, 5, 1, {"jgroup": 2}),
    (24, 24, 20, 1.0, 4, 3, 1, {"chunk_qpwf": 2, "jgroup": 1}),
]


@pytest.mark.parametrize("case", APPLY_CASES, ids=lambda c: "x".join(map(str, c[:3])) + f"_C{c[4]}_p{c[6]}_{c[7]}")
def test_apply_h_matches_oracle(lise, case):
    nx, ny, nz, a, C, M, prec, tun = case
    say(f"apply_h {nx}x{ny}x{nz} C={C} M={M} prec={prec} tuning={tun}")
    lat = wl.Lattice(nx, ny, nz, a)
    fn = wl.Functional(ncomp=C, mu_up=0.4, mu_dn=0.25 if C == 4 else 0.4, beta=0.37, g=1.7, w=2.0 if C == 2 else 1.0,
                       ext_A=-0.2, ext_w=1.5, ext_r0=(1.0 * a, 2.0 * a, 0.0), ext_t_on=0.0, precision=prec)
    psi = random_state(lat, M, C, seed=nx * 100 + ny * 10 + nz + M)
    ctx = lise.Context(lat, M, fn)
    if tun:
        ctx.set_tuning(**tun)
    ctx.set_qpwf(0, psi)
    got = ctx.apply_h(0, M)
    V, D = oracle.hamiltonian_of(psi, lat, fn, 0.0)
    ref = oracle.apply_h(psi, V, D, lat, fn)
    tol = {0: 1e-12, 1: 3e-6, 2: 5e-5}[prec]
    err = rel_max(got, ref)
    say(f"  rel max err {err:.3e}")
    assert err < tol
    # a sub-range
    if M > 2:
        sub = ctx.apply_h(1, M - 2)
        assert rel_max(sub, ref[1:M - 1]) < tol
    n, k = ctx.densities()
    n0, k0 = oracle.densities(psi, fn)
    dtol = 1e-13 if prec == 0 else 1e-6
    assert rel_max(n, n0) < dtol and rel_max(k, k0) < dtol
    ctx.close()


def run_pair(lise, w, nsteps, tuning=None, psi=None):
    psi = w.qpwfs() if psi is None else psi
    ctx = lise.Context(w.lattice, w.M, w.functional)
    if tuning:
        ctx.set_tuning(**tuning)
    ctx.set_qpwf(0, psi)
    ctx.step(w.dt, nsteps)
    got = ctx.get_qpwf(0, w.M)
    n, k = ctx.densities()
    t, s = ctx.time()
    obs = ctx.observables()
    ctx.close()
    ev = oracle.Evolver(w.lattice, w.functional, psi)
    ev.step(w.dt, nsteps)
    return got, n, k, t, s, obs, ev


def test_config1_full_100_steps(lise):
    """8^3, M = 1024, FP64, 3 start-up + 100 ABM steps: psi and densities within 1e-11."""
    w = wl.config1()
    say(f"step {w.name} 100 steps")
    got, n, k, t, s, obs, ev = run_pair(lise, w, 100)
    n0, k0 = oracle.densities(ev.y, w.functional)
    e_psi, e_n, e_k = rel_l2(got, ev.y), rel_l2(n, n0), rel_l2(k, k0)
    say(f"  rel L2: psi {e_psi:.3e} n {e_n:.3e} kappa {e_k:.3e}")
    assert abs(t - ev.t) < 1e-13 and s == 103
    assert e_psi < 1e-11 and e_n < 1e-11 and e_k < 1e-11
    o = oracle.observables(ev.y, w.lattice, w.functional, ev.t)
    for key in ("N", "E", "E_kin", "E_int", "E_pair", "mean_abs_delta"):
        assert abs(obs[key] - o[key]) < 1e-10 * max(1.0, abs(o[key])), key
    assert np.allclose(obs["r_cm"], o["r_cm"], atol=1e-10)


def test_long_run_fp64_stays_on_the_oracle(lise):
    """500 ABM steps (8^3, M = 64, config-1 recipe, then again with phase removal):
    the FP64 path stays on the oracle's trajectory to round-off accumulation."""
    for rp in (0, 1):
        w = wl.config1(M=64)
        w.functional.remove_phase = rp
        say(f"long run {w.name} remove_phase={rp}: 500 steps")
        got, n, k, t, s, obs, ev = run_pair(lise, w, 500)
        n0, k0 = oracle.densities(ev.y, w.functional)
        e = (rel_l2(got, ev.y), rel_l2(n, n0), rel_l2(k, k0))
        say(f"  rel L2 after 500 steps: {e}")
        assert s == 503 and max(e) < 1e-11


def test_config2_reduced_with_bump(lise):
    """32^3 lowest-|k| BCS + ramped Gaussian well, M = 32, 12 ABM steps."""
    w = wl.config2(M=32)
    say(f"step {w.name} 12 steps (chunked, jgroup 5)")
    got, n, k, t, s, obs, ev = run_pair(lise, w, 12, tuning={"chunk_qpwf": 12, "jgroup": 5})
    n0, k0 = oracle.densities(ev.y, w.functional)
    e = (rel_l2(got, ev.y), rel_l2(n, n0), rel_l2(k, k0))
    say(f"  rel L2: {e}")
    assert max(e) < 1e-11
    o = oracle.observables(ev.y, w.lattice, w.functional, ev.t)
    assert abs(obs["E_ext"] - o["E_ext"]) < 1e-10 * abs(o["E_ext"])
    assert abs(obs["E"] - o["E"]) < 1e-10 * abs(o["E"])


def test_regularised_coupling_step(lise):
    """Eq. (geff_3D) coupling (regularize = 1) on the 16^3 config-2 recipe, M = 24, and
    on a C = 4 8^3 set, 12 ABM steps each, against the oracle."""
    for w in (wl.config2(M=24, n=16), wl.config4(M=24, n=8, precision=wl.FP64)):
        w.functional.regularize = 1
        say(f"step {w.name} regularised, 12 steps")
        got, n, k, t, s, obs, ev = run_pair(lise, w, 12)
        n0, k0 = oracle.densities(ev.y, w.functional)
        e = (rel_l2(got, ev.y), rel_l2(n, n0), rel_l2(k, k0))
        say(f"  rel L2: {e}")
        assert max(e) < 1e-11
        o = oracle.observables(ev.y, w.lattice, w.functional, ev.t)
        assert abs(obs["E_pair"] - o["E_pair"]) < 1e-10 * abs(o["E_pair"])


def test_phase_removal_step(lise):
    """Eq. (sp_en) phase removal: FP64 on the fast path (16^3, chunked, overlap) and on
    the fused path (C = 4, 8^3) against the oracle; FP32 and the bf16x3 MFMA form
    against the FP64 oracle densities."""
    cases = [(wl.config2(M=24, n=16), {"chunk_qpwf": 10, "jgroup": 3}, 1e-11),
             (wl.config4(M=24, n=8, precision=wl.FP64), {}, 1e-11),
             (wl.config3(M=16, n=20, precision=wl.FP32), {}, 1e-5),
             (wl.config4(M=12, n=16, precision=wl.FP32_MFMA), {}, 1e-5)]
    for w, tuning, tol in cases:
        w.functional.remove_phase = 1
        prec = w.functional.precision
        say(f"step {w.name} phase removed (precision {prec}), 12 steps")
        got, n, k, t, s, obs, ev = run_pair(lise, w, 12, tuning=tuning)
        n0, k0 = oracle.densities(ev.y, w.functional)
        e = (rel_l2(n, n0), rel_l2(k, k0))
        if prec == wl.FP64:
            e = (rel_l2(got, ev.y),) + e
        say(f"  rel L2: {e}")
        assert max(e) < tol


def test_phase_removal_two_eta_passes_agree(lise):
    """The Parseval eta pass of the register-FFT kernels and the full recomputation of
    the generic kernels give the same evolution to rounding (FP64, 16^3 and 20^3)."""
    for w in (wl.config2(M=12, n=16), wl.config3(M=8, n=20, precision=wl.FP64)):
        w.functional.remove_phase = 1
        outs = []
        for generic in (0, 1):
            say(f"{w.name} phase removed, generic kernels = {generic}, 8 steps")
            ctx = lise.Context(w.lattice, w.M, w.functional)
            ctx.set_tuning(generic=generic)
            ctx.set_qpwf(0, w.qpwfs())
            ctx.step(w.dt, 8)
            outs.append(ctx.get_qpwf(0, w.M))
            ctx.close()
        e = rel_l2(outs[0], outs[1])
        say(f"  rel L2 between the two eta passes {e:.3e}")
        assert e < 1e-12


def test_phase_removal_full_eta_pass_on_register_plane_kernel(lise):
    """Phase removal where the plane kernel is the register-FFT one but the z axis is not
    (nz = 12): the full eta recomputation runs on that plane kernel, in the lane order
    (16^2 FP64) and in the natural order (20^2 FP64 and FP32), against the oracle."""
    for n, prec, tol in ((16, wl.FP64, 1e-11), (20, wl.FP64, 1e-11), (20, wl.FP32, 1e-5)):
        lat = wl.Lattice(n, n, 12, 1.0)
        fn = wl.Functional(ncomp=2, mu_up=0.5, mu_dn=0.5, beta=0.37, g=2.0, w=2.0, ext_A=-0.025, ext_w=3.0,
                           ext_r0=(2.0, 3.0, 4.0), ext_t_on=0.0, remove_phase=1, precision=prec)
        M = 12
        w = wl.Workload(f"eta_full_{n}x{n}x12_p{prec}", lat, fn, M, 0.002, 6,
                        wl.uniform_bcs(lat, fn, M, 0.3, 0.5, eps=1e-2))
        say(f"step {w.name} phase removed, full eta pass, 6 steps")
        got, dn, dk, t, s, obs, ev = run_pair(lise, w, 6)
        n0, k0 = oracle.densities(ev.y, fn)
        e = (rel_l2(dn, n0), rel_l2(dk, k0))
        if prec == wl.FP64:
            e = (rel_l2(got, ev.y),) + e
        say(f"  rel L2: {e}")
        assert max(e) < tol


def test_phase_removal_frozen_eigenvectors_stay_put(lise):
    """Frozen fields, plane-wave BdG eigenvectors: with the phase removed y' = 0."""
    lat = wl.Lattice(16, 16, 16, 1.0)
    U0, D0, mu = 0.15, 0.4 * np.exp(-0.3j), 0.7
    fn = wl.Functional(ncomp=2, mu_up=mu, mu_dn=mu, frozen=1, U0=U0, Delta0=D0, g=1.0, remove_phase=1)
    idx = wl.k_order(lat)[:32]
    pw = wl.plane_waves(lat, idx)
    k2 = np.sum(wl.k_of(lat, idx) ** 2, axis=1)
    ab = []
    for j in range(32):
        xi = 0.5 * k2[j] + U0 - mu
        ab.append(np.linalg.eigh(np.array([[xi, D0], [np.conj(D0), -xi]]))[1][:, j % 2])
    psi = np.array(ab)[:, :, None, None, None] * pw[:, None]
    say("frozen eigenvectors, phase removed, 16^3 M = 32, 40 steps")
    ctx = lise.Context(lat, 32, fn)
    ctx.set_qpwf(0, psi)
    ctx.step(0.004, 40)
    got = ctx.get_qpwf(0, 32)
    ctx.close()
    err = float(np.max(np.abs(got - psi)) / np.max(np.abs(psi)))
    say(f"  max deviation {err:.3e}")
    assert err < 1e-12


def lattice_chi(lat, p, seed=None, amp=0.0):
    """chi = p.r, plus a smooth random periodic part when amp > 0."""
    x = np.arange(lat.nx) * lat.a
    y = np.arange(lat.ny) * lat.a
    z = np.arange(lat.nz) * lat.a
    chi = p[0] * x[None, None, :] + p[1] * y[None, :, None] + p[2] * z[:, None, None]
    if amp:
        rng = np.random.default_rng(seed)
        for _ in range(3):
            m = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            kx, ky, kz = (2 * np.pi * m[0] / (lat.nx * lat.a), 2 * np.pi * m[1] / (lat.ny * lat.a),
                          2 * np.pi * m[2] / (lat.nz * lat.a))
            chi = chi + amp * np.cos(kx * x[None, None, :] + ky * y[None, :, None] + kz * z[:, None, None] + ph)
    return chi


def test_current_density_matches_oracle(lise):
    """Eq. (j) current and P, v_cm of the observables after a few steps: FP64 (C = 2 on
    16^3 and 20^3, C = 4 on 8^3) against the oracle; FP32 within 1e-6."""
    cases = [(wl.config2(M=24, n=16), 1e-12), (wl.config3(M=16, n=20, precision=wl.FP64), 1e-12),
             (wl.config4(M=24, n=8, precision=wl.FP64), 1e-12),
             (wl.config3(M=16, n=20, precision=wl.FP32), 1e-6)]
    for w, tol in cases:
        say(f"current {w.name} precision {w.functional.precision}: 4 steps")
        ctx = lise.Context(w.lattice, w.M, w.functional)
        ctx.set_qpwf(0, w.qpwfs())
        ctx.step(w.dt, 4)
        j = ctx.current()
        obs = ctx.observables()
        ctx.close()
        ev = oracle.Evolver(w.lattice, w.functional, w.qpwfs())
        ev.step(w.dt, 4)
        jr = oracle.current_density(ev.y, w.lattice, w.functional)
        o = oracle.observables(ev.y, w.lattice, w.functional, ev.t)
        e = rel_l2(j, jr)
        scale = max(np.max(np.abs(jr)), 1e-300) * w.lattice.a ** 3 * w.lattice.n
        dP = max(abs(obs["P"][k] - o["P"][k]) for k in range(3)) / scale
        say(f"  j rel L2 {e:.3e}, P diff / scale {dP:.3e}")
        assert e < tol and dP < 10 * tol


def test_total_current_routes_agree(lise):
    """The observables' total current P (Parseval sums of the kinetic pass and of a z pass
    over the v components, register-FFT kernels) equals a^3 times the sum of the
    current-density field, and both equal the oracle's, after a boost: FP64 16^3 (lane
    order), 20^3 (natural order), C = 4 8^3, the generic kernels (field route only), FP32 24^3."""
    cases = [(wl.config2(M=24, n=16), {}, 1e-11), (wl.config3(M=16, n=20, precision=wl.FP64), {}, 1e-11),
             (wl.config4(M=24, n=8, precision=wl.FP64), {}, 1e-11),
             (wl.config2(M=24, n=16), {"generic": 1}, 1e-11),
             (wl.config3(M=16, n=24, precision=wl.FP32), {}, 1e-5)]
    for w, tuning, tol in cases:
        lat = w.lattice
        p = np.array([2 * np.pi / (lat.nx * lat.a), -4 * np.pi / (lat.ny * lat.a), 2 * np.pi / (lat.nz * lat.a)])
        chi = lattice_chi(lat, p, seed=5, amp=0.2)
        say(f"total current {w.name} precision {w.functional.precision} tuning {tuning}: kick, 2 steps")
        ctx = lise.Context(lat, w.M, w.functional)
        if tuning:
            ctx.set_tuning(**tuning)
        ctx.set_qpwf(0, w.qpwfs())
        ctx.kick(chi)
        ctx.step(w.dt, 2)
        obs = ctx.observables()
        j = ctx.current()
        psi = ctx.get_qpwf(0, w.M)
        ctx.close()
        P_field = lat.a ** 3 * j.reshape(3, -1).sum(axis=1)
        P_ref = lat.a ** 3 * oracle.current_density(psi, lat, w.functional).reshape(3, -1).sum(axis=1)
        scale = np.max(np.abs(P_ref))
        d1 = float(np.max(np.abs(np.array(obs["P"]) - P_field)) / scale)
        d2 = float(np.max(np.abs(np.array(obs["P"]) - P_ref)) / scale)
        say(f"  P {obs['P']} field {P_field} oracle {P_ref}: rel diff {d1:.3e} / {d2:.3e}")
        assert scale > 1e-3
        assert d1 < tol and d2 < tol


def test_kick_then_step_matches_oracle(lise):
    """Eq. (kick) with chi = p.r plus a smooth random field, then start-up + 10 ABM
    steps; C = 2 (16^3, FP64) and C = 4 (8^3, FP64)."""
    for w in (wl.config2(M=24, n=16), wl.config4(M=24, n=8, precision=wl.FP64)):
        lat = w.lattice
        p = np.array([2 * np.pi / (lat.nx * lat.a), 0.0, -2 * np.pi / (lat.nz * lat.a)])
        chi = lattice_chi(lat, p, seed=3, amp=0.3)
        say(f"kick {w.name}: 3 steps, kick, 10 steps")
        ctx = lise.Context(lat, w.M, w.functional)
        ctx.set_qpwf(0, w.qpwfs())
        ctx.step(w.dt, 3)
        ctx.kick(chi)
        after_kick = ctx.get_qpwf(0, w.M)
        ctx.step(w.dt, 10)
        got = ctx.get_qpwf(0, w.M)
        (t, s) = ctx.time()
        ctx.close()
        ev = oracle.Evolver(lat, w.functional, w.qpwfs())
        ev.step(w.dt, 3)
        k = oracle.kick(ev.y, chi, w.functional)
        assert rel_l2(after_kick, k) < 1e-14
        ev2 = oracle.Evolver(lat, w.functional, k, ev.t)
        ev2.step_count = ev.step_count
        ev2.step(w.dt, 10)
        assert abs(t - ev2.t) < 1e-13 and s == ev2.step_count
        e = rel_l2(got, ev2.y)
        say(f"  rel L2 after 10 steps {e:.3e}")
        assert e < 1e-11


def test_boosted_uniform_state_velocity(lise):
    """Kicked closed-shell uniform BCS state: v_cm = p while it evolves (Galilean covariance)."""
    lat = wl.Lattice(16, 16, 16, 1.0)
    fn = wl.Functional(ncomp=2, mu_up=0.8, mu_dn=0.8, beta=0.37, g=2.0, w=2.0)
    M = 33
    psi = wl.uniform_bcs(lat, fn, M, 0.45, 0.8)(0, M)
    p = np.array([2 * np.pi / 16, 0.0, 0.0])
    say("boosted uniform state 16^3, M = 33, 40 steps")
    ctx = lise.Context(lat, M, fn)
    ctx.set_qpwf(0, psi)
    ctx.kick(lattice_chi(lat, p))
    v0 = ctx.observables()["v_cm"]
    ctx.step(0.005, 40)
    v1 = ctx.observables()["v_cm"]
    ctx.close()
    say(f"  v_cm before {v0}, after {v1}")
    assert np.allclose(v0, p, atol=1e-12) and np.allclose(v1, p, atol=1e-10)


def test_four_component_step(lise):
    """C = 4 spin-imbalanced set on 8^3 (FP64), 20 ABM steps."""
    w = wl.config4(M=48, n=8, precision=wl.FP64)
    say(f"step {w.name} 20 steps")
    got, n, k, t, s, obs, ev = run_pair(lise, w, 20)
    n0, k0 = oracle.densities(ev.y, w.functional)
    e = (rel_l2(got, ev.y), rel_l2(n, n0), rel_l2(k, k0))
    say(f"  rel L2: {e}")
    assert max(e) < 1e-11


def test_vortex_fp64_reduced(lise):
    """Config-3 recipe (vortex line, phase noise) at 16^3, M = 64, FP64, 20 steps."""
    w = wl.config3(M=64, n=16, precision=wl.FP64)
    say(f"step {w.name} 20 steps")
    got, n, k, t, s, obs, ev = run_pair(lise, w, 20)
    n0, k0 = oracle.densities(ev.y, w.functional)
    e = (rel_l2(got, ev.y), rel_l2(n, n0), rel_l2(k, k0))
    say(f"  rel L2: {e}")
    assert max(e) < 1e-11


def test_fp32_density_error_config1(lise):
    """FP32 bulk with FP64 sums: densities within 1e-5 relative L2 of the FP64 oracle after 100 steps."""
    w = wl.config1()
    w.functional.precision = wl.FP32
    say(f"step {w.name} FP32 100 steps")
    got, n, k, t, s, obs, ev = run_pair(lise, w, 100)
    n0, k0 = oracle.densities(ev.y, w.functional)
    e = (rel_l2(n, n0), rel_l2(k, k0))
    say(f"  FP32 density rel L2 {e}, psi {rel_l2(got, ev.y):.3e}")
    assert max(e) < 1e-5


def test_fp32_density_error_vortex(lise):
    w = wl.config3(M=64, n=24, precision=wl.FP32)
    say(f"step {w.name} FP32 30 steps")
    got, n, k, t, s, obs, ev = run_pair(lise, w, 30)
    n0, k0 = oracle.densities(ev.y, w.functional)
    e = (rel_l2(n, n0), rel_l2(k, k0))
    say(f"  FP32 density rel L2 {e}")
    assert max(e) < 1e-5


def test_mfma_form_density_error_four_component(lise):
    """Split-bf16 MFMA xy-kinetic term (C = 4, spin-imbalanced, 32^3): densities within
    1e-5 relative L2 of the FP64 oracle after 30 steps, next to the FP32 FFT form."""
    errs = {}
    for prec in (wl.FP32, wl.FP32_MFMA):
        w = wl.config4(M=24, n=32, precision=prec)
        say(f"step {w.name} precision {prec} 30 steps")
        got, n, k, t, s, obs, ev = run_pair(lise, w, 30) if prec == wl.FP32 else run_pair(lise, w, 30)
        n0, k0 = oracle.densities(ev.y, w.functional)
        errs[prec] = (rel_l2(n, n0), rel_l2(k, k0))
        say(f"  density rel L2 {errs[prec]}")
    assert max(errs[wl.FP32_MFMA]) < 1e-5
    assert max(errs[wl.FP32]) < 1e-5


def test_frozen_uniform_bcs_closed_form(lise):
    """Frozen U0, Delta0: each momentum evolves by the closed-form 2x2 rotation."""
    import math
    lat = wl.Lattice(8, 8, 8, 1.0)
    U0, D0, mu = 0.15, 0.4 * np.exp(-0.3j), 0.7
    fn = wl.Functional(ncomp=2, mu_up=mu, mu_dn=mu, frozen=1, U0=U0, Delta0=D0, g=1.0)
    M = 40
    idx = wl.k_order(lat)[:M]
    pw = wl.plane_waves(lat, idx)
    rng = np.random.default_rng(11)
    ab = rng.standard_normal((M, 2)) + 1j * rng.standard_normal((M, 2))
    ab /= np.linalg.norm(ab, axis=1, keepdims=True)
    psi = ab[:, :, None, None, None] * pw[:, None]
    say("frozen uniform BCS 8^3 M=40, 200 steps")
    ctx = lise.Context(lat, M, fn)
    ctx.set_qpwf(0, psi)
    dt = 0.004
    ctx.step(dt, 200)
    got = ctx.get_qpwf(0, M)
    t, _ = ctx.time()
    ctx.close()
    k2 = np.sum(wl.k_of(lat, idx) ** 2, axis=1)
    for j in range(M):
        xi = 0.5 * k2[j] + U0 - mu
        Hk = np.array([[xi, D0], [np.conj(D0), -xi]])
        E = math.sqrt(xi * xi + abs(D0) ** 2)
        exact = (math.cos(E * t) * np.eye(2) - 1j * math.sin(E * t) * Hk / E) @ ab[j]
        assert np.max(np.abs(got[j] / pw[j][None] - exact[:, None, None, None])) < 2e-9


def test_free_plane_wave_phase(lise):
    lat = wl.Lattice(16, 16, 16, 1.0)
    fn = wl.Functional(ncomp=2, mu_up=0.0, mu_dn=0.0, beta=0.37, g=1.5, w=2.0)
    idx = np.array([[0, 0, 0], [1, 0, 0], [3, -5, 2], [-8, -8, -8], [7, 7, -8]])
    pw = wl.plane_waves(lat, idx)
    psi = np.zeros((len(idx), 2, 16, 16, 16), dtype=complex)
    psi[:, 0] = pw
    say("free plane waves 16^3, 60 steps")
    ctx = lise.Context(lat, len(idx), fn)
    ctx.set_qpwf(0, psi)
    dt = 0.002
    ctx.step(dt, 60)
    got = ctx.get_qpwf(0, len(idx))
    ctx.close()
    ev = oracle.Evolver(lat, fn, psi)
    ev.step(dt, 60)
    assert rel_max(got, ev.y) < 1e-12
    k2 = np.sum(wl.k_of(lat, idx) ** 2, axis=1)
    t = 63 * dt
    for j in range(len(idx)):
        ph = np.exp(-0.5j * k2[j] * t)
        z = 0.5 * k2[j] * dt
        bound = 2 * (3 * z ** 5 / 120 + 60 * 2e-9 * (z / 0.074) ** 6) + 1e-12
        assert np.max(np.abs(got[j, 0] - ph * pw[j])) < bound * np.max(np.abs(pw[j]))
        assert np.max(np.abs(got[j, 1])) == 0.0


def test_single_qpwf_and_odd_lattice(lise):
    lat = wl.Lattice(5, 3, 4, 1.0)
    fn = wl.Functional(ncomp=2, mu_up=0.3, mu_dn=0.3, beta=0.37, g=1.0, w=2.0)
    psi = random_state(lat, 1, 2, seed=3)
    say("M=1 on 5x3x4, 10 steps")
    ctx = lise.Context(lat, 1, fn)
    ctx.set_qpwf(0, psi)
    ctx.step(0.01, 10)
    got = ctx.get_qpwf(0, 1)
    ctx.close()
    ev = oracle.Evolver(lat, fn, psi)
    ev.step(0.01, 10)
    assert rel_l2(got, ev.y) < 1e-12


def test_overlap_matches_serial_bitwise(lise):
    """The z kernel running one chunk ahead on the internal stream gives bit-identical results."""
    w = wl.config2(M=40, n=16, steps=10)
    psi = w.qpwfs()
    outs = []
    for no_ov in (0, 1):
        say(f"overlap={1 - no_ov} 16^3 M=40 chunk 7, 6 steps")
        ctx = lise.Context(w.lattice, w.M, w.functional)
        ctx.set_tuning(chunk_qpwf=7, jgroup=3, no_overlap=no_ov)
        ctx.set_qpwf(0, psi)
        ctx.step(w.dt, 6)
        outs.append(ctx.get_qpwf(0, w.M))
        ctx.close()
    assert np.array_equal(outs[0], outs[1])


def test_graph_replay_matches_eager_bitwise(lise):
    """Four-step graph replays (plus an eager remainder) equal eager stepping bit for bit,
    including the time-dependent external well (time read from device memory)."""
    w = wl.config2(M=20, n=16, steps=10)
    psi = w.qpwfs()
    outs = []
    for graph in (0, 1):
        say(f"graph={graph} 16^3 M=20, 11 steps")
        ctx = lise.Context(w.lattice, w.M, w.functional)
        ctx.set_tuning(chunk_qpwf=8, jgroup=3, graph=graph)
        ctx.set_qpwf(0, psi)
        ctx.step(w.dt, 11)
        ctx.step(w.dt, 9)
        outs.append((ctx.get_qpwf(0, w.M), ctx.densities()[0], ctx.time()))
        ctx.close()
    assert outs[0][2] == outs[1][2]
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def read_checkpoint(path):
    """Reader of the checkpoint layout documented with lise_save."""
    import struct
    with open(path, "rb") as f:
        hdr = f.read(112)
        assert hdr[:8] == b"LISECKP1"
        version, ncomp, prec, nx, ny, nz, hist, eb = struct.unpack("<8i", hdr[8:40])
        a, M, t, step, dt = struct.unpack("<dqdqd", hdr[40:80])
        dtype = np.complex128 if eb == 16 else np.complex64
        shp = (M, ncomp, nz, ny, nx)
        cnt = int(np.prod(shp))
        arrays = [np.fromfile(f, dtype=dtype, count=cnt).reshape(shp) for _ in range(6 if hist else 1)]
        dens = np.fromfile(f, dtype=np.float64, count=3 * nx * ny * nz) if hist else None
        norms = np.fromfile(f, dtype=np.float64, count=M)
        assert f.read() == b""
    return dict(version=version, ncomp=ncomp, precision=prec, shape=shp, history=hist, a=a, t=t,
                step=step, dt=dt, arrays=arrays, dens=dens, norms=norms)


def test_checkpoint_with_history_continues_bitwise(lise, tmp_path):
    """save(with_history) + load + step equals uninterrupted stepping bit for bit (FP64 with
    overlap and graph replays, FP32, FP64 32^3 on the in-kernel z-term path), and the saved
    ABM history matches the oracle's."""
    cases = [(wl.config2(M=24, n=16), {"graph": 1}), (wl.config3(M=16, n=20, precision=wl.FP32), {}),
             (wl.config2(M=6, n=32), {"z_dense": 1, "jgroup": 2})]
    for w, tuning in cases:
        path = str(tmp_path / f"{w.name}.ckpt")
        say(f"checkpoint {w.name}: 7 steps, save, 9 more; reload and 9 steps")
        a = lise.Context(w.lattice, w.M, w.functional)
        a.set_tuning(**tuning)
        a.set_qpwf(0, w.qpwfs())
        a.step(w.dt, 7)
        a.save(path, with_history=True)
        a.step(w.dt, 9)
        ya, ta = a.get_qpwf(0, w.M), a.time()
        na, ka = a.densities()
        a.close()
        b = lise.Context(w.lattice, w.M, w.functional)
        b.set_tuning(**tuning)
        b.load(path)
        b.step(w.dt, 9)
        yb, tb = b.get_qpwf(0, w.M), b.time()
        nb, kb = b.densities()
        b.close()
        assert ta == tb
        assert np.array_equal(ya, yb) and np.array_equal(na, nb) and np.array_equal(ka, kb)
        if w.functional.precision == wl.FP64:
            ck = read_checkpoint(path)
            ev = oracle.Evolver(w.lattice, w.functional, w.qpwfs())
            ev.step(w.dt, 7)
            ref = ev.checkpoint()
            assert ck["history"] == 1 and ck["step"] == ev.step_count and abs(ck["t"] - ev.t) < 1e-14
            assert ck["dt"] == w.dt
            pairs = [(ck["arrays"][0], ref["y"]), (ck["arrays"][1], ref["y_nm1"]),
                     (ck["arrays"][2], ref["dprev"][0]), (ck["arrays"][3], ref["dprev"][1]),
                     (ck["arrays"][4], ref["dprev"][2])]
            errs = [rel_l2(g, r) for g, r in pairs]
            # p_n - c_n is O(dt^6 y^(6)): compare on the scale of y'
            errs.append(float(np.linalg.norm(ck["arrays"][5] - ref["d_n"]) / np.linalg.norm(ref["dprev"][0])))
            n0, k0 = oracle.densities(ref["y"], w.functional)
            N = w.lattice.n
            errs += [rel_l2(ck["dens"][:N], n0.ravel()),
                     rel_l2(ck["dens"][N:2 * N] + 1j * ck["dens"][2 * N:], k0.ravel())]
            say(f"  saved history vs oracle: {errs}")
            assert max(errs) < 1e-11


def test_checkpoint_qpwfs_only_restarts_like_the_oracle(lise, tmp_path):
    """The paper's restart: latest qpwfs only, series start-up again after load."""
    w = wl.config2(M=16, n=16)
    path = str(tmp_path / "latest.ckpt")
    say("checkpoint without history: 5 steps, save, load, start-up + 6 steps")
    a = lise.Context(w.lattice, w.M, w.functional)
    a.set_qpwf(0, w.qpwfs())
    a.step(w.dt, 5)
    a.save(path, with_history=False)
    a.close()
    b = lise.Context(w.lattice, w.M, w.functional)
    b.load(path)
    b.step(w.dt, 6)
    got, (t, s) = b.get_qpwf(0, w.M), b.time()
    b.close()
    ev = oracle.Evolver(w.lattice, w.functional, w.qpwfs())
    ev.step(w.dt, 5)
    r = oracle.Evolver.restore(w.lattice, w.functional, ev.checkpoint(with_history=False))
    r.step(w.dt, 6)
    assert s == r.step_count and abs(t - r.t) < 1e-13
    assert rel_l2(got, r.y) < 1e-11
    ck = read_checkpoint(path)
    assert ck["history"] == 0 and ck["dens"] is None and len(ck["arrays"]) == 1


def test_plane_size_limits(lise):
    """Planes beyond the plane kernel's capacity are refused with UNSUPPORTED; the largest
    supported shapes run (64 x 64 FP64 on the register-FFT path, 50 x 50 FP64 and
    80 x 50 FP32 on the LDS path)."""
    fn64 = wl.Functional(ncomp=2, mu_up=0.5, mu_dn=0.5, beta=0.37, g=1.0)
    fn32 = wl.Functional(ncomp=2, mu_up=0.5, mu_dn=0.5, beta=0.37, g=1.0, precision=wl.FP32)
    for (nx, ny, nz), fn in (((80, 80, 4), fn64), ((80, 60, 2), fn32)):
        say(f"unsupported plane {nx}x{ny}x{nz} precision {fn.precision}")
        with pytest.raises(lise.LiseError, match="UNSUPPORTED"):
            lise.Context(wl.Lattice(nx, ny, nz, 1.0), 2, fn)
    for (nx, ny, nz), fn in (((64, 64, 4), fn64), ((50, 50, 2), fn64), ((80, 50, 2), fn32)):
        lat = wl.Lattice(nx, ny, nz, 1.0)
        say(f"largest planes {nx}x{ny}x{nz} precision {fn.precision}: apply H vs oracle")
        psi = random_state(lat, 2, 2, seed=nx + ny)
        ctx = lise.Context(lat, 2, fn)
        ctx.set_qpwf(0, psi)
        got = ctx.apply_h(0, 2)
        n, k = ctx.densities()
        ctx.close()
        n0, k0 = oracle.densities(psi, fn)
        V, D = oracle.potentials(n0, k0, lat, fn, 0.0)
        ref = oracle.apply_h(psi, V, D, lat, fn)
        tol = 1e-12 if fn.precision == wl.FP64 else 3e-6
        assert rel_max(got, ref) < tol


def test_checkpoint_with_options_continues_bitwise(lise, tmp_path):
    """Phase removal and the regularised coupling together, on the bf16x3 MFMA form (C = 4,
    16^3): save with history, reload, continue bit for bit."""
    w = wl.config4(M=12, n=16, precision=wl.FP32_MFMA)
    w.functional.remove_phase = 1
    w.functional.regularize = 1
    path = str(tmp_path / "opts.ckpt")
    say("checkpoint MFMA C=4 with phase removal and g_eff: 5 steps, save, 6 more; reload, 6")
    a = lise.Context(w.lattice, w.M, w.functional)
    a.set_qpwf(0, w.qpwfs())
    a.step(w.dt, 5)
    a.save(path)
    a.step(w.dt, 6)
    ya, ta = a.get_qpwf(0, w.M), a.time()
    a.close()
    b = lise.Context(w.lattice, w.M, w.functional)
    b.load(path)
    b.step(w.dt, 6)
    yb, tb = b.get_qpwf(0, w.M), b.time()
    b.close()
    assert ta == tb and np.array_equal(ya, yb)


def test_kick_and_current_fp32_four_components(lise):
    """FP32 C = 4 (16^3): kick, then the current of Eq. (j) against the oracle's of the
    kicked FP64 state (FP32 rounding of the state only)."""
    w = wl.config4(M=12, n=16, precision=wl.FP32)
    lat = w.lattice
    p = np.array([0.0, 2 * np.pi / (lat.ny * lat.a), 0.0])
    chi = lattice_chi(lat, p, seed=9, amp=0.2)
    say("FP32 C=4 16^3: kick and current")
    ctx = lise.Context(lat, w.M, w.functional)
    ctx.set_qpwf(0, w.qpwfs())
    ctx.kick(chi)
    j = ctx.current()
    obs = ctx.observables()
    ctx.close()
    k = oracle.kick(w.qpwfs(), chi, w.functional)
    jr = oracle.current_density(k, lat, w.functional)
    o = oracle.observables(k, lat, w.functional, 0.0)
    e = rel_l2(j, jr)
    say(f"  j rel L2 {e:.3e}, v_cm {obs['v_cm']} vs {o['v_cm']}")
    assert e < 1e-5
    assert np.allclose(obs["v_cm"], o["v_cm"], rtol=1e-5, atol=1e-9)


def test_checkpoint_errors(lise, tmp_path):
    w = wl.config1(M=16)
    path = str(tmp_path / "e.ckpt")
    c = lise.Context(w.lattice, w.M, w.functional)
    c.set_qpwf(0, w.qpwfs())
    with pytest.raises(lise.LiseError, match="STATE"):
        c.save(path, with_history=True)          # no history yet
    c.save(path, with_history=False)
    c.close()
    other = lise.Context(w.lattice, w.M + 1, w.functional)
    with pytest.raises(lise.LiseError, match="ARG"):
        other.load(path)                          # M differs
    with pytest.raises(lise.LiseError, match="ARG"):
        other.load(str(tmp_path / "missing.ckpt"))
    other.close()


def test_autotune_runs_and_keeps_invariants(lise):
    w = wl.config2(M=64, n=16)
    say("autotune 16^3 M=64")
    ctx = lise.Context(w.lattice, w.M, w.functional)
    ctx.set_qpwf(0, w.qpwfs())
    t = ctx.autotune(w.dt, 1)
    assert t["jgroup"] in (2, 4, 8, 16, 32, 64, 128, 256) and t["chunk_qpwf"] >= 1
    assert t["z_lanes"] in (0, 2, 4) and t["single_pass"] in (-1, 0, 1) and t["z_dense"] in (-1, 0, 1)
    ctx.step(w.dt, 4)
    o = ctx.observables()
    assert o["norm_drift_max"] < 1e-10
    ctx.close()


def test_deterministic_repeats(lise):
    w = wl.config2(M=24, n=16, steps=10)
    psi = w.qpwfs()
    outs = []
    for _ in range(2):
        say("determinism 16^3 M=24, 8 steps")
        ctx = lise.Context(w.lattice, w.M, w.functional)
        ctx.set_tuning(chunk_qpwf=10, jgroup=4)
        ctx.set_qpwf(0, psi)
        ctx.step(w.dt, 8)
        outs.append((ctx.get_qpwf(0, w.M), ctx.densities()[0]))
        ctx.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("case", ["8c_single_pass", "32c_in_kernel_z"])
def test_time_reversal(lise, case):
    """40 ABM steps forward and 40 back (dt -> -dt) return to the initial qpwfs: the 8^3
    single-pass path and the 32^3 FP64 default path (z-term inside the plane kernel;
    the external well's ramp depends on t only, so the backward run retraces it)."""
    w, dt = (wl.config1(M=128), 0.004) if case == "8c_single_pass" else (wl.config2(M=8), 0.002)
    psi = w.qpwfs()
    say(f"time reversal {w.name}: 40 forward, 40 backward, dt {dt}")
    ctx = lise.Context(w.lattice, w.M, w.functional)
    ctx.set_qpwf(0, psi)
    ctx.step(dt, 40)
    ctx.step(-dt, 40)
    got = ctx.get_qpwf(0, w.M)
    t, _ = ctx.time()
    ctx.close()
    assert abs(t) < 1e-13
    assert rel_max(got, psi) < 1e-6


def test_error_paths(lise):
    lat = wl.Lattice(8, 8, 8, 1.0)
    fn = wl.Functional(ncomp=2)
    ctx = lise.Context(lat, 4, fn)
    with pytest.raises(lise.LiseError, match="STATE"):
        ctx.step(0.01, 1)            # qpwfs not set
    with pytest.raises(lise.LiseError, match="ARG"):
        ctx.set_qpwf(3, np.zeros((2, 2, 8, 8, 8), dtype=complex))
    with pytest.raises(lise.LiseError, match="ARG"):
        ctx.step(0.0, 1)
    ctx.set_qpwf(0, random_state(lat, 4, 2, 1) * np.nan)
    with pytest.raises(lise.LiseError, match="NAN"):
        ctx.step(0.01, 1)
    ctx.close()
