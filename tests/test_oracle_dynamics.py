"""Oracle pins: dynamics with closed forms, an independent 0-D reduction, invariants."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import workloads as wl


def signed(n):
    return np.array([i if 2 * i < n else i - n for i in range(n)])


def scalar_abm_run(lam, dt, nsteps):
    """Start-up + ABM for the scalar ODE y' = -i lam y, y(0) = 1, written out here.

    Start-up: y_{s+1} = sum_{q<=4} (-i lam dt)^q / q! y_s (H does not change for a
    free plane wave, so predictor and corrector coincide); then abm_update.
    """
    z = -1j * lam * dt
    P = sum(z ** q / math.factorial(q) for q in range(5))
    ys = [1.0 + 0j]
    for _ in range(3):
        ys.append(P * ys[-1])
    f = lambda y: -1j * lam * y
    y_n, y_nm1 = ys[3], ys[2]
    prev = [f(ys[2]), f(ys[1]), f(ys[0])]
    d = 0j
    for _ in range(nsteps):
        dyn = f(y_n)
        y_next, d = oracle.abm_update(y_n, y_nm1, (dyn, prev[0], prev[1], prev[2]), d, f, dt)
        prev = [dyn, prev[0], prev[1]]
        y_nm1, y_n = y_n, y_next
    return y_n


def test_free_plane_wave_phase():
    """u = e^{ik.r}/sqrt(V), v = 0: n = kappa = 0, so u(t) = exp(-i k^2 t / 2) u(0)."""
    lat = wl.Lattice(8, 8, 8, 1.0)
    fn = wl.Functional(ncomp=2, mu_up=0.0, mu_dn=0.0, beta=0.37, g=1.5, w=2.0)
    idx = np.array([[0, 0, 0], [1, 0, 0], [1, 2, -3], [-4, -4, -4], [3, -2, 1]])
    pw = wl.plane_waves(lat, idx)
    psi = np.zeros((len(idx), 2, 8, 8, 8), dtype=complex)
    psi[:, 0] = pw
    dt, nsteps = 0.005, 60
    ev = oracle.Evolver(lat, fn, psi)
    ev.step(dt, nsteps)
    t = (nsteps + 3) * dt
    assert abs(ev.t - t) < 1e-14
    k2 = np.sum(wl.k_of(lat, idx) ** 2, axis=1)
    for j in range(len(idx)):
        lam = 0.5 * k2[j]
        rec = scalar_abm_run(lam, dt, nsteps)
        # the 3D solver equals the scalar recurrence to round-off ...
        assert np.max(np.abs(ev.y[j, 0] - rec * pw[j])) < 1e-13
        assert np.max(np.abs(ev.y[j, 1])) == 0.0
        # ... and the exact phase within the integrator's truncation error
        z = lam * dt
        bound = 2 * (3 * z ** 5 / 120 + nsteps * 2e-9 * (z / 0.074) ** 6) + 1e-13
        assert abs(rec - np.exp(-1j * lam * t)) < bound


def test_frozen_uniform_bcs_closed_form():
    """Frozen U0, Delta0: each k evolves by exp(-i H_k t) = cos(E t) - i sin(E t) H_k / E."""
    lat = wl.Lattice(4, 4, 6, 1.0)
    U0, D0, mu = 0.15, 0.4 * np.exp(-0.3j), 0.7
    fn = wl.Functional(ncomp=2, mu_up=mu, mu_dn=mu, frozen=1, U0=U0, Delta0=D0, g=1.0)
    idx = wl.k_order(lat)[:20]
    pw = wl.plane_waves(lat, idx)
    rng = np.random.default_rng(11)
    ab = rng.standard_normal((20, 2)) + 1j * rng.standard_normal((20, 2))
    ab /= np.linalg.norm(ab, axis=1, keepdims=True)
    psi = ab[:, :, None, None, None] * pw[:, None]
    dt, nsteps = 0.004, 100
    ev = oracle.Evolver(lat, fn, psi)
    ev.step(dt, nsteps)
    t = ev.t
    k2 = np.sum(wl.k_of(lat, idx) ** 2, axis=1)
    for j in range(20):
        xi = 0.5 * k2[j] + U0 - mu
        Hk = np.array([[xi, D0], [np.conj(D0), -xi]])
        E = math.sqrt(xi * xi + abs(D0) ** 2)
        Ut = math.cos(E * t) * np.eye(2) - 1j * math.sin(E * t) * Hk / E
        exact = Ut @ ab[j]
        got = ev.y[j] / pw[j][None]
        assert np.max(np.abs(got - exact[:, None, None, None])) < 1e-9


def zero_d_fields(fn, Vbox, a, b):
    n = fn.w * np.sum(np.abs(b) ** 2) / Vbox
    kap = 0.5 * fn.w * np.sum(np.conj(b) * a) / Vbox
    return n, kap


def zero_d_h(fn, k2, n, kap):
    """Per-momentum 2x2 blocks [[xi, Delta], [Delta^*, -xi]], xi = k^2/2 + beta n^{2/3} - mu."""
    xi = 0.5 * k2 + fn.beta * np.cbrt(n) ** 2 - fn.mu_up
    D = -fn.g * kap
    return xi, D


def zero_d_rhs(fn, k2, Vbox):
    M = len(k2)

    def f(t, y):
        a = y[:M] + 1j * y[M:2 * M]
        b = y[2 * M:3 * M] + 1j * y[3 * M:]
        xi, D = zero_d_h(fn, k2, *zero_d_fields(fn, Vbox, a, b))
        da = -1j * (xi * a + D * b)
        db = -1j * (np.conj(D) * a - xi * b)
        return np.concatenate([da.real, da.imag, db.real, db.imag])
    return f


def zero_d_same_scheme(fn, k2, Vbox, a, b, dt, nsteps):
    """The same start-up and ABM applied to the 0-D system, written out per momentum."""
    def apply(xi, D, x):
        return np.stack([xi * x[0] + D * x[1], np.conj(D) * x[0] - xi * x[1]])

    def taylor(x, xi, D):
        acc, term = x.copy(), x
        for q in range(1, 5):
            term = (-1j * dt / q) * apply(xi, D, term)
            acc = acc + term
        return acc

    def f(x):
        return -1j * apply(*zero_d_h(fn, k2, *zero_d_fields(fn, Vbox, x[0], x[1])), x)

    ys = [np.stack([a, b])]
    ds = []
    for _ in range(3):
        x = ys[-1]
        n0, k0 = zero_d_fields(fn, Vbox, x[0], x[1])
        ds.append(f(x))
        pre = taylor(x, *zero_d_h(fn, k2, n0, k0))
        n1, k1 = zero_d_fields(fn, Vbox, pre[0], pre[1])
        ys.append(taylor(x, *zero_d_h(fn, k2, 0.5 * (n0 + n1), 0.5 * (k0 + k1))))
    y_n, y_nm1 = ys[3], ys[2]
    prev = [ds[2], ds[1], ds[0]]
    d = np.zeros_like(y_n)
    for _ in range(nsteps):
        dyn = f(y_n)
        y_next, d = oracle.abm_update(y_n, y_nm1, (dyn, prev[0], prev[1], prev[2]), d, f, dt)
        prev = [dyn, prev[0], prev[1]]
        y_nm1, y_n = y_n, y_next
    return y_n


def uniform_case():
    lat = wl.Lattice(4, 4, 4, 1.0)
    fn = wl.Functional(ncomp=2, mu_up=0.8, mu_dn=0.8, beta=0.37, g=2.0, w=2.0)
    M = 40
    psi = wl.uniform_bcs(lat, fn, M, 0.45, 0.8)(0, M)
    idx = wl.k_order(lat)[:M]
    k2 = np.sum(wl.k_of(lat, idx) ** 2, axis=1)
    pw = wl.plane_waves(lat, idx)
    a0 = psi[:, 0, 0, 0, 0] / pw[:, 0, 0, 0]
    b0 = psi[:, 1, 0, 0, 0] / pw[:, 0, 0, 0]
    return lat, fn, psi, k2, pw, a0, b0


def test_self_consistent_uniform_matches_zero_d_replica_to_roundoff():
    """Uniform states stay uniform; the 3D solver equals the same scheme run on the
    M coupled 2x2 momentum-space systems (no FFT, no lattice) to round-off."""
    lat, fn, psi, k2, pw, a0, b0 = uniform_case()
    dt, nsteps = 0.005, 100
    ev = oracle.Evolver(lat, fn, psi)
    ev.step(dt, nsteps)
    ab = zero_d_same_scheme(fn, k2, lat.n, a0, b0, dt, nsteps)
    ref = ab.T[:, :, None, None, None] * pw[:, None]
    assert np.max(np.abs(ev.y - ref)) / np.max(np.abs(ref)) < 1e-12


def test_self_consistent_uniform_converges_to_dop853():
    """Against SciPy's DOP853 (rtol 1e-12) the error falls with dt at least as dt^2."""
    lat, fn, psi, k2, pw, a0, b0 = uniform_case()
    T = 0.5
    errs = []
    for dt in (0.01, 0.005):
        nsteps = int(round(T / dt)) - 3
        ab = zero_d_same_scheme(fn, k2, lat.n, a0, b0, dt, nsteps)
        y0 = np.concatenate([a0.real, a0.imag, b0.real, b0.imag])
        sol = solve_ivp(zero_d_rhs(fn, k2, lat.n), (0.0, T), y0, method="DOP853",
                        rtol=1e-12, atol=1e-14)
        M = len(k2)
        y = sol.y[:, -1]
        ref = np.stack([y[:M] + 1j * y[M:2 * M], y[2 * M:3 * M] + 1j * y[3 * M:]])
        errs.append(np.max(np.abs(ab - ref)))
    assert errs[1] < 1e-6
    assert errs[0] / errs[1] > 4


def test_uniform_bcs_density_closed_form_and_loops():
    lat = wl.Lattice(4, 4, 4, 1.0)
    fn = wl.Functional(ncomp=2, w=2.0)
    M = 33
    psi = wl.uniform_bcs(lat, fn, M, 0.3, 0.5)(0, M)
    n, kap = oracle.densities(psi, fn)
    idx = wl.k_order(lat)[:M]
    k2 = np.sum(wl.k_of(lat, idx) ** 2, axis=1)
    u, v = wl.bcs_uv(0.5 * k2 - 0.5, 0.3)
    Vbox = lat.n
    assert np.allclose(n, 2.0 * np.sum(v * v) / Vbox, atol=1e-14, rtol=0)
    assert np.allclose(kap, np.sum(u * v) / Vbox, atol=1e-14, rtol=0)
    # brute-force loop sum at a few points
    for r in [(0, 0, 0), (1, 2, 3), (3, 3, 0)]:
        ns = 0.0
        ks = 0j
        for j in range(M):
            ns += fn.w * abs(psi[j, 1][r]) ** 2
            ks += 0.5 * fn.w * np.conj(psi[j, 1][r]) * psi[j, 0][r]
        assert abs(ns - n[r]) < 1e-15 and abs(ks - kap[r]) < 1e-15


def test_four_component_kappa_matches_paper_for_spin_symmetric_sets():
    """For block A (u_up=u, v_dn=v) and block B (u_dn=u, v_up=-v) on the same momenta,
    the singlet average equals Eq. (nu_t), sum v_dn^* u_up."""
    lat = wl.Lattice(4, 4, 4, 1.0)
    fn = wl.Functional(ncomp=4, w=1.0)
    rng = np.random.default_rng(3)
    M = 6
    u = rng.standard_normal((M, 4, 4, 4)) + 1j * rng.standard_normal((M, 4, 4, 4))
    v = rng.standard_normal((M, 4, 4, 4)) + 1j * rng.standard_normal((M, 4, 4, 4))
    psi = np.zeros((2 * M, 4, 4, 4, 4), dtype=complex)
    psi[:M, 0], psi[:M, 3] = u, v
    psi[M:, 1], psi[M:, 2] = u, -v
    n, kap = oracle.densities(psi, fn)
    paper = np.sum(np.conj(psi[:, 3]) * psi[:, 0], axis=0)
    assert np.max(np.abs(kap - paper)) < 1e-13
    assert np.max(np.abs(n - np.sum(np.abs(v) ** 2, axis=0) * 2)) < 1e-12


def conserved_run(M_copies=2, dt=0.005, nsteps=60, eps=1e-2):
    lat = wl.Lattice(4, 4, 4, 1.0)
    fn = wl.Functional(ncomp=2, mu_up=1.0, mu_dn=1.0, beta=0.37, g=1.5, w=1.0)
    M = 64 * M_copies
    psi = wl.uniform_bcs(lat, fn, M, 0.5, 1.0, copies=M_copies, eps=eps, seed=2)(0, M)
    ev = oracle.Evolver(lat, fn, psi)
    return lat, fn, psi, ev


def test_invariants_noisy_set():
    """N, norms and the Gram matrix are exact invariants of the flow (H is Hermitian and
    shared by all qpwfs): their drift is the integrator's, O(dt^4)."""
    drifts = []
    for dt in (0.01, 0.005):
        lat, fn, psi, ev = conserved_run(dt=dt)
        o0 = oracle.observables(psi, lat, fn, 0.0)
        ev.step(dt, int(round(0.3 / dt)))
        o1 = oracle.observables(ev.y, lat, fn, ev.t)
        dS = np.max(np.abs(oracle.gram(ev.y, lat) - oracle.gram(psi, lat)))
        drifts.append((abs(o1["N"] - o0["N"]), dS, np.max(np.abs(o1["norms"] - o0["norms"]))))
    (n1, s1, m1), (n2, s2, m2) = drifts
    assert n2 < 2e-6 and s2 < 2e-6 and m2 < 2e-6
    assert n1 / n2 > 8 and s1 / s2 > 8


def test_energy_drift_of_vacuum_is_integrator_error():
    """For a complete quasiparticle vacuum E is an exact invariant; its drift falls as dt^4."""
    from test_oracle_fields import bdg_vacuum
    lat = wl.Lattice(4, 4, 4, 1.0)
    fn = wl.Functional(ncomp=2, mu_up=0.7, mu_dn=0.7, beta=0.37, g=1.5, w=2.0)
    psi = bdg_vacuum(lat, fn, seed=3)
    e0 = oracle.observables(psi, lat, fn, 0.0)["E"]
    drift = []
    for dt in (0.01, 0.005):
        ev = oracle.Evolver(lat, fn, psi)
        ev.step(dt, int(round(0.3 / dt)) - 3)
        drift.append(abs(oracle.observables(ev.y, lat, fn, ev.t)["E"] - e0))
    assert drift[1] < 1e-7 * abs(e0)
    assert drift[0] / drift[1] > 10


def test_time_reversal_returns_initial_state():
    lat, fn, psi, ev = conserved_run(dt=0.004, eps=1e-3)
    ev.step(0.004, 40)
    ev.step(-0.004, 40)
    assert abs(ev.t) < 1e-14
    err = np.max(np.abs(ev.y - psi)) / np.max(np.abs(psi))
    assert err < 1e-6


def test_series_step_orders():
    """Frozen H: the order-4 series has local error O(dt^5) (halving dt: ~32x).
    Self-consistent: the density-averaging predictor-corrector is a midpoint
    rule for the nonlinear part, local error O(dt^3) (halving dt: ~8x)."""
    lat, fn, psi, _ = conserved_run(eps=1e-3)
    frozen = wl.Functional(**{**fn.as_dict(), "frozen": 1, "U0": 0.3, "Delta0": 0.2 + 0.1j})

    def local_err(f, dt):
        one = oracle.series_step(psi, lat, f, 0.0, dt)
        two = psi
        for s in range(16):
            two = oracle.series_step(two, lat, f, s * dt / 16, dt / 16)
        return np.max(np.abs(one - two))
    rf = local_err(frozen, 0.02) / local_err(frozen, 0.01)
    rs = local_err(fn, 0.02) / local_err(fn, 0.01)
    assert rf > 24
    assert 6 < rs < 12
