"""Pins of the trivial-phase removal of Eq. (sp_en) in the oracle."""
import math

import numpy as np
from scipy.integrate import solve_ivp

import oracle
import workloads as wl
from test_oracle_dynamics import uniform_case, zero_d_fields, zero_d_h
from test_oracle_operators import dense_bdg


def test_eta_of_bdg_eigenvectors_is_the_eigenvalue():
    """For eigenvectors of a dense BdG matrix (built without the oracle's FFT), the
    quasiparticle energy <psi|H|psi> is the eigenvalue."""
    lat = wl.Lattice(4, 4, 2, 1.0)
    for ncomp in (2, 4):
        fn = wl.Functional(ncomp=ncomp, mu_up=0.6, mu_dn=0.4 if ncomp == 4 else 0.6)
        rng = np.random.default_rng(7)
        shp = (lat.nz, lat.ny, lat.nx)
        V = 0.3 * rng.standard_normal(shp)
        D = 0.4 + 0.2 * (rng.standard_normal(shp) + 1j * rng.standard_normal(shp))
        H4 = dense_bdg(lat, fn, V, D)
        N = lat.n
        H = H4[np.ix_(np.r_[0:N, 3 * N:4 * N], np.r_[0:N, 3 * N:4 * N])] if ncomp == 2 else H4
        e, U = np.linalg.eigh(H)
        sel = np.r_[0:3, len(e) - 3:len(e)]
        vecs = U[:, sel]
        psi = np.stack([vecs[c * N:(c + 1) * N].T.reshape(-1, *shp) for c in range(ncomp)], axis=1)
        psi = psi / lat.a ** 1.5
        eta = oracle.quasiparticle_energies(psi, V, D, lat, fn)
        assert np.allclose(eta, e[sel], rtol=0, atol=1e-12)


def frozen_case():
    lat = wl.Lattice(4, 4, 6, 1.0)
    U0, D0, mu = 0.15, 0.4 * np.exp(-0.3j), 0.7
    fn = wl.Functional(ncomp=2, mu_up=mu, mu_dn=mu, frozen=1, U0=U0, Delta0=D0, g=1.0, remove_phase=1)
    idx = wl.k_order(lat)[:20]
    pw = wl.plane_waves(lat, idx)
    k2 = np.sum(wl.k_of(lat, idx) ** 2, axis=1)
    blocks = []
    for j in range(20):
        xi = 0.5 * k2[j] + U0 - mu
        blocks.append(np.array([[xi, D0], [np.conj(D0), -xi]]))
    return lat, fn, pw, blocks


def test_frozen_eigenvectors_are_stationary():
    """A qpwf that is an eigenvector of the frozen H has H psi = eta psi: with the phase
    removed its derivative vanishes and it stays put (without removal it rotates)."""
    lat, fn, pw, blocks = frozen_case()
    ab = np.array([np.linalg.eigh(Hk)[1][:, 1] for Hk in blocks])
    psi = ab[:, :, None, None, None] * pw[:, None]
    ev = oracle.Evolver(lat, fn, psi)
    ev.step(0.004, 60)
    assert np.max(np.abs(ev.y - psi)) < 1e-13
    fn.remove_phase = 0
    ev = oracle.Evolver(lat, fn, psi)
    ev.step(0.004, 60)
    assert np.max(np.abs(ev.y - psi)) > 1e-3


def test_frozen_superposition_gains_exactly_the_removed_phase():
    """Frozen H: <psi|H|psi> is constant, so psi_k(t) = exp(+i eta_k t) exp(-i H_k t) psi_k(0)."""
    lat, fn, pw, blocks = frozen_case()
    rng = np.random.default_rng(11)
    ab = rng.standard_normal((20, 2)) + 1j * rng.standard_normal((20, 2))
    ab /= np.linalg.norm(ab, axis=1, keepdims=True)
    psi = ab[:, :, None, None, None] * pw[:, None]
    ev = oracle.Evolver(lat, fn, psi)
    ev.step(0.004, 100)
    t = ev.t
    for j, Hk in enumerate(blocks):
        eta = float(np.real(np.conj(ab[j]) @ Hk @ ab[j]))
        E = math.sqrt(Hk[0, 0].real ** 2 + abs(Hk[0, 1]) ** 2)
        Ut = math.cos(E * t) * np.eye(2) - 1j * math.sin(E * t) * Hk / E
        exact = np.exp(1j * eta * t) * (Ut @ ab[j])
        got = ev.y[j] / pw[j][None]
        assert np.max(np.abs(got - exact[:, None, None, None])) < 1e-9


def zero_d_eta(fn, k2, Vbox, x):
    """eta_k = x_k^dagger H_k x_k of the 0-D momentum-space system."""
    xi, D = zero_d_h(fn, k2, *zero_d_fields(fn, Vbox, x[0], x[1]))
    return zero_d_eta_fields(xi, D, x)


def zero_d_eta_fields(xi, D, x):
    hx = np.stack([xi * x[0] + D * x[1], np.conj(D) * x[0] - xi * x[1]])
    return np.real(np.conj(x[0]) * hx[0] + np.conj(x[1]) * hx[1])


def zero_d_scheme_phase_removed(fn, k2, Vbox, a, b, dt, nsteps):
    """Start-up + ABM on the 0-D system with f(x) = -i (H - eta) x, written out per momentum."""
    def apply(xi, D, x, eta):
        return np.stack([xi * x[0] + D * x[1] - eta * x[0], np.conj(D) * x[0] - xi * x[1] - eta * x[1]])

    def taylor(x, xi, D):
        eta = zero_d_eta_fields(xi, D, x)
        acc, term = x.copy(), x
        for q in range(1, 5):
            term = (-1j * dt / q) * apply(xi, D, term, eta)
            acc = acc + term
        return acc

    def f(x):
        xi, D = zero_d_h(fn, k2, *zero_d_fields(fn, Vbox, x[0], x[1]))
        return -1j * apply(xi, D, x, zero_d_eta_fields(xi, D, x))

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


def test_uniform_phase_removed_matches_zero_d_replica_to_roundoff():
    lat, fn, psi, k2, pw, a0, b0 = uniform_case()
    fn.remove_phase = 1
    dt, nsteps = 0.005, 60
    ev = oracle.Evolver(lat, fn, psi)
    ev.step(dt, nsteps)
    ab = zero_d_scheme_phase_removed(fn, k2, lat.n, a0, b0, dt, nsteps)
    ref = ab.T[:, :, None, None, None] * pw[:, None]
    assert np.max(np.abs(ev.y - ref)) / np.max(np.abs(ref)) < 1e-12


def test_phase_removal_leaves_densities_of_the_exact_flow_unchanged():
    """DOP853 on the 0-D system with and without the eta shift: each momentum's
    (a, b) differ by a phase only, so n and kappa agree; the dropped phase is
    the integral of eta."""
    lat, fn, psi, k2, pw, a0, b0 = uniform_case()
    M = len(k2)
    Vbox = lat.n

    def rhs(remove):
        def f(t, y):
            a = y[:M] + 1j * y[M:2 * M]
            b = y[2 * M:3 * M] + 1j * y[3 * M:4 * M]
            xi, D = zero_d_h(fn, k2, *zero_d_fields(fn, Vbox, a, b))
            eta = zero_d_eta_fields(xi, D, np.stack([a, b])) if remove else 0.0
            da = -1j * (xi * a + D * b - eta * a)
            db = -1j * (np.conj(D) * a - xi * b - eta * b)
            out = [da.real, da.imag, db.real, db.imag]
            if remove:
                out.append(eta)          # accumulates the integral of eta_k
            return np.concatenate(out)
        return f

    y0 = np.concatenate([a0.real, a0.imag, b0.real, b0.imag])
    T = 0.6
    s0 = solve_ivp(rhs(False), (0, T), y0, method="DOP853", rtol=1e-12, atol=1e-14).y[:, -1]
    s1 = solve_ivp(rhs(True), (0, T), np.concatenate([y0, np.zeros(M)]), method="DOP853",
                   rtol=1e-12, atol=1e-14).y[:, -1]
    a_0, b_0 = s0[:M] + 1j * s0[M:2 * M], s0[2 * M:3 * M] + 1j * s0[3 * M:]
    a_1, b_1 = s1[:M] + 1j * s1[M:2 * M], s1[2 * M:3 * M] + 1j * s1[3 * M:4 * M]
    theta = s1[4 * M:]
    assert np.max(np.abs(zero_d_fields(fn, Vbox, a_0, b_0)[0] - zero_d_fields(fn, Vbox, a_1, b_1)[0])) < 1e-10
    assert np.max(np.abs(zero_d_fields(fn, Vbox, a_0, b_0)[1] - zero_d_fields(fn, Vbox, a_1, b_1)[1])) < 1e-10
    assert np.max(np.abs(np.exp(1j * theta) * a_0 - a_1)) < 1e-9
    assert np.max(np.abs(np.exp(1j * theta) * b_0 - b_1)) < 1e-9
    assert np.max(np.abs(theta)) > 1e-2      # the phase is not trivially zero


def test_phase_removal_keeps_densities_within_integration_error():
    """3D self-consistent run (config-1 recipe, noisy): with and without phase removal
    the densities differ by far less than they change over the run."""
    w = wl.config1(M=64)
    psi = w.qpwfs()
    runs = []
    for rp in (0, 1):
        w.functional.remove_phase = rp
        ev = oracle.Evolver(w.lattice, w.functional, psi)
        ev.step(w.dt, 30)
        runs.append(oracle.densities(ev.y, w.functional))
    n0, _ = oracle.densities(psi, w.functional)
    d_rm = np.max(np.abs(runs[0][0] - runs[1][0]))
    d_k = np.max(np.abs(runs[0][1] - runs[1][1]))
    change = np.max(np.abs(runs[0][0] - n0))
    assert d_rm < 1e-6 * np.max(n0) and d_k < 1e-6 * np.max(np.abs(runs[0][1]))
    assert change > 1e3 * d_rm
