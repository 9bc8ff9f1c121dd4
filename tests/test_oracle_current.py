"""Pins of the spectral gradient, the current density of Eq. (j), the boost of
Eq. (kick) and the centre-of-mass velocity of Eq. (vel) in the oracle."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


@pytest.mark.parametrize("n,a", [(8, 1.0), (9, 0.7), (12, 1.3)])
def test_derivative_of_plane_waves(n, a):
    """D e^{i k_m x} = i k_m e^{i k_m x} for every mode but the N/2 mode of an even
    axis, whose derivative the paper sets to zero."""
    D = oracle.derivative_matrix(n, a)
    x = np.arange(n) * a
    L = n * a
    for m in range(n):
        ms = m if 2 * m < n else m - n
        k = 2 * math.pi * ms / L
        f = np.exp(1j * k * x)
        want = np.zeros(n) if 2 * m == n else 1j * k * f
        assert np.max(np.abs(D @ f - want)) < 1e-12


def test_derivative_of_nyquist_real_function_is_real():
    """cos(pi x / a) on an even axis: the zeroed N/2 mode keeps its derivative real (zero)."""
    n, a = 8, 1.0
    f = np.cos(math.pi * np.arange(n))
    d = oracle.derivative_matrix(n, a) @ f
    assert np.max(np.abs(d)) < 1e-13


def band_limited(lat, M, C, seed, margin=2):
    """Random qpwfs made of modes at least `margin` indices inside the zone on every axis."""
    rng = np.random.default_rng(seed)
    out = np.zeros((M, C, lat.nz, lat.ny, lat.nx), complex)
    lim = [n // 2 - margin for n in (lat.nx, lat.ny, lat.nz)]
    for mx in range(-lim[0], lim[0] + 1):
        for my in range(-lim[1], lim[1] + 1):
            for mz in range(-lim[2], lim[2] + 1):
                pw = wl.plane_waves(lat, np.array([[mx, my, mz]]))[0]
                c = rng.standard_normal((M, C)) + 1j * rng.standard_normal((M, C))
                out += c[:, :, None, None, None] * pw[None, None]
    return out / np.sqrt(np.sum(np.abs(out) ** 2, axis=(1, 2, 3, 4), keepdims=True) * lat.a ** 3)


@pytest.mark.parametrize("ncomp", [2, 4])
def test_total_current_by_parseval(ncomp):
    """a^3 sum_r j = -w a^3 / N sum_j sum_m k_m |v^_j(m)|^2 (k-space route, numpy FFT,
    the N/2 momentum of even axes counted as zero)."""
    lat = wl.Lattice(6, 8, 5, 0.9)
    fn = wl.Functional(ncomp=ncomp, w=2.0 if ncomp == 2 else 1.0)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((4, ncomp, 5, 8, 6)) + 1j * rng.standard_normal((4, ncomp, 5, 8, 6))
    j = oracle.current_density(psi, lat, fn)
    P = lat.a ** 3 * j.reshape(3, -1).sum(axis=1)
    vs = [1] if ncomp == 2 else [2, 3]
    wt = fn.w if ncomp == 2 else 1.0

    def kaxis(n):
        k = 2 * np.pi * np.fft.fftfreq(n, d=lat.a)
        if n % 2 == 0:
            k[n // 2] = 0.0
        return k
    kx, ky, kz = kaxis(lat.nx), kaxis(lat.ny), kaxis(lat.nz)
    ref = np.zeros(3)
    for c in vs:
        p2 = np.abs(np.fft.fftn(psi[:, c], axes=(1, 2, 3))) ** 2
        ref[0] -= wt * np.sum(p2 * kx[None, None, None, :])
        ref[1] -= wt * np.sum(p2 * ky[None, None, :, None])
        ref[2] -= wt * np.sum(p2 * kz[None, :, None, None])
    ref *= lat.a ** 3 / lat.n
    assert np.allclose(P, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("ncomp", [2, 4])
def test_kick_adds_n_grad_chi_to_the_current(ncomp):
    """chi = p.r with p on the momentum grid and band-limited qpwfs: j' = j + n p exactly,
    n and |kappa| unchanged, kappa' = exp(2 i chi) kappa."""
    lat = wl.Lattice(8, 8, 8, 1.0)
    fn = wl.Functional(ncomp=ncomp, w=2.0 if ncomp == 2 else 1.0)
    psi = band_limited(lat, 3, ncomp, seed=5)
    p = 2 * np.pi / (lat.n ** (1 / 3) * lat.a) * np.array([1.0, -1.0, 0.0])
    x = np.arange(8) * lat.a
    chi = p[0] * x[None, None, :] + p[1] * x[None, :, None] + p[2] * x[:, None, None]
    kicked = oracle.kick(psi, chi, fn)
    n0, k0 = oracle.densities(psi, fn)
    n1, k1 = oracle.densities(kicked, fn)
    assert np.allclose(n1, n0, atol=1e-15)
    assert np.allclose(k1, np.exp(2j * chi) * k0, atol=1e-15)
    j0 = oracle.current_density(psi, lat, fn)
    j1 = oracle.current_density(kicked, lat, fn)
    for ax in range(3):
        assert np.max(np.abs(j1[ax] - j0[ax] - p[ax] * n0)) < 1e-12


def test_boosted_uniform_state_moves_at_p():
    """A kicked uniform BCS state (closed shells, no external field) carries j = p n and
    v_cm = p while it evolves; its n and |kappa| follow the unkicked evolution
    (Galilean covariance)."""
    lat = wl.Lattice(8, 8, 8, 1.0)
    fn = wl.Functional(ncomp=2, mu_up=0.8, mu_dn=0.8, beta=0.37, g=2.0, w=2.0)
    M = 33                                  # shells |m|^2 <= 2: 1 + 6 + 12 + 8 + 6 = 33
    psi = wl.uniform_bcs(lat, fn, M, 0.45, 0.8)(0, M)
    p = np.array([2 * np.pi / 8, 0.0, 0.0])
    x = np.arange(8) * lat.a
    chi = p[0] * x[None, None, :] + 0 * x[:, None, None]
    kicked = oracle.kick(psi, chi, fn)
    o = oracle.observables(kicked, lat, fn, 0.0)
    assert np.allclose(o["v_cm"], p, atol=1e-13)
    a = oracle.Evolver(lat, fn, psi)
    b = oracle.Evolver(lat, fn, kicked)
    a.step(0.005, 40)
    b.step(0.005, 40)
    ob = oracle.observables(b.y, lat, fn, b.t)
    assert np.allclose(ob["v_cm"], p, atol=1e-10)
    na, ka = oracle.densities(a.y, fn)
    nb, kb = oracle.densities(b.y, fn)
    jb = oracle.current_density(b.y, lat, fn)
    assert np.max(np.abs(jb[0] - p[0] * nb)) < 1e-10 and np.max(np.abs(jb[1:])) < 1e-10
    assert np.max(np.abs(nb - na)) < 1e-8 * np.max(na)
    assert np.max(np.abs(np.abs(kb) - np.abs(ka))) < 1e-8 * np.max(np.abs(ka))
    # the unkicked state changes over the run: the comparison is not vacuous
    n0, k0 = oracle.densities(psi, fn)
    assert np.max(np.abs(np.abs(ka) - np.abs(k0))) > 1e-5
