"""Oracle pins: kinetic operator, DVR matrices, BdG Hamiltonian."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


def plane_wave(lat, n):
    """exp(i k.r) with k from signed integer indices, written out directly."""
    kx = 2 * math.pi * n[0] / (lat.nx * lat.a)
    ky = 2 * math.pi * n[1] / (lat.ny * lat.a)
    kz = 2 * math.pi * n[2] / (lat.nz * lat.a)
    z, y, x = np.meshgrid(np.arange(lat.nz) * lat.a, np.arange(lat.ny) * lat.a,
                          np.arange(lat.nx) * lat.a, indexing="ij")
    return np.exp(1j * (kx * x + ky * y + kz * z)), kx * kx + ky * ky + kz * kz


@pytest.mark.parametrize("dims,a", [((4, 4, 4), 1.0), ((6, 4, 5), 0.7), ((8, 3, 2), 1.3)])
def test_kinetic_plane_wave_eigen(dims, a):
    """T e^{ik.r} = (k^2/2) e^{ik.r} for every lattice momentum (Nyquist kept)."""
    lat = wl.Lattice(*dims, a)
    for nz in range(-(lat.nz // 2), lat.nz - lat.nz // 2):
        for ny in range(-(lat.ny // 2), lat.ny - lat.ny // 2):
            for nx in range(-(lat.nx // 2), lat.nx - lat.nx // 2):
                f, k2 = plane_wave(lat, (nx, ny, nz))
                Tf = oracle.kinetic(f, lat)
                assert np.max(np.abs(Tf - 0.5 * k2 * f)) < 1e-12 * max(1.0, k2)


def dvr_d2(N, a, prefactor):
    """Second-derivative DVR matrix of Eq. (d2) with a chosen off-diagonal prefactor."""
    D = np.zeros((N, N))
    for n in range(N):
        for m in range(N):
            if n == m:
                D[n, m] = -(math.pi ** 2 / (3 * a * a)) * (1 + 2.0 / (N * N))
            else:
                D[n, m] = prefactor * (-1) ** (n - m) * (-1.0) / math.sin(math.pi * (n - m) / N) ** 2
    return D


def dvr_d1(N, a):
    """First-derivative DVR matrix of Eq. (d1)."""
    D = np.zeros((N, N))
    for n in range(N):
        for m in range(N):
            if n != m:
                D[n, m] = (math.pi / (N * a)) * (-1) ** (n - m) / math.tan(math.pi * (n - m) / N)
    return D


@pytest.mark.parametrize("N,a", [(4, 1.0), (6, 0.8), (8, 1.0), (10, 1.25), (32, 1.0)])
def test_kinetic_equals_dvr_second_derivative(N, a):
    """The 1D spectral kinetic operator is -1/2 times Eq. (d2) with prefactor 2 pi^2/(N^2 a^2).

    The printed prefactor pi^2/(2 N^2 a^2) is off by a factor of 4; the test
    records that it does not match.
    """
    lat = wl.Lattice(N, 1, 1, a)
    T = np.zeros((N, N), dtype=complex)
    for m in range(N):
        e = np.zeros((1, 1, N), dtype=complex)
        e[0, 0, m] = 1.0
        T[:, m] = oracle.kinetic(e, lat)[0, 0]
    good = dvr_d2(N, a, 2 * math.pi ** 2 / (N * N * a * a))
    printed = dvr_d2(N, a, math.pi ** 2 / (2 * N * N * a * a))
    assert np.max(np.abs(T + 0.5 * good)) < 1e-12 * np.max(np.abs(good))
    assert np.max(np.abs(T + 0.5 * printed)) > 1e-3


@pytest.mark.parametrize("N,a", [(4, 1.0), (8, 0.9)])
def test_first_derivative_dvr_matches_fft_with_nyquist_zeroed(N, a):
    """Eq. (d1) equals the FFT derivative i k with the -k_{N/2} mode set to zero."""
    k = oracle.wavenumbers(N, a).astype(complex)
    k[N // 2] = 0.0
    W = oracle.dft_matrix(N, -1)
    D = (np.conj(W) @ np.diag(1j * k) @ W) / N
    assert np.max(np.abs(D - dvr_d1(N, a))) < 1e-12 * N


def dense_bdg(lat, fn, V, Delta):
    """The 4N x 4N matrix of Eq. (tdslda) with h = T + V from Eq. (d2) DVR blocks."""
    def d2(N):
        return dvr_d2(N, lat.a, 2 * math.pi ** 2 / (N * N * lat.a * lat.a))
    Ix, Iy, Iz = np.eye(lat.nx), np.eye(lat.ny), np.eye(lat.nz)
    lap = (np.kron(np.kron(Iz, Iy), d2(lat.nx)) + np.kron(np.kron(Iz, d2(lat.ny)), Ix)
           + np.kron(np.kron(d2(lat.nz), Iy), Ix))
    h = -0.5 * lap + np.diag(V.ravel())
    D = np.diag(Delta.ravel())
    Z = np.zeros_like(h)
    I = np.eye(h.shape[0])
    mu_u, mu_d = fn.mu_up, fn.mu_dn
    return np.block([
        [h - mu_u * I, Z, Z, D],
        [Z, h - mu_d * I, -D, Z],
        [Z, -np.conj(D), -np.conj(h) + mu_u * I, Z],
        [np.conj(D), Z, Z, -np.conj(h) + mu_d * I]])


@pytest.mark.parametrize("ncomp", [2, 4])
def test_apply_h_matches_dense_bdg_matrix(ncomp):
    lat = wl.Lattice(4, 6, 2, 0.9)
    fn = wl.Functional(ncomp=ncomp, mu_up=0.45, mu_dn=0.3 if ncomp == 4 else 0.45)
    rng = np.random.default_rng(5)
    shp = (lat.nz, lat.ny, lat.nx)
    V = rng.standard_normal(shp)
    Delta = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    M = 3
    psi = rng.standard_normal((M, ncomp) + shp) + 1j * rng.standard_normal((M, ncomp) + shp)
    H = dense_bdg(lat, fn, V, Delta)
    N = lat.n
    got = oracle.apply_h(psi, V, Delta, lat, fn)
    for j in range(M):
        if ncomp == 4:
            vec = psi[j].reshape(4 * N)
            ref = (H @ vec).reshape(4, *shp)
        else:   # (u_up, v_dn) block: rows/cols 0 and 3
            full = np.zeros(4 * N, dtype=complex)
            full[0:N] = psi[j, 0].ravel()
            full[3 * N:] = psi[j, 1].ravel()
            out = H @ full
            ref = np.stack([out[0:N].reshape(shp), out[3 * N:].reshape(shp)])
        assert np.max(np.abs(got[j] - ref)) < 1e-11


def test_apply_h_hermitian():
    lat = wl.Lattice(6, 4, 4, 1.0)
    fn = wl.Functional(ncomp=4, mu_up=0.6, mu_dn=0.4)
    rng = np.random.default_rng(7)
    shp = (lat.nz, lat.ny, lat.nx)
    V = rng.standard_normal(shp)
    Delta = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    a = rng.standard_normal((1, 4) + shp) + 1j * rng.standard_normal((1, 4) + shp)
    b = rng.standard_normal((1, 4) + shp) + 1j * rng.standard_normal((1, 4) + shp)
    lhs = np.vdot(a, oracle.apply_h(b, V, Delta, lat, fn))
    rhs = np.vdot(oracle.apply_h(a, V, Delta, lat, fn), b)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_uniform_frozen_bcs_eigenstates():
    """H (u_k, v_k) e^{ik.r} = +E_k (u_k, v_k) e^{ik.r}, E_k = sqrt(xi^2 + |Delta0|^2)."""
    lat = wl.Lattice(4, 4, 4, 1.0)
    U0, D0, mu = 0.2, 0.35 * np.exp(0.7j), 0.8
    fn = wl.Functional(ncomp=2, mu_up=mu, mu_dn=mu, frozen=1, U0=U0, Delta0=D0)
    shp = (4, 4, 4)
    V = np.full(shp, U0)
    Delta = np.full(shp, D0)
    for n in [(0, 0, 0), (1, 0, 0), (1, -1, 2), (-2, -2, -2), (1, 1, 1)]:
        f, k2 = plane_wave(lat, n)
        xi = 0.5 * k2 + U0 - mu
        E = math.sqrt(xi * xi + abs(D0) ** 2)
        u = math.sqrt(0.5 * (1 + xi / E))
        v = math.sqrt(0.5 * (1 - xi / E)) * np.conj(D0) / abs(D0)
        psi = np.stack([u * f, v * f])[None]
        Hpsi = oracle.apply_h(psi, V, Delta, lat, fn)
        assert np.max(np.abs(Hpsi - E * psi)) < 1e-12
