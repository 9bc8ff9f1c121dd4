"""Oracle pins: the dense DFT of Sec. Discretization against brute force."""
import cmath
import math

import numpy as np
import pytest

import oracle


def brute_force_dft3(f, sign):
    """Triple sum over every lattice point, written out with cmath.exp."""
    nz, ny, nx = f.shape
    out = np.zeros_like(f, dtype=np.complex128)
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx):
                s = 0j
                for z in range(nz):
                    for y in range(ny):
                        for x in range(nx):
                            ph = 2 * math.pi * (kx * x / nx + ky * y / ny + kz * z / nz)
                            s += cmath.exp(sign * 1j * ph) * f[z, y, x]
                out[kz, ky, kx] = s
    return out


@pytest.mark.parametrize("shape", [(4, 4, 4), (5, 5, 5), (3, 4, 5), (6, 2, 3)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_dft3_matches_triple_sum(shape, sign):
    rng = np.random.default_rng(1)
    f = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = brute_force_dft3(f, sign)
    got = oracle.dft3(f, sign)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8, 12, 20, 24, 32, 48, 64])
def test_dft_matrix_unitary_up_to_n(n):
    W = oracle.dft_matrix(n, -1)
    assert np.allclose(W @ np.conj(W.T), n * np.eye(n), atol=1e-11 * n)
    assert np.allclose(oracle.dft_matrix(n, 1), np.conj(W), atol=1e-14)


def test_dft3_inverse_and_parseval():
    rng = np.random.default_rng(2)
    f = rng.standard_normal((2, 6, 10, 8)) + 1j * rng.standard_normal((2, 6, 10, 8))
    F = oracle.dft3(f, -1)
    back = oracle.dft3(F, +1) / (6 * 10 * 8)
    assert np.max(np.abs(back - f)) < 1e-13
    assert abs(np.sum(np.abs(f) ** 2) - np.sum(np.abs(F) ** 2) / 480) < 1e-11 * np.sum(np.abs(f) ** 2)


def test_wavenumbers_fft_order():
    # k_n = 2 pi n / L below N/2 and 2 pi (n - N) / L from N/2 on; the
    # printed second branch (2n - N) pi / L would put k = 0 at n = N/2.
    k = oracle.wavenumbers(8, 0.5)
    L = 4.0
    assert np.allclose(k, 2 * np.pi / L * np.array([0, 1, 2, 3, -4, -3, -2, -1]))
    k5 = oracle.wavenumbers(5, 1.0)
    assert np.allclose(k5, 2 * np.pi / 5 * np.array([0, 1, 2, -2, -1]))
