"""The dense z-term operator of the in-kernel z-term path against the oracle.

The ABM phases at 32^3 FP64 apply the kinetic term along z as the real symmetric
circulant matrix T_z[z][z'] = c_z sum_k m_k^2 cos(2 pi k (z - z') / N), with
c_z = (2 pi^2 / L_z^2) / N and m_k the signed index of k (the Nyquist term kept, as
for every even derivative).  On a function of z alone the oracle's kinetic operator
F^-1 (|k|^2 / 2) F (Sec. "Discretization", built from its own dense DFT matrices)
reduces to exactly that term, so the two must agree to rounding; and T_z must be
symmetric with the plane waves as eigenvectors.  (The library builds the same matrix
in long double on the host; the GPU tests compare its steps with the oracle.)
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


def t_z(n, a):
    lz = n * a
    cz = 2.0 * math.pi ** 2 / lz ** 2 / n
    row = np.zeros(n)
    for d in range(n):
        s = 0.0
        for k in range(n):
            m = k if 2 * k < n else k - n
            s += m * m * math.cos(2.0 * math.pi * ((k * d) % n) / n)
        row[d] = cz * s
    return np.array([[row[(z - zp) % n] for zp in range(n)] for z in range(n)])


@pytest.mark.parametrize("n", [8, 9, 16, 20, 24, 32])
@pytest.mark.parametrize("a", [1.0, 0.7])
def test_dense_z_operator_is_the_kinetic_term_along_z(n, a):
    lat = wl.Lattice(1, 1, n, a)
    rng = np.random.default_rng(n)
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = oracle.kinetic(f.reshape(n, 1, 1), lat).reshape(n)
    got = t_z(n, a) @ f
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [16, 32])
def test_dense_z_operator_symmetry_and_plane_waves(n):
    T = t_z(n, 1.0)
    assert np.allclose(T, T.T, rtol=0, atol=1e-15 * np.max(np.abs(T)))
    z = np.arange(n)
    for k in (0, 1, n // 2 - 1, n // 2):
        kk = oracle.wavenumbers(n, 1.0)[k]
        e = np.exp(1j * kk * z)
        # the Nyquist plane wave is real (cos(pi z)) and keeps its eigenvalue kk^2 / 2
        assert np.max(np.abs(T @ e - 0.5 * kk * kk * e)) < 1e-12 * max(1.0, kk * kk)
