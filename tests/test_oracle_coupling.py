"""Pins of the regularised pairing coupling of Eq. (geff_3D) in the oracle."""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from test_oracle_fields import bdg_vacuum, ddt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lattice_K.txt")


def golden_K():
    lines = [ln for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    return float(lines[0])


def test_K_matches_printed_value():
    """The quadrature of the printed integral reproduces the printed digits."""
    assert abs(oracle.lattice_K() - golden_K()) < 2e-15


def test_K_equals_cube_face_integral():
    """Independent route: K / (4 pi a) is the Brillouin-zone integral of 1/k^2 over
    (2 pi)^3, i.e. K = (1 / 2 pi^2) int over [-pi, pi]^3 of d^3k / k^2.  In spherical
    shells the radial integral gives the distance to the cube's surface, and projecting
    one face onto its tangent plane turns the angular integral into
    K = (12 / pi) int_0^1 int_0^1 du dv / (1 + u^2 + v^2)."""
    from scipy.integrate import dblquad
    val, _ = dblquad(lambda v, u: 1.0 / (1.0 + u * u + v * v), 0.0, 1.0, 0.0, 1.0,
                     epsabs=1e-14, epsrel=1e-13)
    assert abs(12.0 / math.pi * val - oracle.lattice_K()) < 1e-13


def test_K_against_zone_sum():
    """The zone sum (1/L^3) sum_{k != 0} 1/k^2 on an n^3 lattice (a = 1) approaches
    K / (4 pi) with a finite-size error ~ 1/n: Richardson extrapolation in 1/n of
    the sums at n = 24, 48 lands within 2e-3 of K / (4 pi)."""
    def zone_sum(n):
        k = 2 * np.pi * np.fft.fftfreq(n)
        k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
        k2[0, 0, 0] = np.inf
        return float(np.sum(1.0 / k2)) / n ** 3
    s1, s2 = zone_sum(24), zone_sum(48)
    extrap = 2 * s2 - s1
    assert abs(extrap - oracle.lattice_K() / (4 * math.pi)) < 2e-3
    assert abs(s2 - oracle.lattice_K() / (4 * math.pi)) > abs(extrap - oracle.lattice_K() / (4 * math.pi))


def test_bare_coupling_without_regularisation():
    lat = wl.Lattice(4, 4, 4, 1.0)
    fn = wl.Functional(ncomp=2, g=1.7)
    assert oracle.effective_coupling(fn, lat) == 1.7


@pytest.mark.parametrize("g", [1.5, -2.0])
def test_regularised_coupling_shift_scales_with_inverse_spacing(g):
    """1/g_eff - 1/g = -K / (4 pi a): halving a doubles the shift."""
    fn = wl.Functional(ncomp=2, g=g, regularize=1)
    s1 = 1 / oracle.effective_coupling(fn, wl.Lattice(4, 4, 4, 1.0)) - 1 / g
    s2 = 1 / oracle.effective_coupling(fn, wl.Lattice(4, 4, 4, 0.5)) - 1 / g
    assert abs(s2 - 2 * s1) < 1e-14
    assert abs(s1 + golden_K() / (4 * math.pi)) < 1e-14


def test_regularised_delta_uses_g_eff():
    lat = wl.Lattice(4, 4, 4, 1.0)
    fn = wl.Functional(ncomp=2, beta=0.37, g=1.5, regularize=1)
    rng = np.random.default_rng(3)
    n = rng.random((4, 4, 4))
    kappa = rng.standard_normal((4, 4, 4)) + 1j * rng.standard_normal((4, 4, 4))
    _, D = oracle.potentials(n, kappa, lat, fn, 0.0)
    geff = oracle.effective_coupling(fn, lat)
    assert geff > 1.5
    assert np.allclose(D, -geff * kappa, rtol=1e-15, atol=0)


def test_energy_constant_along_exact_flow_regularised():
    """Delta and E_pair use the same g_eff: dE/dt = 0 along the exact flow."""
    lat = wl.Lattice(4, 4, 4, 1.0)
    fn = wl.Functional(ncomp=2, mu_up=0.7, mu_dn=0.7, beta=0.37, g=1.5, w=2.0, regularize=1)
    psi = bdg_vacuum(lat, fn, seed=1)
    o = oracle.observables(psi, lat, fn, 0.0)
    assert abs(ddt("E", psi, lat, fn)) < 1e-8 * o["E_kin"]
    assert abs(ddt("E_pair", psi, lat, fn)) > 1e-4 * abs(o["E_pair"])
