"""Oracle pins: the ABM integrator against the printed coefficients and error constants."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "abm_coefficients.txt")


def load_golden():
    vals = {}
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split()
        vals[k] = None if v == "missing" else Fraction(v)
    return vals


def test_printed_coefficients_match_oracle():
    g = load_golden()
    assert g["predictor.y'_n"] is None
    assert [Fraction(c) for c in oracle.ABM_P[1:]] == [g["predictor.y'_n-1"], g["predictor.y'_n-2"],
                                                       g["predictor.y'_n-3"]]
    assert [Fraction(c) for c in oracle.ABM_C] == [g["corrector.m'_n+1"], g["corrector.y'_n"],
                                                   g["corrector.y'_n-1"], g["corrector.y'_n-2"]]
    assert Fraction(oracle.ABM_M).limit_denominator(1000) == g["modifier.weight"]
    assert Fraction(oracle.ABM_Y).limit_denominator(1000) == g["final.weight"]
    # The modifier and final weights follow from the two printed error constants:
    # 161/170 = E_p / (E_p - E_c), 9/170 = -E_c / (E_p - E_c).
    ep, ec = g["predictor.error"], g["corrector.error"]
    assert ep / (ep - ec) == g["modifier.weight"]
    assert -ec / (ep - ec) == g["final.weight"]


def derive_missing_predictor_coefficient():
    """Solve for the y'_n weight that makes Eq. (p) exact for y = t (from exact arithmetic)."""
    g = load_golden()
    # y = t, t_n = 0, dt = 1: y_{n+1} = 1 = (0 + -1)/2 + (1/48)(c0 + -99 + 69 - 17)
    rest = g["predictor.y'_n-1"] + g["predictor.y'_n-2"] + g["predictor.y'_n-3"]
    return (Fraction(1) + Fraction(1, 2)) / g["predictor.dt_factor"] - rest


def test_missing_predictor_coefficient_is_119():
    assert derive_missing_predictor_coefficient() == 119
    assert oracle.ABM_P[0] == 119.0


def run_one_abm_step(deg, dt=0.3, t0=0.7):
    """Apply the oracle's abm_update once to y(t) = t^deg with exact history."""
    y = lambda t: t ** deg
    yp = lambda t: deg * t ** (deg - 1) if deg > 0 else 0.0 * t
    tn = t0
    dy = tuple(yp(tn - i * dt) for i in range(4))
    # d_n = p_n - c_n: with exact history both are exact for deg <= 4
    y_next, d_next = oracle.abm_update(y(tn), y(tn - dt), dy, 0.0,
                                       lambda m: yp(tn + dt), dt)
    return y_next, d_next, y(tn + dt)


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_abm_exact_for_polynomials_up_to_degree_4(deg):
    y_next, d_next, exact = run_one_abm_step(deg)
    assert abs(y_next - exact) < 1e-13 * max(1.0, abs(exact))
    assert abs(d_next) < 1e-13 * max(1.0, abs(exact))


def test_abm_error_constants_degree_5():
    """For y = t^5 (y^(5) = 120): y - p = 161/480 dt^5 y^(5), y - c = -9/480 dt^5 y^(5)."""
    g = load_golden()
    dt, t0 = 0.25, 0.5
    y = lambda t: t ** 5
    yp = lambda t: 5 * t ** 4
    dy = tuple(yp(t0 - i * dt) for i in range(4))
    half = 0.5 * (y(t0) + y(t0 - dt))
    p = half + dt / 48 * sum(c * d for c, d in zip(oracle.ABM_P, dy))
    c = half + dt / 48 * (oracle.ABM_C[0] * yp(t0 + dt) + oracle.ABM_C[1] * dy[0]
                          + oracle.ABM_C[2] * dy[1] + oracle.ABM_C[3] * dy[2])
    exact = y(t0 + dt)
    assert abs((exact - p) - float(g["predictor.error"]) * dt ** 5 * 120) < 1e-13
    assert abs((exact - c) - float(g["corrector.error"]) * dt ** 5 * 120) < 1e-13
    # the oracle's update, fed the exact derivative at t_{n+1}, gives c + 9/170 (p - c)
    y_next, d_next = oracle.abm_update(y(t0), y(t0 - dt), dy, 0.0, lambda m: yp(t0 + dt), dt)
    assert abs(d_next - (p - c)) < 1e-14
    assert abs(y_next - (c + 9.0 / 170.0 * (p - c))) < 1e-14


def companion(omega_dt):
    """Transition matrix of one ABM step for y' = -i w y, dt = 1.

    The oracle's abm_update is linear in the state
    (y_n, y_{n-1}, y'_{n-1}, y'_{n-2}, y'_{n-3}, d_n); its columns are the
    images of the unit vectors.
    """
    lam = -1j * omega_dt
    f = lambda y: lam * y

    def step(s):
        yn, ynm1, d1, d2, d3, dn = s
        dyn = lam * yn
        yx, dx = oracle.abm_update(yn, ynm1, (dyn, d1, d2, d3), dn, f, 1.0)
        return np.array([yx, yn, dyn, d1, d2, dx])
    return np.stack([step(e) for e in np.eye(6, dtype=complex)], axis=1)


@pytest.mark.parametrize("wdt", [0.03, 0.074, 0.2, 0.25])
def test_abm_stable_on_imaginary_axis_below_limit(wdt):
    assert np.max(np.abs(np.linalg.eigvals(companion(wdt)))) <= 1.0 + 1e-12


@pytest.mark.parametrize("wdt", [0.3, 0.6])
def test_abm_unstable_beyond_limit(wdt):
    assert np.max(np.abs(np.linalg.eigvals(companion(wdt)))) > 1.0 + 1e-7


@pytest.mark.parametrize("wdt,lo,hi", [(0.074, 1.5e-9, 2.2e-9), (0.03, 6e-12, 9e-12)])
def test_abm_principal_root_error_per_step(wdt, lo, hi):
    """The principal root approximates exp(-i w dt) to O((w dt)^6) per step."""
    ev = np.linalg.eigvals(companion(wdt))
    pr = ev[np.argmin(np.abs(ev - np.exp(-1j * wdt)))]
    assert lo < abs(pr - np.exp(-1j * wdt)) < hi
