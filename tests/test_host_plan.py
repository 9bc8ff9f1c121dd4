"""Host logic of the library (CPU only): FFT plans, twiddle tables and the bf16 kinetic
matrix, checked against the oracle's DFT and kinetic operator."""
import ctypes as ct
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_00745_amd", "csrc")


@pytest.fixture(scope="module")
def hp(tmp_path_factory):
    out = tmp_path_factory.mktemp("hp") / "libhp.so"
    src = os.path.join(os.path.dirname(__file__), "host_plan_helper.cpp")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, "-o", str(out), src], check=True)
    return ct.CDLL(str(out))


def plan(hp, n):
    nst = ct.c_int()
    radix = (ct.c_int * 7)()
    p = (ct.c_int * 7)()
    off = (ct.c_int * 7)()
    tw = np.zeros(2 * 4096)
    m = hp.hp_plan(n, ct.byref(nst), radix, p, off, tw.ctypes.data_as(ct.c_void_p), 2048)
    if m < 0:
        return None
    tw = tw[:2 * m:2] + 1j * tw[1:2 * m:2]
    return [(radix[s], p[s], off[s]) for s in range(nst.value)], tw


def smooth(n):
    m = n
    for q in (2, 3, 5):
        while m % q == 0:
            m //= q
    return m == 1


def test_plan_factorisation(hp):
    for n in range(1, 129):
        pl = plan(hp, n)
        if smooth(n):
            radices = [r for r, _, _ in pl[0]]
            assert int(np.prod(radices)) == n and all(r in (2, 3, 4, 5, 8) for r in radices), n
            ps = [p for _, p, _ in pl[0]]
            assert ps == [int(np.prod(radices[:s])) for s in range(len(radices))], n
        else:
            assert pl is None, n


def stockham_with_plan(x, stages, tw, inverse):
    """The device's Stockham stage indexing (inputs i + q m, outputs (i/p) p R + k + s p,
    twiddles tw[off + k (R-1) + q - 1], conjugated for the inverse) applied with numpy."""
    n = len(x)
    sig = 1 if inverse else -1
    for R, p, off in stages:
        m = n // R
        y = np.empty_like(x)
        for i in range(m):
            k = i % p
            a = np.array([x[i + q * m] for q in range(R)])
            if p > 1:
                for q in range(1, R):
                    w = tw[off + k * (R - 1) + q - 1]
                    a[q] *= np.conj(w) if inverse else w
            b = np.array([np.sum(a * np.exp(sig * 2j * np.pi * np.arange(R) * s / R)) for s in range(R)])
            j = (i // p) * p * R + k
            for s in range(R):
                y[j + s * p] = b[s]
        x = y
    return x


@pytest.mark.parametrize("n", [2, 3, 5, 6, 8, 12, 16, 20, 24, 30, 32, 48, 64, 96, 120, 128])
def test_plan_and_twiddles_reproduce_dft(hp, n):
    stages, tw = plan(hp, n)
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    W = oracle.dft_matrix(n, -1)
    assert np.max(np.abs(stockham_with_plan(x, stages, tw, False) - W @ x)) < 1e-13 * n
    assert np.max(np.abs(stockham_with_plan(x, stages, tw, True) - np.conj(W) @ x)) < 1e-13 * n


@pytest.mark.parametrize("n", [8, 16, 20, 24, 32, 48, 64])
def test_full_tables(hp, n):
    tw = np.zeros(2 * n)
    assert hp.hp_full_table(n, tw.ctypes.data_as(ct.c_void_p)) == n
    w = tw[0::2] + 1j * tw[1::2]
    # reference in 80-bit long double (numpy's float64 angle 2 pi j / n is itself off by ~1e-15)
    ang = -2 * np.longdouble("3.14159265358979323846264338327950288") * np.arange(n, dtype=np.longdouble) / n
    ref = np.cos(ang).astype(np.float64) + 1j * np.sin(ang).astype(np.float64)
    assert np.max(np.abs(w - ref)) < 1.2e-16
    assert np.max(np.abs(w - oracle.dft_matrix(n, -1)[1])) < 4e-15


def bf16_value(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("n,a", [(16, 1.0), (32, 1.0), (48, 0.8), (64, 1.0)])
def test_kinetic_matrix_bf16_split(hp, n, a):
    """hi + lo of the bf16 split equals the oracle's 1D kinetic matrix to ~2^-16."""
    out = np.zeros(2 * n * n, dtype=np.uint16)
    hp.hp_kinetic_bf16(n, ct.c_double(a), out.ctypes.data_as(ct.c_void_p))
    hi = bf16_value(out[:n * n]).reshape(n, n)
    lo = bf16_value(out[n * n:]).reshape(n, n)
    lat = wl.Lattice(n, 1, 1, a)
    T = np.zeros((n, n))
    for m in range(n):
        e = np.zeros((1, 1, n), dtype=complex)
        e[0, 0, m] = 1.0
        T[:, m] = oracle.kinetic(e, lat)[0, 0].real
    scale = np.max(np.abs(T))
    assert np.max(np.abs(hi + lo - T)) < 2.0 ** -15 * scale
    assert np.max(np.abs(hi - T)) > 2.0 ** -12 * scale     # the lo part matters
    assert np.allclose(hi, hi.T) and np.allclose(lo, lo.T)
