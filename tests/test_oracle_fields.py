"""Oracle pins: external potential, potentials and observables closed forms."""
import math

import numpy as np

import oracle
import workloads as wl


def test_external_potential_minimum_image_and_ramp():
    lat = wl.Lattice(8, 6, 10, 0.5)
    fn = wl.Functional(ext_A=-0.3, ext_w=0.9, ext_r0=(3.5, 0.0, 4.5), ext_t_on=2.0)
    for t, ramp in [(0.0, 0.0), (1.0, 0.5), (2.0, 1.0), (5.0, 1.0), (0.5, math.sin(math.pi / 8) ** 2)]:
        U = oracle.external_potential(lat, fn, t)
        for (z, y, x) in [(0, 0, 0), (9, 5, 7), (4, 3, 1), (9, 0, 7)]:
            d2 = 0.0
            for i, n, r0 in ((x, lat.nx, 3.5), (y, lat.ny, 0.0), (z, lat.nz, 4.5)):
                L = n * lat.a
                d = abs(i * lat.a - r0)
                d = min(d, L - d)          # periodic images
                d2 += d * d
            ref = -0.3 * ramp * math.exp(-d2 / (2 * 0.81))
            assert abs(U[z, y, x] - ref) < 1e-15


def test_potentials_self_consistent_and_frozen():
    lat = wl.Lattice(4, 4, 4, 1.0)
    rng = np.random.default_rng(0)
    n = rng.random((4, 4, 4))
    kap = rng.standard_normal((4, 4, 4)) + 1j * rng.standard_normal((4, 4, 4))
    fn = wl.Functional(beta=0.37, g=1.5)
    V, D = oracle.potentials(n, kap, lat, fn, 0.0)
    assert np.allclose(V, 0.37 * n ** (2.0 / 3.0), rtol=1e-14, atol=0)
    assert np.allclose(D, -1.5 * kap, rtol=1e-15, atol=0)
    V0, D0 = oracle.potentials(np.zeros((4, 4, 4)), kap, lat, fn, 0.0)
    assert np.all(V0 == 0.0)
    fz = wl.Functional(frozen=1, U0=0.25, Delta0=0.1 - 0.2j)
    V, D = oracle.potentials(n, kap, lat, fz, 0.0)
    assert np.all(V == 0.25) and np.all(D == 0.1 - 0.2j)


def test_observables_uniform_bcs_closed_forms():
    lat = wl.Lattice(4, 6, 8, 1.0)
    fn = wl.Functional(ncomp=2, mu_up=0.5, mu_dn=0.5, beta=0.37, g=2.0, w=2.0)
    M = 50
    psi = wl.uniform_bcs(lat, fn, M, 0.3, 0.5)(0, M)
    idx = wl.k_order(lat)[:M]
    k2 = np.sum(wl.k_of(lat, idx) ** 2, axis=1)
    u, v = wl.bcs_uv(0.5 * k2 - 0.5, 0.3)
    Vbox = lat.n
    n = 2 * np.sum(v * v) / Vbox
    kap = np.sum(u * v) / Vbox
    o = oracle.observables(psi, lat, fn, 0.0)
    assert abs(o["N"] - 2 * np.sum(v * v)) < 1e-12
    assert abs(o["E_kin"] - 2 * np.sum(0.5 * k2 * v * v)) < 1e-12
    assert abs(o["E_int"] - Vbox * 0.6 * 0.37 * n ** (5.0 / 3.0)) < 1e-12
    assert abs(o["E_pair"] - Vbox * 2.0 * kap * kap) < 1e-12
    assert o["E_ext"] == 0.0
    assert abs(o["mean_abs_delta"] - 2.0 * kap) < 1e-13
    assert np.allclose(o["r_cm"], [1.5, 2.5, 3.5], atol=1e-12)
    assert np.allclose(o["norms"], 1.0, atol=1e-13)


def bdg_vacuum(lat, fn, seed, ncomp=2):
    """Positive-energy eigenvectors of a non-uniform dense BdG matrix (Eq. tdslda).

    The matrix is built independently of the oracle from the DVR blocks of
    Eq. (d2) with random smooth-free V(r) and Delta(r).  The eigenvectors form a
    complete orthonormal quasiparticle vacuum, the kind of input the paper's
    static solver hands to the time-dependent code; for such a set the
    energy is an exact invariant of the flow.
    """
    from test_oracle_operators import dense_bdg
    rng = np.random.default_rng(seed)
    shp = (lat.nz, lat.ny, lat.nx)
    N = lat.n
    V = 0.3 * rng.standard_normal(shp)
    D = 0.4 + 0.2 * (rng.standard_normal(shp) + 1j * rng.standard_normal(shp))
    H4 = dense_bdg(lat, fn, V, D)
    if ncomp == 2:
        idx = np.r_[0:N, 3 * N:4 * N]
        H = H4[np.ix_(idx, idx)]
    else:
        H = H4
    e, U = np.linalg.eigh(H)
    pos = U[:, e > 0]
    psi = np.stack([pos[c * N:(c + 1) * N].T.reshape(-1, *shp) for c in range(ncomp)], axis=1)
    return psi / lat.a ** 1.5


def ddt(q, psi, lat, fn, h=1e-5):
    f = oracle.rhs(psi, lat, fn, 0.0)
    return (oracle.observables(psi + h * f, lat, fn, 0.0)[q]
            - oracle.observables(psi - h * f, lat, fn, 0.0)[q]) / (2 * h)


def test_energy_and_number_constant_along_exact_flow():
    """dE/dt = dN/dt = 0 along f(psi) = -i H psi for a complete quasiparticle vacuum.

    Central differences of E and N along the exact right-hand side: no
    integrator is involved, so this ties the energy formula, the densities,
    the potentials and the Hamiltonian to one functional.
    """
    lat = wl.Lattice(4, 4, 4, 1.0)
    fn = wl.Functional(ncomp=2, mu_up=0.7, mu_dn=0.7, beta=0.37, g=1.5, w=2.0)
    psi = bdg_vacuum(lat, fn, seed=1)
    o = oracle.observables(psi, lat, fn, 0.0)
    assert abs(ddt("E", psi, lat, fn)) < 1e-8 * o["E_kin"]
    assert abs(ddt("N", psi, lat, fn)) < 1e-8 * o["N"]
    # the parts do change: the test is not vacuous
    assert abs(ddt("E_pair", psi, lat, fn)) > 1e-4 * abs(o["E_pair"])
    assert abs(ddt("E_int", psi, lat, fn)) > 1e-4 * abs(o["E_int"])


def test_energy_rate_is_second_order_in_independent_noise():
    """Independent complex noise breaks the r <-> r' symmetry: dE/dt = O(eps^2), N exact."""
    lat = wl.Lattice(4, 4, 4, 1.0)
    fn = wl.Functional(ncomp=2, mu_up=1.0, mu_dn=1.0, beta=0.37, g=1.5, w=1.0)
    rates = []
    for eps in (0.04, 0.02):
        psi = wl.uniform_bcs(lat, fn, 128, 0.5, 1.0, copies=2, eps=eps, seed=4)(0, 128)
        rates.append(ddt("E", psi, lat, fn))
        assert abs(ddt("N", psi, lat, fn)) < 1e-9
    assert 3.5 < rates[0] / rates[1] < 4.5


def test_energy_flow_with_four_components():
    """C = 4 with spin-dependent mu: the positive-energy eigenvectors of the full
    4N x 4N matrix conserve E along the exact flow."""
    lat = wl.Lattice(4, 4, 2, 1.0)
    fn = wl.Functional(ncomp=4, mu_up=0.6, mu_dn=0.4, beta=0.37, g=2.0, w=1.0)
    psi = bdg_vacuum(lat, fn, seed=2, ncomp=4)
    o = oracle.observables(psi, lat, fn, 0.0)
    assert abs(ddt("E", psi, lat, fn)) < 1e-8 * o["E_kin"]
    assert abs(ddt("E_pair", psi, lat, fn)) > 1e-4 * abs(o["E_pair"])


def test_spin_resolved_numbers_closed_form():
    """N_up, N_dn of the spin sum of Eq. (rho_t) on a spin-imbalanced C = 4 BCS set.

    Block A states carry (u_up, v_dn) = (u_k, v_k) e^{ik.r}/sqrt(V), block B states
    (u_dn, v_up) = (u_k, -v_k) e^{ik.r}/sqrt(V); with na != nb the two spin numbers
    differ, so a swapped or dropped component fails: N_dn = sum_A v_k^2,
    N_up = sum_B v_k^2, N = N_up + N_dn.  The C = 2 reduction is spin-symmetric."""
    lat = wl.Lattice(4, 4, 6, 0.9)
    N3 = lat.n
    fn = wl.Functional(ncomp=4, mu_up=0.6, mu_dn=0.4, beta=0.37, g=2.0, w=1.0)
    na, nb = 11, 5
    kx = 2 * np.pi * np.fft.fftfreq(4, d=lat.a)
    kz = 2 * np.pi * np.fft.fftfreq(6, d=lat.a)
    ks = sorted(((a, b, c) for a in kx for b in kx for c in kz), key=lambda k: (k[0] ** 2 + k[1] ** 2 + k[2] ** 2, k))
    z, y, x = np.meshgrid(np.arange(6) * lat.a, np.arange(4) * lat.a, np.arange(4) * lat.a, indexing="ij")
    vol = N3 * lat.a ** 3
    psi = np.zeros((na + nb, 4, 6, 4, 4), dtype=complex)
    vsq = []
    for j in range(na + nb):
        k = ks[j if j < na else j - na]
        xi = 0.5 * (k[0] ** 2 + k[1] ** 2 + k[2] ** 2) - 0.5
        E = math.sqrt(xi * xi + 0.25 ** 2)
        u, v = math.sqrt(0.5 * (1 + xi / E)), math.sqrt(0.5 * (1 - xi / E))
        pw = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z)) / math.sqrt(vol)
        if j < na:
            psi[j, 0], psi[j, 3] = u * pw, v * pw
        else:
            psi[j, 1], psi[j, 2] = u * pw, -v * pw
        vsq.append(v * v)
    o = oracle.observables(psi, lat, fn, 0.0)
    assert abs(o["N_dn"] - sum(vsq[:na])) < 1e-13
    assert abs(o["N_up"] - sum(vsq[na:])) < 1e-13
    assert abs(o["N"] - o["N_up"] - o["N_dn"]) < 1e-13
    assert abs(o["N_dn"] - o["N_up"]) > 0.01
    # C = 2: spin-symmetric halves
    f2 = wl.Functional(ncomp=2, mu_up=0.5, mu_dn=0.5, beta=0.37, g=2.0, w=2.0)
    p2 = psi[:na][:, [0, 3]]
    o2 = oracle.observables(p2, lat, f2, 0.0)
    assert o2["N_up"] == o2["N_dn"] == 0.5 * o2["N"]
    assert abs(o2["N"] - 2 * sum(vsq[:na])) < 1e-13


def test_spin_numbers_constant_along_exact_flow():
    """dN_up/dt = dN_dn/dt = 0 along f = -i H psi for a complete C = 4 quasiparticle
    vacuum whose chemical potentials differ enough to leave one unpaired spin-up
    state: the vacuum then holds exactly one more up than down particle."""
    lat = wl.Lattice(4, 4, 4, 1.0)
    fn = wl.Functional(ncomp=4, mu_up=1.2, mu_dn=0.2, beta=0.37, g=1.5, w=1.0)
    psi = bdg_vacuum(lat, fn, 7, ncomp=4)
    o = oracle.observables(psi, lat, fn, 0.0)
    assert abs(o["N_up"] - o["N_dn"] - 1.0) < 1e-12
    assert abs(ddt("N_up", psi, lat, fn)) < 1e-9 and abs(ddt("N_dn", psi, lat, fn)) < 1e-9
