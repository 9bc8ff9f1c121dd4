"""CPU FP64 oracle of the TDSLDA time step (TEST INFRASTRUCTURE ONLY).

This module is the slow, plain reference that the GPU library is checked
against.  Only the test suite, the smoke check of the entry module and
the CPU-baseline leg of the benchmark may import it; the product path never
calls it.  It shares no code with the HIP library: it has its own lattice,
its own dense DFT matrices (no FFT library), its own Hamiltonian, densities,
potentials, series-expansion start-up and Adams-Bashforth-Milne integrator.

Everything is float64 / complex128.  Arrays of qpwfs have shape
(M, C, nz, ny, nx) with C = 2 for (u, v) and C = 4 for
(u_up, u_dn, v_up, v_dn); x is the fastest axis.

Citations name the paper's sections and equations (arXiv:2009.00745, "The
LISE package: solvers for static and time-dependent superfluid local density
approximation equations in three dimensions").

Readings of passages that are silent, ambiguous or garbled:
  * k_n for n >= N/2 is 2*pi*(n-N)/L (the printed second branch is garbled);
    for odd N the threshold N/2 is taken as a real number.
  * The predictor's missing y'_n coefficient is 119 (the unique value that
    makes Eq. (p) exact for polynomials of degree <= 4 and reproduces the
    printed error constant 161/480).
  * Start-up: three series-expansion steps (order 4) fill y'_0..y'_2, y_2,
    y_3; the first modifier uses p_3 - c_3 = 0.
  * Trivial-phase removal (Eq. sp_en) is optional (fn.remove_phase): every
    right-hand side takes eta_k of the vector it acts on; each series
    propagation takes eta from its starting psi and its own H.  Per-step
    renormalisation is not done (the paper finds it unnecessary).
  * C = 2 keeps the (u_up, v_dn) block of Eq. (tdslda) with h_updn = 0; its
    densities carry a weight w: n = w sum |v|^2, kappa = (w/2) sum v* u.
  * C = 4 uses the singlet average kappa = 1/2 sum (v_dn* u_up - v_up* u_dn),
    which equals Eq. (nu_t) for spin-symmetric sets; spin-dependent chemical
    potentials mu_up, mu_dn sit on the u_sigma and v_sigma diagonals.
  * Local potentials of the cold-atom functional: U = beta n^{2/3} plus an
    optional external scalar potential, Delta = -g kappa (Eq. pairingfield).
"""
import math
import numpy as np


# ---------------------------------------------------------------------------
# Lattice and discrete Fourier transform (Sec. Discretization)

def wavenumbers(n, a):
    """k_n = 2 pi n / L for n < N/2 and 2 pi (n - N) / L for n >= N/2, L = N a.

    The paper states the rule for even N.  For odd N the same rule with the
    real number N/2 keeps the symmetric set |n| <= (N - 1)/2.
    """
    L = n * a
    return np.array([2.0 * math.pi * (i if 2 * i < n else i - n) / L for i in range(n)])


def dft_matrix(n, sign):
    """W[j, l] = exp(sign * 2 pi i (j l mod n) / n)  (dense, built explicitly)."""
    j = np.arange(n)
    return np.exp(sign * 2j * math.pi * ((j[:, None] * j[None, :]) % n) / n)


def dft3(f, sign):
    """Apply the 1D transform with matrix W(sign) along x, y and z.

    sign = -1 is the forward transform of Sec. Discretization,
    F[f](k) = sum_x exp(-i k x) f(x); sign = +1 without the 1/N factor is the
    unnormalised inverse.
    """
    nz, ny, nx = f.shape[-3:]
    out = np.matmul(f, dft_matrix(nx, sign).T)                      # x
    out = np.matmul(dft_matrix(ny, sign), out)                      # y
    out = np.einsum("kz,...zyx->...kyx", dft_matrix(nz, sign), out)  # z
    return out


def k_squared(lat):
    kx = wavenumbers(lat.nx, lat.a)
    ky = wavenumbers(lat.ny, lat.a)
    kz = wavenumbers(lat.nz, lat.a)
    return kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2


def kinetic(f, lat):
    """T f = F^{-1}[ (|k|^2 / 2) F f ]  (hbar = m = 1, Nyquist mode kept).

    The Laplacian is an even derivative, so the Nyquist component is not
    zeroed (zeroing applies to odd derivatives only).
    """
    F = dft3(f, -1)
    F = F * (0.5 * k_squared(lat))
    return dft3(F, +1) / lat.n


def derivative_matrix(n, a):
    """D = F^{-1} diag(i k) F on one axis (Sec. Discretization): the spectral first
    derivative, with the N/2 mode of an even axis set to zero as the paper does
    for odd derivatives."""
    k = wavenumbers(n, a).copy()
    if n % 2 == 0:
        k[n // 2] = 0.0
    return dft_matrix(n, +1) @ np.diag(1j * k) @ dft_matrix(n, -1) / n


def gradient(f, lat):
    """(d/dx f, d/dy f, d/dz f) of arrays (..., nz, ny, nx) by dense spectral derivatives."""
    dx = np.matmul(f, derivative_matrix(lat.nx, lat.a).T)
    dy = np.matmul(derivative_matrix(lat.ny, lat.a), f)
    dz = np.einsum("kz,...zyx->...kyx", derivative_matrix(lat.nz, lat.a), f)
    return dx, dy, dz


# ---------------------------------------------------------------------------
# Densities (Eq. rho_t, nu_t) and potentials (Eq. pairingfield)

def densities(psi, fn):
    """Normal density n(r) and anomalous density kappa(r).

    C = 4 (Eq. rho_t, nu_t with the singlet average):
        n = sum_k (|v_up|^2 + |v_dn|^2),
        kappa = 1/2 sum_k (v_dn^* u_up - v_up^* u_dn).
    C = 2 (block (u_up, v_dn), each state standing for w spin states):
        n = w sum_k |v|^2,  kappa = (w/2) sum_k v^* u.
    """
    if fn.ncomp == 2:
        u, v = psi[:, 0], psi[:, 1]
        n = fn.w * np.sum(np.abs(v) ** 2, axis=0)
        kappa = 0.5 * fn.w * np.sum(np.conj(v) * u, axis=0)
    elif fn.ncomp == 4:
        uu, ud, vu, vd = psi[:, 0], psi[:, 1], psi[:, 2], psi[:, 3]
        n = np.sum(np.abs(vu) ** 2 + np.abs(vd) ** 2, axis=0)
        kappa = 0.5 * np.sum(np.conj(vd) * uu - np.conj(vu) * ud, axis=0)
    else:
        raise ValueError("ncomp must be 2 or 4")
    return n, kappa


def current_density(psi, lat, fn):
    """j(r) = (1 / 2i) sum_k [v_k grad v_k^* - v_k^* grad v_k] = -sum_k Im(v_k^* grad v_k)
    (Eq. j), over the v components (v for C = 2 with the weight w; v_up and v_dn
    for C = 4).  Returns an array (3, nz, ny, nx) ordered x, y, z."""
    if fn.ncomp == 2:
        vs, wt = [1], fn.w
    else:
        vs, wt = [2, 3], 1.0
    j = np.zeros((3, lat.nz, lat.ny, lat.nx))
    for c in vs:
        v = psi[:, c]
        for ax, dv in enumerate(gradient(v, lat)):
            j[ax] -= wt * np.sum(np.imag(np.conj(v) * dv), axis=0)
    return j


def kick(psi, chi, fn):
    """Gauge transformation of Eq. (kick): u -> exp(i chi) u, v -> exp(-i chi) v for
    every qpwf (C = 2: (u, v); C = 4: (u_up, u_dn, v_up, v_dn))."""
    out = np.array(psi, dtype=np.complex128, copy=True)
    ph = np.exp(1j * np.asarray(chi, dtype=np.float64))
    nu = 1 if fn.ncomp == 2 else 2
    out[:, :nu] *= ph
    out[:, nu:] *= np.conj(ph)
    return out


def external_potential(lat, fn, t):
    """Scalar external potential U_ext(r, t) (Sec. External boosts and external potentials).

    A Gaussian well A*ramp(t)*exp(-d^2 / (2 w^2)) about r0, d the
    minimum-image distance on the periodic box, ramp = sin^2(pi t / (2 t_on))
    for 0 <= t < t_on and 1 afterwards (and 1 when t_on = 0).
    """
    if fn.ext_A == 0.0:
        return np.zeros((lat.nz, lat.ny, lat.nx))
    if fn.ext_t_on > 0.0 and t < fn.ext_t_on:
        ramp = math.sin(math.pi * max(t, 0.0) / (2.0 * fn.ext_t_on)) ** 2
    else:
        ramp = 1.0

    def dist1(n, r0):
        L = n * lat.a
        d = np.arange(n) * lat.a - r0
        return d - L * np.round(d / L)

    dx = dist1(lat.nx, fn.ext_r0[0])
    dy = dist1(lat.ny, fn.ext_r0[1])
    dz = dist1(lat.nz, fn.ext_r0[2])
    d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
    return fn.ext_A * ramp * np.exp(-d2 / (2.0 * fn.ext_w ** 2))


def lattice_K():
    """K = (12 / pi) * int_0^{pi/4} ln(1 + 1 / cos^2 theta) d theta (Eq. geff_3D),
    by adaptive quadrature of the printed integral."""
    from scipy.integrate import quad
    val, _ = quad(lambda th: math.log1p(1.0 / math.cos(th) ** 2), 0.0, math.pi / 4.0,
                  epsabs=1e-14, epsrel=1e-13, limit=200)
    return 12.0 / math.pi * val


def effective_coupling(fn, lat):
    """Coupling used in Delta = -g kappa and E_pair.

    fn.regularize = 0: the bare g.  fn.regularize = 1: the lattice
    renormalisation of Eq. (geff_3D) for a cubic lattice with its natural
    cutoff, 1/g_eff = 1/g - (m* / (4 pi^2 hbar^2)) (pi / a) K, here with
    m* = m = hbar = 1, i.e. 1/g_eff = 1/g - K / (4 pi a).
    """
    if not getattr(fn, "regularize", 0):
        return fn.g
    inv = 1.0 / fn.g - lattice_K() / (4.0 * math.pi * lat.a)
    if inv == 0.0:
        raise ValueError("regularised coupling diverges (1/g = K / (4 pi a))")
    return 1.0 / inv


def potentials(n, kappa, lat, fn, t):
    """V = U + U_ext and Delta.

    Self-consistent: U = beta n^{2/3}, Delta = -g kappa (Eq. pairingfield),
    g replaced by g_eff of Eq. (geff_3D) when fn.regularize is set.
    Frozen (test mode): U = U0 and Delta = Delta0 everywhere.
    """
    if fn.frozen:
        U = np.full(n.shape, float(fn.U0))
        Delta = np.full(n.shape, complex(fn.Delta0))
    else:
        U = fn.beta * np.cbrt(n) ** 2
        Delta = -effective_coupling(fn, lat) * kappa
    return U + external_potential(lat, fn, t), Delta


# ---------------------------------------------------------------------------
# Quasiparticle Hamiltonian (Eq. tdslda, h = T + V, h_updn = 0)

def apply_h(psi, V, Delta, lat, fn):
    """H psi for every qpwf, with the local fields V (real) and Delta (complex).

    C = 4, rows of Eq. (tdslda) with h* = h (T and V are real):
        H u_up = (h - mu_up) u_up + Delta v_dn
        H u_dn = (h - mu_dn) u_dn - Delta v_up
        H v_up = -Delta^* u_dn - (h - mu_up) v_up
        H v_dn =  Delta^* u_up - (h - mu_dn) v_dn
    C = 2 is the (u_up, v_dn) block with mu = mu_up:
        H u = (h - mu) u + Delta v,   H v = Delta^* u - (h - mu) v.
    """
    Tpsi = kinetic(psi, lat)
    h = lambda c: Tpsi[:, c] + V * psi[:, c]
    out = np.empty_like(psi)
    Dc = np.conj(Delta)
    if fn.ncomp == 2:
        mu = fn.mu_up
        out[:, 0] = h(0) - mu * psi[:, 0] + Delta * psi[:, 1]
        out[:, 1] = Dc * psi[:, 0] - (h(1) - mu * psi[:, 1])
    else:
        mu_u, mu_d = fn.mu_up, fn.mu_dn
        out[:, 0] = h(0) - mu_u * psi[:, 0] + Delta * psi[:, 3]
        out[:, 1] = h(1) - mu_d * psi[:, 1] - Delta * psi[:, 2]
        out[:, 2] = -Dc * psi[:, 1] - (h(2) - mu_u * psi[:, 2])
        out[:, 3] = Dc * psi[:, 0] - (h(3) - mu_d * psi[:, 3])
    return out


def quasiparticle_energies(psi, V, Delta, lat, fn):
    """eta_k = <psi_k | H | psi_k> = a^3 sum_r sum_c psi_c^* (H psi)_c (Eq. sp_en).

    H is Hermitian, so eta_k is real; the real part of the sum is taken.
    """
    Hpsi = apply_h(psi, V, Delta, lat, fn)
    return lat.a ** 3 * np.real(np.sum(np.conj(psi) * Hpsi, axis=(1, 2, 3, 4)))


def apply_h_shifted(psi, V, Delta, lat, fn, eta):
    """(H - eta_k) psi_k for every qpwf k; eta None means plain H."""
    Hpsi = apply_h(psi, V, Delta, lat, fn)
    if eta is None:
        return Hpsi
    return Hpsi - eta[:, None, None, None, None] * psi


def hamiltonian_of(psi, lat, fn, t):
    """Local fields of the Hamiltonian built from the densities of psi at time t."""
    n, kappa = densities(psi, fn)
    return potentials(n, kappa, lat, fn, t)


def rhs(psi, lat, fn, t):
    """Right-hand side f(psi, t) = -i H[n(psi), kappa(psi), t] psi (Eq. tdslda, hbar = 1).

    With fn.remove_phase the trivial phase is removed (Eq. sp_en):
    f = -i (H - eta_k) psi_k with eta_k = <psi_k | H | psi_k> of this psi.
    """
    V, Delta = hamiltonian_of(psi, lat, fn, t)
    eta = quasiparticle_energies(psi, V, Delta, lat, fn) if getattr(fn, "remove_phase", 0) else None
    return -1j * apply_h_shifted(psi, V, Delta, lat, fn, eta)


# ---------------------------------------------------------------------------
# Series-expansion predictor-corrector (Sec. TDSLDA, "Time evolution")

def taylor_propagate(psi, V, Delta, lat, fn, dt, order=4, eta=None):
    """sum_{q=0}^{order} (-i dt (H - eta))^q / q! psi with H (and eta) fixed."""
    acc = psi.copy()
    term = psi
    for q in range(1, order + 1):
        term = (-1j * dt / q) * apply_h_shifted(term, V, Delta, lat, fn, eta)
        acc = acc + term
    return acc


def series_step(psi, lat, fn, t, dt, order=4):
    """One predictor-corrector step of the series-expansion propagator.

    1. H(t) from the densities of psi(t); predictor psi_pre = exp(-i H dt) psi.
    2. Corrector densities (n_pre + n(t)) / 2 give H_cor, taken at t + dt/2.
    3. psi(t + dt) = exp(-i H_cor dt) psi(t).
    The exponential is the order-4 series.  With phase removal (Eq. sp_en)
    each propagation uses H - eta with eta = <psi(t)|H|psi(t)> of the H of
    that propagation (H(t) for the predictor, H_cor for the corrector).
    """
    rp = getattr(fn, "remove_phase", 0)
    n0, k0 = densities(psi, fn)
    V, Delta = potentials(n0, k0, lat, fn, t)
    eta = quasiparticle_energies(psi, V, Delta, lat, fn) if rp else None
    pre = taylor_propagate(psi, V, Delta, lat, fn, dt, order, eta)
    n1, k1 = densities(pre, fn)
    Vc, Dc = potentials(0.5 * (n1 + n0), 0.5 * (k1 + k0), lat, fn, t + 0.5 * dt)
    eta_c = quasiparticle_energies(psi, Vc, Dc, lat, fn) if rp else None
    return taylor_propagate(psi, Vc, Dc, lat, fn, dt, order, eta_c)


# ---------------------------------------------------------------------------
# Adams-Bashforth-Milne predictor-modifier-corrector (Eq. p, m, c, y)

ABM_P = (119.0, -99.0, 69.0, -17.0)     # y'_n, y'_{n-1}, y'_{n-2}, y'_{n-3}
ABM_C = (17.0, 51.0, 3.0, 1.0)          # m'_{n+1}, y'_n, y'_{n-1}, y'_{n-2}
ABM_M = 161.0 / 170.0
ABM_Y = 9.0 / 170.0


def abm_update(y_n, y_nm1, dy, d_n, f_of_m, dt):
    """One ABM step for y' = f(y).

    dy = (y'_n, y'_{n-1}, y'_{n-2}, y'_{n-3}); d_n = p_n - c_n;
    f_of_m(m) evaluates f at the modifier (time t_{n+1}).
    Returns (y_{n+1}, d_{n+1}).
    """
    half = 0.5 * (y_n + y_nm1)
    p = half + (dt / 48.0) * (ABM_P[0] * dy[0] + ABM_P[1] * dy[1]
                              + ABM_P[2] * dy[2] + ABM_P[3] * dy[3])
    m = p - ABM_M * d_n
    dm = f_of_m(m)
    c = half + (dt / 48.0) * (ABM_C[0] * dm + ABM_C[1] * dy[0]
                              + ABM_C[2] * dy[1] + ABM_C[3] * dy[2])
    y_next = c + ABM_Y * (p - c)
    return y_next, p - c


class Evolver:
    """TDSLDA time evolution: series-expansion start-up, then ABM steps."""

    def __init__(self, lat, fn, psi0, t0=0.0):
        self.lat, self.fn = lat, fn
        self.y = np.array(psi0, dtype=np.complex128)
        self.t = float(t0)
        self.step_count = 0
        self.hist = None
        self.dt = None

    def f(self, psi, t):
        return rhs(psi, self.lat, self.fn, t)

    def startup(self, dt):
        """Three series-expansion steps; keeps y_3, y_2, y'_2, y'_1, y'_0 and d_3 = 0."""
        ys = [self.y]
        ds = []
        t = self.t
        for s in range(3):
            ds.append(self.f(ys[-1], t))
            ys.append(series_step(ys[-1], self.lat, self.fn, t, dt))
            t += dt
        self.hist = dict(y_n=ys[3], y_nm1=ys[2], dprev=[ds[2], ds[1], ds[0]],
                         d_n=np.zeros_like(ys[3]))
        self.y = ys[3]
        self.t = t
        self.dt = dt
        self.step_count += 3

    def abm_step(self):
        h, dt, t = self.hist, self.dt, self.t
        dy_n = self.f(h["y_n"], t)
        dy = (dy_n, h["dprev"][0], h["dprev"][1], h["dprev"][2])
        y_next, d_next = abm_update(h["y_n"], h["y_nm1"], dy, h["d_n"],
                                    lambda m: self.f(m, t + dt), dt)
        h["y_nm1"], h["y_n"] = h["y_n"], y_next
        h["dprev"] = [dy_n, h["dprev"][0], h["dprev"][1]]
        h["d_n"] = d_next
        self.y = y_next
        self.t = t + dt
        self.step_count += 1

    def checkpoint(self, with_history=True):
        """Copy of what a restart needs (Sec. Checkpoint and restart).

        The paper saves the latest qpwfs only and restarts with the series
        expansion; with_history additionally keeps y_{n-1}, the three previous
        derivatives and p_n - c_n, so that the ABM continues as if never
        interrupted.
        """
        ck = dict(y=self.y.copy(), t=self.t, step=self.step_count)
        if with_history and self.hist is not None:
            h = self.hist
            ck.update(y_nm1=h["y_nm1"].copy(), dprev=[d.copy() for d in h["dprev"]],
                      d_n=h["d_n"].copy(), dt=self.dt)
        return ck

    @classmethod
    def restore(cls, lat, fn, ck):
        """Evolver continuing from a checkpoint (start-up first when it holds no history)."""
        ev = cls(lat, fn, ck["y"], ck["t"])
        ev.step_count = ck["step"]
        if "d_n" in ck:
            ev.hist = dict(y_n=ev.y, y_nm1=ck["y_nm1"].copy(), dprev=[d.copy() for d in ck["dprev"]],
                           d_n=ck["d_n"].copy())
            ev.dt = ck["dt"]
        return ev

    def step(self, dt, nsteps):
        """Advance nsteps ABM steps; the start-up runs first when needed."""
        if self.hist is None or self.dt != dt:
            self.hist = None
            self.startup(dt)
        for _ in range(nsteps):
            self.abm_step()


# ---------------------------------------------------------------------------
# Observables (Sec. Miscellaneous quantities; the cold-atom energy)

def observables(psi, lat, fn, t):
    """Particle number, energy and its parts, mean gap, centre of mass, norms.

    E = E_kin + E_int + E_pair + E_ext with
      E_kin  = a^3 sum_r [weight * sum_k v_k^* (T v_k)]   (same T as the step),
      E_int  = a^3 sum_r (3/5) beta n^{5/3}   (so that dE/dn = U),
      E_pair = a^3 sum_r g |kappa|^2          (Eq. pairing; g_eff when regularised),
      E_ext  = a^3 sum_r U_ext n.
    <|Delta|> = int |Delta| n / int n; r_cm = int r n / int n.
    P = int j (total current, Eq. j) and v_cm = P / N (Eq. vel with m = hbar = 1).
    Spin-resolved numbers from the spin sum of Eq. (rho_t): N_sigma = int sum_k
    |v_{k,sigma}|^2, i.e. the v_up and v_dn components for C = 4.  The C = 2
    reduction is spin-symmetric by construction (each state of the (u_up, v_dn)
    block stands for itself and its time-reversed partner): N_up = N_dn = N / 2.
    """
    a3 = lat.a ** 3
    n, kappa = densities(psi, fn)
    V, Delta = potentials(n, kappa, lat, fn, t)
    Uext = external_potential(lat, fn, t)
    if fn.ncomp == 2:
        vs, wt = [1], fn.w
    else:
        vs, wt = [2, 3], 1.0
    ekin = 0.0
    for c in vs:
        ekin += wt * a3 * float(np.sum(np.real(np.conj(psi[:, c]) * kinetic(psi[:, c], lat))))
    N = a3 * float(np.sum(n))
    e_int = a3 * float(np.sum(0.6 * fn.beta * np.cbrt(n) ** 5))
    e_pair = a3 * float(np.sum(effective_coupling(fn, lat) * np.abs(kappa) ** 2))
    e_ext = a3 * float(np.sum(Uext * n))
    xs = [np.arange(m) * lat.a for m in (lat.nx, lat.ny, lat.nz)]
    tot = float(np.sum(n))
    rcm = [float(np.sum(n * xs[0][None, None, :])) / tot if tot else 0.0,
           float(np.sum(n * xs[1][None, :, None])) / tot if tot else 0.0,
           float(np.sum(n * xs[2][:, None, None])) / tot if tot else 0.0]
    norms = a3 * np.sum(np.abs(psi) ** 2, axis=(1, 2, 3, 4))
    if fn.ncomp == 4:
        n_up = a3 * float(np.sum(np.abs(psi[:, 2]) ** 2))
        n_dn = a3 * float(np.sum(np.abs(psi[:, 3]) ** 2))
    else:
        n_up = n_dn = 0.5 * N
    P = [a3 * float(np.sum(c)) for c in current_density(psi, lat, fn)]
    return dict(t=t, N=N, N_up=n_up, N_dn=n_dn, E=ekin + e_int + e_pair + e_ext, E_kin=ekin, E_int=e_int,
                E_pair=e_pair, E_ext=e_ext,
                mean_abs_delta=float(np.sum(np.abs(Delta) * n)) / tot if tot else 0.0,
                r_cm=rcm, norms=norms, P=P, v_cm=[p / N if N else 0.0 for p in P])


def gram(psi, lat):
    """Overlap matrix S_ij = <psi_i | psi_j> = a^3 sum_c sum_r psi_i^* psi_j."""
    m = psi.reshape(psi.shape[0], -1)
    return lat.a ** 3 * (np.conj(m) @ m.T)
