"""Seeded synthetic cold-atom workloads (initial quasiparticle wavefunctions).

These inputs stand in for the nuclear qpwfs of the paper's test cases, which
come from a static solver and NEDF parameter sets that are not available.
Every workload is a unitary-Fermi-gas-like superfluid on a periodic cubic
lattice built from BCS plane-wave states, optionally perturbed by the
multiplicative noise model of the paper's noise study (Sec. "Various numerical
tests", Eq. noise).  Nothing here performs the time step: this module only
builds inputs, which both the oracle and the GPU library consume.

Layout of a qpwf array: complex128, shape (count, C, nz, ny, nx); C = 2 is
(u, v), C = 4 is (u_up, u_dn, v_up, v_dn).  Normalisation a^3 sum |psi|^2 = 1.
"""
from dataclasses import dataclass, field, asdict
import math
import numpy as np

from . import rng

FP64, FP32, FP32_MFMA = 0, 1, 2


@dataclass
class Lattice:
    nx: int
    ny: int
    nz: int
    a: float = 1.0

    @property
    def n(self):
        return self.nx * self.ny * self.nz


@dataclass
class Functional:
    ncomp: int = 2
    mu_up: float = 0.0
    mu_dn: float = 0.0
    beta: float = 0.37
    g: float = 0.0
    w: float = 2.0
    frozen: int = 0
    regularize: int = 0
    U0: float = 0.0
    Delta0: complex = 0j
    ext_A: float = 0.0
    ext_w: float = 1.0
    ext_r0: tuple = (0.0, 0.0, 0.0)
    ext_t_on: float = 0.0
    remove_phase: int = 0
    precision: int = FP64

    def as_dict(self):
        return asdict(self)


@dataclass
class Workload:
    name: str
    lattice: Lattice
    functional: Functional
    M: int
    dt: float
    steps: int
    gen: object = field(repr=False, default=None)
    seed: int = 0
    notes: str = ""

    def qpwfs(self, first=0, count=None):
        if count is None:
            count = self.M - first
        if first < 0 or first + count > self.M:
            raise ValueError("qpwf range out of bounds")
        return self.gen(first, count)


# ----------------------------------------------------------------------------
# plane-wave basis helpers (input construction only)

def signed_index(n):
    i = np.arange(n)
    return np.where(i < n // 2, i, i - n)


def k_order(lat):
    """All lattice momenta ordered by |k|^2, then by pair {n, -n}.

    Returns an int array (N, 3) of signed integer indices (nx_s, ny_s, nz_s).
    Ties in |k| are broken by the smaller flat FFT index of the pair {n, -n},
    and within a pair the member with the smaller flat index comes first, so
    that +k and -k stay adjacent.
    """
    L = math.lcm(lat.nx, lat.ny, lat.nz)
    sz, sy, sx = np.meshgrid(signed_index(lat.nz), signed_index(lat.ny),
                             signed_index(lat.nx), indexing="ij")
    sx, sy, sz = sx.ravel(), sy.ravel(), sz.ravel()
    k2 = (sx * (L // lat.nx)) ** 2 + (sy * (L // lat.ny)) ** 2 + (sz * (L // lat.nz)) ** 2
    flat = (sz % lat.nz) * lat.ny * lat.nx + (sy % lat.ny) * lat.nx + (sx % lat.nx)
    neg = ((-sz) % lat.nz) * lat.ny * lat.nx + ((-sy) % lat.ny) * lat.nx + ((-sx) % lat.nx)
    pair = np.minimum(flat, neg)
    order = np.lexsort((flat, pair, k2))
    return np.stack([sx[order], sy[order], sz[order]], axis=1)


def k_of(lat, idx):
    """Physical momenta (count, 3) for signed integer indices (count, 3)."""
    dims = np.array([lat.nx, lat.ny, lat.nz], dtype=np.float64)
    return 2.0 * np.pi * idx / (dims * lat.a)


def plane_waves(lat, idx):
    """exp(i k.r)/sqrt(N a^3) for each row of idx; shape (count, nz, ny, nx)."""
    k = k_of(lat, idx)
    x = np.arange(lat.nx) * lat.a
    y = np.arange(lat.ny) * lat.a
    z = np.arange(lat.nz) * lat.a
    px = np.exp(1j * k[:, 0:1] * x[None, :])
    py = np.exp(1j * k[:, 1:2] * y[None, :])
    pz = np.exp(1j * k[:, 2:3] * z[None, :])
    norm = 1.0 / math.sqrt(lat.n * lat.a ** 3)
    return norm * pz[:, :, None, None] * py[:, None, :, None] * px[:, None, None, :]


def bcs_uv(xi, delta_abs):
    """Positive-branch BCS amplitudes u, v >= 0 for xi and |Delta|."""
    xi = np.asarray(xi, dtype=np.float64)
    d = np.asarray(delta_abs, dtype=np.float64)
    e = np.sqrt(xi * xi + d * d)
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.where(e > 0, xi / np.where(e > 0, e, 1.0), 0.0)
    return np.sqrt(0.5 * (1.0 + r)), np.sqrt(0.5 * (1.0 - r))


def noise_factors(seed, system, j, ncomp, npts, eps):
    """(1 + eps*alpha) per (j, c, r); alpha complex with Re, Im uniform on [-1, 1)."""
    base = rng.key(seed, rng.STREAM_NOISE, system)
    kj = rng.splitmix64(base ^ np.asarray(j, dtype=np.uint64))[:, None, None]
    kc = rng.splitmix64(kj ^ np.arange(ncomp, dtype=np.uint64)[None, :, None])
    kr = rng.splitmix64(kc ^ np.arange(npts, dtype=np.uint64)[None, None, :])
    re = rng.uniform_pm1(kr ^ np.uint64(0))
    im = rng.uniform_pm1(kr ^ np.uint64(1))
    return 1.0 + eps * (re + 1j * im)


def phase_noise(seed, system, j, ncomp, npts, eps):
    """exp(i*eps*theta) per (j, c, r), theta uniform on [-1, 1)."""
    base = rng.key(seed, rng.STREAM_PHASE, system)
    kj = rng.splitmix64(base ^ np.asarray(j, dtype=np.uint64))[:, None, None]
    kc = rng.splitmix64(kj ^ np.arange(ncomp, dtype=np.uint64)[None, :, None])
    kr = rng.splitmix64(kc ^ np.arange(npts, dtype=np.uint64)[None, None, :])
    return np.exp(1j * eps * rng.uniform_pm1(kr))


def seeded_lattice_point(seed, system, lat):
    k = rng.key(seed, rng.STREAM_BUMP, system)
    ks = [rng.splitmix64(k ^ np.uint64(i)) for i in range(3)]
    dims = (lat.nx, lat.ny, lat.nz)
    return tuple(float(min(int(rng.uniform01(kk) * d), d - 1)) * lat.a for kk, d in zip(ks, dims))


# ----------------------------------------------------------------------------
# generic builders

def uniform_bcs(lat, fn, M, delta0, mu, order="lowest", copies=1, eps=0.0,
                seed=0, system=0, xi_shift=0.0):
    """Uniform BCS states (u_k, v_k) e^{ik.r}/sqrt(V) on the M lowest |k| (C = 2).

    With copies > 1, the first M/copies momenta are each used `copies` times
    (j = copy*(M/copies) + rank), each copy with its own noise.
    """
    per = M // copies
    if per * copies != M:
        raise ValueError("M must be divisible by copies")
    ks = k_order(lat)
    if per > len(ks):
        raise ValueError("more states than lattice momenta")
    ks = ks[:per]
    k2 = np.sum(k_of(lat, ks) ** 2, axis=1)
    u, v = bcs_uv(0.5 * k2 - mu + xi_shift, abs(delta0))
    ph = delta0 / abs(delta0) if abs(delta0) > 0 else 1.0

    def gen(first, count):
        j = np.arange(first, first + count)
        rank = j % per
        pw = plane_waves(lat, ks[rank])
        out = np.empty((count, 2, lat.nz, lat.ny, lat.nx), dtype=np.complex128)
        out[:, 0] = u[rank, None, None, None] * pw
        out[:, 1] = (v[rank] * np.conj(ph))[:, None, None, None] * pw
        if eps:
            out *= noise_factors(seed, system, j, 2, lat.n, eps).reshape(out.shape)
        return out
    return gen


# ----------------------------------------------------------------------------
# the five benchmark workloads

def config1(seed=0, M=None):
    """8^3, FP64, M = 1024 = every BCS momentum twice, w = 1, noise 1e-3."""
    lat = Lattice(8, 8, 8, 1.0)
    fn = Functional(ncomp=2, mu_up=1.0, mu_dn=1.0, beta=0.37, g=1.5, w=1.0)
    M = 1024 if M is None else M
    copies = 2 if M % 2 == 0 else 1
    gen = uniform_bcs(lat, fn, M, 0.5, 1.0, copies=copies, eps=1e-3, seed=seed)
    return Workload(f"cfg1_fp64_8c_m{M}", lat, fn, M, 0.005, 100, gen, seed,
                    "8^3 uniform BCS, both spin blocks explicit (w=1), 1e-3 noise")


def config2(seed=0, M=None, n=32, steps=500):
    """32^3, FP64, M = 8192 lowest-|k| BCS states, w = 2, Gaussian bump."""
    lat = Lattice(n, n, n, 1.0)
    mu = 0.5
    r0 = seeded_lattice_point(seed, 0, lat)
    fn = Functional(ncomp=2, mu_up=mu, mu_dn=mu, beta=0.37, g=2.0, w=2.0,
                    ext_A=-0.05 * mu, ext_w=3.0, ext_r0=r0, ext_t_on=100 * 0.002)
    M = 8192 if M is None else M
    gen = uniform_bcs(lat, fn, M, 0.3, mu)
    return Workload(f"cfg2_fp64_{n}c_m{M}", lat, fn, M, 0.002, steps, gen, seed,
                    "lowest-|k| BCS states plus ramped Gaussian external well")


def config3(seed=0, M=None, n=48, steps=1000, precision=FP32):
    """48^3, FP32 bulk, M = 16384, LDA vortex line along z, phase noise 1e-3."""
    lat = Lattice(n, n, n, 1.0)
    mu = 0.5
    fn = Functional(ncomp=2, mu_up=mu, mu_dn=mu, beta=0.37, g=2.0, w=2.0,
                    precision=precision)
    M = 16384 if M is None else M
    ks = k_order(lat)[:M]
    k2 = np.sum(k_of(lat, ks) ** 2, axis=1)
    c = (lat.nx / 2 - 0.5) * lat.a
    x = np.arange(lat.nx) * lat.a - c
    y = np.arange(lat.ny) * lat.a - c
    X, Y = np.meshgrid(x, y, indexing="xy")          # (ny, nx)
    rho = np.sqrt(X * X + Y * Y)
    phi = np.arctan2(Y, X)
    dabs = 0.4 * np.tanh(rho / 2.0)                     # |Delta(r)|, same for all z
    eu = np.exp(0.5j * phi)

    def gen(first, count):
        j = np.arange(first, first + count)
        pw = plane_waves(lat, ks[j])
        u, v = bcs_uv(0.5 * k2[j][:, None, None] - mu, dabs[None])   # (count, ny, nx)
        out = np.empty((count, 2, lat.nz, lat.ny, lat.nx), dtype=np.complex128)
        out[:, 0] = (u * eu[None])[:, None] * pw
        out[:, 1] = (v * np.conj(eu)[None])[:, None] * pw
        out *= phase_noise(seed, 0, j, 2, lat.n, 1e-3).reshape(out.shape)
        return out
    return Workload(f"cfg3_{('fp64', 'fp32', 'mfma')[precision]}_{n}c_m{M}", lat, fn, M, 0.002, steps, gen, seed,
                    "LDA vortex Delta=0.4 tanh(rho/2) e^{i phi}, phase noise 1e-3")


def config4(seed=0, M=None, n=64, steps=200, precision=FP32_MFMA):
    """64^3, C = 4, M = 4096 spin-imbalanced BCS states, Delta0 = 0.25."""
    lat = Lattice(n, n, n, 1.0)
    fn = Functional(ncomp=4, mu_up=0.6, mu_dn=0.4, beta=0.37, g=2.0, w=1.0,
                    precision=precision)
    M = 4096 if M is None else M
    half = M // 2
    kd = rng.key(seed, rng.STREAM_IMBALANCE, 0)
    dmax = min(256, half - 2)
    dmin = min(64, dmax)
    delta = dmin + 2 * int(rng.uniform01(kd) * ((dmax - dmin) // 2 + 1))
    delta = min(delta, dmax) & ~1
    na, nb = half + delta, M - half - delta
    ks = k_order(lat)
    mubar = 0.5 * (fn.mu_up + fn.mu_dn)

    def uv(idx):
        k2 = np.sum(k_of(lat, idx) ** 2, axis=1)
        return bcs_uv(0.5 * k2 - mubar, 0.25)

    ua, va = uv(ks[:na])
    ub, vb = uv(ks[:nb])

    def gen(first, count):
        j = np.arange(first, first + count)
        out = np.zeros((count, 4, lat.nz, lat.ny, lat.nx), dtype=np.complex128)
        kg = rng.key(seed, rng.STREAM_GLOBAL_PHASE, 0)
        th = 2 * np.pi * rng.uniform01(rng.splitmix64(kg ^ j.astype(np.uint64)))
        gph = np.exp(1j * th)
        isa = j < na
        ia = j[isa]
        ib = j[~isa] - na
        if ia.size:
            pw = plane_waves(lat, ks[ia]) * gph[isa][:, None, None, None]
            out[isa, 0] = ua[ia, None, None, None] * pw
            out[isa, 3] = va[ia, None, None, None] * pw
        if ib.size:
            pw = plane_waves(lat, ks[ib]) * gph[~isa][:, None, None, None]
            out[~isa, 1] = ub[ib, None, None, None] * pw
            out[~isa, 2] = -vb[ib, None, None, None] * pw
        out *= noise_factors(seed, 0, j, 4, lat.n, 1e-3).reshape(out.shape)
        return out
    wl = Workload(f"cfg4_c4_{n}c_m{M}", lat, fn, M, 0.002, steps, gen, seed,
                  f"spin-imbalanced: {na} up-pair states, {nb} down-pair states")
    wl.imbalance = delta
    return wl


def config5_systems(seed=0, nsys=64, scale=1.0):
    """Batched workload: nsys independent systems of uneven size (FP32)."""
    out = []
    for s in range(nsys):
        k = rng.key(seed, rng.STREAM_SYSTEM, s)
        r = [rng.uniform01(rng.splitmix64(k ^ np.uint64(i))) for i in range(3)]
        n = (16, 20, 24)[min(int(r[0] * 3), 2)]
        M = 512 + int(r[1] * (3072 - 512 + 1))
        M = max(2, int(M * scale)) & ~1
        M = min(M, n ** 3)
        d0 = 0.1 + 0.5 * float(r[2])
        lat = Lattice(n, n, n, 1.0)
        fn = Functional(ncomp=2, mu_up=0.5, mu_dn=0.5, beta=0.37, g=2.0, w=2.0,
                        precision=FP32)
        gen = uniform_bcs(lat, fn, M, d0, 0.5)
        out.append(Workload(f"cfg5_sys{s}_{n}c_m{M}", lat, fn, M, 0.002, 300, gen, seed,
                            f"batched system {s}: Delta0={d0:.4f}"))
    return out
