"""Python binding of liblise (ctypes, argument marshalling only).

Every computation runs in the HIP kernels of liblise.so.  The binding loads
the in-tree library and raises if it is missing; there is no fallback.
Device buffers passed in or out may be PyTorch tensors (their data_ptr is
used) or NumPy arrays (host memory).
"""
import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblise.so")

LISE_FP64, LISE_FP32, LISE_FP32_MFMA = 0, 1, 2
ERRORS = {0: "OK", -1: "LISE_E_ARG", -2: "LISE_E_NOMEM", -3: "LISE_E_UNSUPPORTED",
          -4: "LISE_E_HIP", -5: "LISE_E_STATE", -6: "LISE_E_NAN"}

# every entry point declared in include/lise.h
SYMBOLS = ["lise_init", "lise_set_qpwf", "lise_get_qpwf", "lise_apply_h", "lise_apply_h_noalloc", "lise_startup",
           "lise_step", "lise_densities", "lise_observables", "lise_get_time", "lise_set_time",
           "lise_set_stream", "lise_set_tuning", "lise_profile", "lise_profile_read",
           "lise_memory", "lise_last_error", "lise_version", "lise_free", "lise_autotune", "lise_coupling",
           "lise_save", "lise_load", "lise_kick", "lise_current",
           "lise_batch_create", "lise_batch_step", "lise_batch_set_graph", "lise_batch_info",
           "lise_batch_profile", "lise_batch_profile_read", "lise_batch_last_error", "lise_batch_free"]


class Lattice(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32),
                ("reserved", ct.c_int32), ("a", ct.c_double)]


class Functional(ct.Structure):
    _fields_ = [("ncomp", ct.c_int32), ("precision", ct.c_int32),
                ("mu_up", ct.c_double), ("mu_dn", ct.c_double),
                ("beta", ct.c_double), ("g", ct.c_double), ("w", ct.c_double),
                ("frozen", ct.c_int32), ("regularize", ct.c_int32),
                ("U0", ct.c_double), ("Delta0_re", ct.c_double), ("Delta0_im", ct.c_double),
                ("ext_A", ct.c_double), ("ext_w", ct.c_double),
                ("ext_r0", ct.c_double * 3), ("ext_t_on", ct.c_double),
                ("remove_phase", ct.c_int32), ("reserved", ct.c_int32)]


class Obs(ct.Structure):
    _fields_ = [("t", ct.c_double), ("step", ct.c_int64),
                ("N", ct.c_double), ("E", ct.c_double), ("E_kin", ct.c_double),
                ("E_int", ct.c_double), ("E_pair", ct.c_double), ("E_ext", ct.c_double),
                ("mean_abs_delta", ct.c_double), ("r_cm", ct.c_double * 3),
                ("norm_drift_max", ct.c_double), ("norm_drift_mean", ct.c_double),
                ("P", ct.c_double * 3), ("v_cm", ct.c_double * 3),
                ("N_up", ct.c_double), ("N_dn", ct.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        for k in ("r_cm", "P", "v_cm"):
            d[k] = list(getattr(self, k))
        return d


class Tuning(ct.Structure):
    _fields_ = [("chunk_qpwf", ct.c_int32), ("jgroup", ct.c_int32),
                ("fused", ct.c_int32), ("generic", ct.c_int32),
                ("no_overlap", ct.c_int32), ("graph", ct.c_int32),
                ("single_pass", ct.c_int32), ("z_lanes", ct.c_int32),
                ("z_dense", ct.c_int32)]


_lib = None


def load_library(path=LIB_PATH):
    """Load liblise.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"liblise.so not found at {path}: build it with "
                           "`python -m paper_2009_00745_amd.build` (no CPU fallback exists)")
    lib = ct.CDLL(path)
    P = ct.c_void_p
    sig = {
        "lise_init": ([ct.POINTER(P), ct.POINTER(Lattice), ct.c_int64, ct.POINTER(Functional), P], ct.c_int),
        "lise_set_qpwf": ([P, ct.c_int64, ct.c_int64, P, ct.c_int32], ct.c_int),
        "lise_get_qpwf": ([P, ct.c_int64, ct.c_int64, P, ct.c_int32], ct.c_int),
        "lise_apply_h": ([P, ct.c_int64, ct.c_int64, P, ct.c_int32], ct.c_int),
        "lise_apply_h_noalloc": ([P, ct.c_int64, ct.c_int64, P], ct.c_int),
        "lise_startup": ([P, ct.c_double], ct.c_int),
        "lise_step": ([P, ct.c_double, ct.c_int64], ct.c_int),
        "lise_densities": ([P, P, P, ct.c_int32], ct.c_int),
        "lise_observables": ([P, ct.POINTER(Obs)], ct.c_int),
        "lise_get_time": ([P, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64)], ct.c_int),
        "lise_set_time": ([P, ct.c_double], ct.c_int),
        "lise_set_stream": ([P, P], ct.c_int),
        "lise_set_tuning": ([P, ct.POINTER(Tuning)], ct.c_int),
        "lise_profile": ([P, ct.c_int32], ct.c_int),
        "lise_profile_read": ([P, ct.c_int32, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double)], ct.c_int),
        "lise_memory": ([P, ct.POINTER(ct.c_int64)], ct.c_int),
        "lise_last_error": ([P], ct.c_char_p),
        "lise_version": ([], ct.c_char_p),
        "lise_free": ([P], None),
        "lise_autotune": ([P, ct.c_double, ct.c_int32, ct.POINTER(Tuning)], ct.c_int),
        "lise_kick": ([P, P, ct.c_int32], ct.c_int),
        "lise_current": ([P, P, ct.c_int32], ct.c_int),
        "lise_save": ([P, ct.c_char_p, ct.c_int32], ct.c_int),
        "lise_load": ([P, ct.c_char_p], ct.c_int),
        "lise_coupling": ([ct.POINTER(Lattice), ct.POINTER(Functional), ct.POINTER(ct.c_double)], ct.c_int),
        "lise_batch_create": ([ct.POINTER(P), ct.c_int32, ct.POINTER(P), P], ct.c_int),
        "lise_batch_step": ([P, ct.c_double, ct.c_int64], ct.c_int),
        "lise_batch_set_graph": ([P, ct.c_int32], ct.c_int),
        "lise_batch_info": ([P, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)], ct.c_int),
        "lise_batch_profile": ([P, ct.c_int32], ct.c_int),
        "lise_batch_profile_read": ([P, ct.c_int32, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double)], ct.c_int),
        "lise_batch_last_error": ([P], ct.c_char_p),
        "lise_batch_free": ([P], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


class LiseError(RuntimeError):
    pass


def functional_struct(f):
    """lise_functional from an object with the fields of workloads.Functional."""
    d0 = complex(f.Delta0)
    return Functional(f.ncomp, f.precision, f.mu_up, f.mu_dn, f.beta, f.g, f.w,
                      int(f.frozen), int(getattr(f, "regularize", 0)), f.U0, d0.real, d0.imag,
                      f.ext_A, f.ext_w, (ct.c_double * 3)(*f.ext_r0), f.ext_t_on,
                      int(getattr(f, "remove_phase", 0)), 0)


def coupling(lattice, functional):
    """The coupling g of Delta = -g kappa that the library uses (host-only call)."""
    lib = load_library()
    lat = Lattice(lattice.nx, lattice.ny, lattice.nz, 0, lattice.a)
    fn = functional_struct(functional)
    g = ct.c_double()
    rc = lib.lise_coupling(ct.byref(lat), ct.byref(fn), ct.byref(g))
    if rc != 0:
        raise LiseError(f"lise_coupling: {ERRORS.get(rc, rc)}")
    return g.value


def _ptr(x):
    """(address, is_device) of a torch tensor or a NumPy array."""
    if hasattr(x, "data_ptr"):
        return ct.c_void_p(x.data_ptr()), int(x.is_cuda)
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return ct.c_void_p(x.ctypes.data), 0
    raise TypeError("expected a torch tensor or a numpy array")


class Context:
    """One TDSLDA system on the current HIP device (see include/lise.h)."""

    def __init__(self, lattice, n_qpwf, functional, stream=None):
        self.lib = load_library()
        self.nx, self.ny, self.nz = lattice.nx, lattice.ny, lattice.nz
        self.a = lattice.a
        self.M = int(n_qpwf)
        self.C = int(functional.ncomp)
        self.N = self.nx * self.ny * self.nz
        lat = Lattice(lattice.nx, lattice.ny, lattice.nz, 0, lattice.a)
        fn = functional_struct(functional)
        self._h = ct.c_void_p()
        rc = self.lib.lise_init(ct.byref(self._h), ct.byref(lat), self.M, ct.byref(fn),
                                ct.c_void_p(stream or 0))
        if rc != 0:
            raise LiseError(f"lise_init failed: {ERRORS.get(rc, rc)}")

    def _check(self, rc, what):
        if rc != 0:
            msg = self.lib.lise_last_error(self._h).decode()
            raise LiseError(f"{what}: {ERRORS.get(rc, rc)}: {msg}")

    def close(self):
        if self._h:
            self.lib.lise_free(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_qpwf(self, first, data):
        p, dev = _ptr(data)
        count = data.shape[0]
        self._check(self.lib.lise_set_qpwf(self._h, first, count, p, dev), "lise_set_qpwf")

    def get_qpwf(self, first, count, out=None):
        if out is None:
            out = np.empty((count, self.C, self.nz, self.ny, self.nx), dtype=np.complex128)
        p, dev = _ptr(out)
        self._check(self.lib.lise_get_qpwf(self._h, first, count, p, dev), "lise_get_qpwf")
        return out

    def apply_h(self, first, count, out=None):
        if out is None:
            out = np.empty((count, self.C, self.nz, self.ny, self.nx), dtype=np.complex128)
        p, dev = _ptr(out)
        self._check(self.lib.lise_apply_h(self._h, first, count, p, dev), "lise_apply_h")
        return out

    def apply_h_noalloc(self, first, count, out):
        """H psi into `out` (a device tensor of count*C*N complex128), staged through the
        library's fixed per-GPU array: the call allocates nothing."""
        p, dev = _ptr(out)
        if not dev:
            raise ValueError("apply_h_noalloc writes device memory only")
        self._check(self.lib.lise_apply_h_noalloc(self._h, first, count, p), "lise_apply_h_noalloc")
        return out

    def startup(self, dt):
        self._check(self.lib.lise_startup(self._h, dt), "lise_startup")

    def step(self, dt, nsteps):
        self._check(self.lib.lise_step(self._h, dt, nsteps), "lise_step")

    def densities(self):
        n = np.empty((self.nz, self.ny, self.nx), dtype=np.float64)
        k = np.empty((self.nz, self.ny, self.nx), dtype=np.complex128)
        self._check(self.lib.lise_densities(self._h, ct.c_void_p(n.ctypes.data),
                                            ct.c_void_p(k.ctypes.data), 0), "lise_densities")
        return n, k

    def observables(self):
        o = Obs()
        self._check(self.lib.lise_observables(self._h, ct.byref(o)), "lise_observables")
        return o.as_dict()

    def time(self):
        t = ct.c_double()
        s = ct.c_int64()
        self._check(self.lib.lise_get_time(self._h, ct.byref(t), ct.byref(s)), "lise_get_time")
        return t.value, s.value

    def set_time(self, t):
        self._check(self.lib.lise_set_time(self._h, t), "lise_set_time")

    def set_stream(self, stream):
        self._check(self.lib.lise_set_stream(self._h, ct.c_void_p(stream or 0)), "lise_set_stream")

    def set_tuning(self, chunk_qpwf=0, jgroup=0, fused=0, generic=0, no_overlap=0, graph=0, single_pass=0,
                   z_lanes=0, z_dense=0):
        t = Tuning(chunk_qpwf, jgroup, fused, generic, no_overlap, graph, single_pass, z_lanes, z_dense)
        self._check(self.lib.lise_set_tuning(self._h, ct.byref(t)), "lise_set_tuning")

    def profile(self, enable):
        self._check(self.lib.lise_profile(self._h, int(enable)), "lise_profile")

    def profile_read(self, which):
        n = ct.c_int64()
        ms = ct.c_double()
        self._check(self.lib.lise_profile_read(self._h, which, ct.byref(n), ct.byref(ms)),
                    "lise_profile_read")
        return n.value, ms.value

    def autotune(self, dt, trial_steps=2):
        t = Tuning()
        self._check(self.lib.lise_autotune(self._h, dt, trial_steps, ct.byref(t)), "lise_autotune")
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def kick(self, chi):
        """Eq. (kick) with the real phase field chi (shape (nz, ny, nx) or N values)."""
        chi = np.ascontiguousarray(np.asarray(chi, dtype=np.float64).reshape(-1))
        if chi.size != self.nx * self.ny * self.nz:
            raise ValueError("chi must hold one value per lattice point")
        self._check(self.lib.lise_kick(self._h, chi.ctypes.data, 0), "lise_kick")

    def current(self):
        """Current density of Eq. (j) as an array (3, nz, ny, nx): j_x, j_y, j_z."""
        out = np.empty((3, self.nz, self.ny, self.nx), dtype=np.float64)
        self._check(self.lib.lise_current(self._h, out.ctypes.data, 0), "lise_current")
        return out

    def save(self, path, with_history=True):
        """Write a checkpoint file (with the ABM history: bit-exact continuation)."""
        self._check(self.lib.lise_save(self._h, os.fsencode(path), int(bool(with_history))), "lise_save")

    def load(self, path):
        """Read a checkpoint written by save() for the same lattice, C, M and precision."""
        self._check(self.lib.lise_load(self._h, os.fsencode(path)), "lise_load")

    def memory(self):
        b = ct.c_int64()
        self._check(self.lib.lise_memory(self._h, ct.byref(b)), "lise_memory")
        return b.value


class Batch:
    """Independent systems advanced together: systems of one lattice side and
    precision share one z-axis and one plane-kernel launch per ABM phase, and
    four steps replay as one captured graph."""

    def __init__(self, contexts, stream=None):
        self.lib = load_library()
        self.contexts = list(contexts)
        arr = (ct.c_void_p * len(self.contexts))(*[c._h.value for c in self.contexts])
        self._h = ct.c_void_p()
        rc = self.lib.lise_batch_create(ct.byref(self._h), len(self.contexts), arr, ct.c_void_p(stream or 0))
        if rc != 0:
            raise LiseError(f"lise_batch_create failed: {ERRORS.get(rc, rc)}")

    def _check(self, rc, what):
        if rc != 0:
            msg = self.lib.lise_batch_last_error(self._h).decode()
            raise LiseError(f"{what}: {ERRORS.get(rc, rc)}: {msg}")

    def step(self, dt, nsteps):
        self._check(self.lib.lise_batch_step(self._h, dt, nsteps), "lise_batch_step")

    def set_graph(self, enable):
        self._check(self.lib.lise_batch_set_graph(self._h, int(bool(enable))), "lise_batch_set_graph")

    def info(self):
        """(number of groups, number of systems stepped one by one) of the last step."""
        g, s = ct.c_int32(), ct.c_int32()
        self._check(self.lib.lise_batch_info(self._h, ct.byref(g), ct.byref(s)), "lise_batch_info")
        return g.value, s.value

    def profile(self, enable):
        self._check(self.lib.lise_batch_profile(self._h, int(bool(enable))), "lise_batch_profile")

    def profile_read(self, which):
        """(launches, total ms) of kernel class which: 0 plane kernel of ABM phase 1,
        1 z axis, 2 fields, 3 plane kernel of ABM phase 2."""
        n, ms = ct.c_int64(), ct.c_double()
        self._check(self.lib.lise_batch_profile_read(self._h, which, ct.byref(n), ct.byref(ms)),
                    "lise_batch_profile_read")
        return n.value, ms.value

    def close(self):
        if self._h:
            self.lib.lise_batch_free(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version():
    return load_library().lise_version().decode()
