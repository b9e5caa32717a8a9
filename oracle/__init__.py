"""FP64 CPU oracle of the hybrid LB/FD lamellar-fluid model (arXiv:1102.3094).

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
import this package; the GPU library never does, and this package never imports the GPU one.

``Oracle`` wraps the C library ``liblam_oracle.so`` (time stepping, force, observables);
``spectra`` holds the structure factor and orientation histogram in numpy.  Parameters are plain
dicts with the keys of ``synthetic.MODEL_KEYS`` (plus ``n_phi_sub``, ``n_T_sub``, ``force_form``,
``body_force``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB_PATH, build as _build
from .spectra import orientation, structure_factor  # noqa: F401

_lib = None
_lib_path = LIB_PATH


def use_library(path: str) -> None:
    """Load the oracle from another build of the same source (the CPU baseline's -O3
    -march=native build); only before the first use in the process."""
    global _lib_path
    if _lib is not None and path != _lib_path:
        raise RuntimeError("the oracle library is already loaded from " + _lib_path)
    _lib_path = path


class orc_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("walls", C.c_int32), ("hydro", C.c_int32),
                ("tau", C.c_double), ("Gamma", C.c_double), ("b", C.c_double),
                ("kappa", C.c_double), ("c", C.c_double),
                ("Tc", C.c_double), ("T0", C.c_double), ("Tw", C.c_double), ("xi", C.c_double),
                ("n_phi_sub", C.c_int32), ("n_T_sub", C.c_int32), ("force_form", C.c_int32),
                ("pad_", C.c_int32), ("body_force", C.c_double * 3)]


class orc_obs(C.Structure):
    _fields_ = [("mass_dev", C.c_double), ("mom", C.c_double * 3), ("phi_sum", C.c_double),
                ("max_u", C.c_double), ("mach", C.c_double), ("free_energy", C.c_double),
                ("step", C.c_int64), ("nonfinite", C.c_int32), ("pad_", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if _lib_path == LIB_PATH and not os.path.exists(LIB_PATH):
            _build()
        L = C.CDLL(_lib_path)
        dp = C.POINTER(C.c_double)
        L.orc_create.argtypes = [C.POINTER(orc_params), C.POINTER(C.c_void_p)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_destroy.restype = None
        L.orc_substeps.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.orc_lattice.argtypes = [C.c_int32, C.POINTER(C.c_int32), dp, C.POINTER(C.c_int32)]
        L.orc_init_fields.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_observables.argtypes = [C.c_void_p, C.POINTER(orc_obs)]
        L.orc_get_fields.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_get_populations.argtypes = [C.c_void_p, dp]
        L.orc_eval_mu.argtypes = [C.c_void_p, dp]
        L.orc_eval_force.argtypes = [C.c_void_p, dp]
        L.orc_feq.argtypes = [C.c_int32, C.c_double, dp, dp]
        L.orc_guo.argtypes = [C.c_int32, C.c_double, dp, dp, dp]
        L.orc_state_bytes.argtypes = [C.c_void_p]
        L.orc_state_bytes.restype = C.c_size_t
        L.orc_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.orc_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.orc_threads.argtypes = [C.c_int32]
        _lib = L
    return _lib


def threads(n: int = 0) -> int:
    """OpenMP threads of the oracle's loops (n > 0 sets them); returns the number in use."""
    return int(lib().orc_threads(int(n)))


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(p: dict) -> orc_params:
    q = orc_params()
    q.dim = p["dim"]
    q.nx, q.ny = p["nx"], p["ny"]
    q.nz = p.get("nz", 1) if p["dim"] == 3 else 1
    q.walls = p.get("walls", 1)
    q.hydro = p.get("hydro", 1)
    for k in ("tau", "Gamma", "b", "kappa", "c", "Tc", "T0", "Tw", "xi"):
        setattr(q, k, float(p[k]))
    q.n_phi_sub = p.get("n_phi_sub", 0)
    q.n_T_sub = p.get("n_T_sub", 0)
    q.force_form = p.get("force_form", 0)
    g = list(p.get("body_force", (0.0, 0.0, 0.0))) + [0.0, 0.0, 0.0]
    for k in range(3):
        q.body_force[k] = g[k]
    return q


def lattice(dim: int):
    """(e [Q,3] int, w [Q], opp [Q]) of the oracle's velocity set."""
    e = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    Q = lib().orc_lattice(dim, e.ctypes.data_as(C.POINTER(C.c_int32)), _dp(w),
                          opp.ctypes.data_as(C.POINTER(C.c_int32)))
    return e[:Q].copy(), w[:Q].copy(), opp[:Q].copy()


def feq(dim: int, n: float, u) -> np.ndarray:
    u3 = np.zeros(3)
    u3[:len(u)] = u
    out = np.zeros(19)
    Q = lib().orc_feq(dim, n, _dp(u3), _dp(out))
    return out[:Q].copy()


def guo(dim: int, tau: float, u, F) -> np.ndarray:
    u3, F3 = np.zeros(3), np.zeros(3)
    u3[:len(u)] = u
    F3[:len(F)] = F
    out = np.zeros(19)
    Q = lib().orc_guo(dim, tau, _dp(u3), _dp(F3), _dp(out))
    return out[:Q].copy()


class Oracle:
    """One oracle simulation.  Fields are numpy arrays shaped (ny, nx) or (nz, ny, nx)."""

    def __init__(self, params: dict):
        self.params = dict(params)
        self.dim = params["dim"]
        self.shape = ((params["ny"], params["nx"]) if self.dim == 2
                      else (params["nz"], params["ny"], params["nx"]))
        self.N = int(np.prod(self.shape))
        self.Q = 9 if self.dim == 2 else 19
        self._p = make_params(params)
        h = C.c_void_p()
        rc = lib().orc_create(C.byref(self._p), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_create failed ({rc}) for {params}")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_destroy(self._h)
            self._h = None

    @property
    def substeps(self):
        a, b = C.c_int32(), C.c_int32()
        lib().orc_substeps(self._h, C.byref(a), C.byref(b))
        return a.value, b.value

    def init_fields(self, phi0, u0=None, n0=None):
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1)
        u0 = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64).reshape(-1)
        n0 = None if n0 is None else np.ascontiguousarray(n0, dtype=np.float64).reshape(-1)
        assert phi0.size == self.N
        rc = lib().orc_init_fields(self._h, _dp(phi0), _dp(u0), _dp(n0))
        assert rc == 0
        return self

    def step(self, n: int = 1):
        assert lib().orc_step(self._h, int(n)) == 0
        return self

    def observables(self) -> dict:
        o = orc_obs()
        assert lib().orc_observables(self._h, C.byref(o)) == 0
        return dict(mass_dev=o.mass_dev, mom=list(o.mom)[:self.dim], phi_sum=o.phi_sum,
                    max_u=o.max_u, mach=o.mach, free_energy=o.free_energy, step=o.step,
                    nonfinite=o.nonfinite)

    def fields(self) -> dict:
        phi = np.zeros(self.N)
        u = np.zeros(self.dim * self.N)
        n = np.zeros(self.N)
        T = np.zeros(self.N)
        assert lib().orc_get_fields(self._h, _dp(phi), _dp(u), _dp(n), _dp(T)) == 0
        return dict(phi=phi.reshape(self.shape), u=u.reshape((self.dim,) + self.shape),
                    n=n.reshape(self.shape), T=T.reshape(self.shape))

    def populations(self) -> np.ndarray:
        f = np.zeros(self.Q * self.N)
        assert lib().orc_get_populations(self._h, _dp(f)) == 0
        return f.reshape((self.Q,) + self.shape)

    def mu(self) -> np.ndarray:
        out = np.zeros(self.N)
        assert lib().orc_eval_mu(self._h, _dp(out)) == 0
        return out.reshape(self.shape)

    def force(self) -> np.ndarray:
        out = np.zeros(self.dim * self.N)
        assert lib().orc_eval_force(self._h, _dp(out)) == 0
        return out.reshape((self.dim,) + self.shape)

    def get_state(self) -> bytes:
        n = lib().orc_state_bytes(self._h)
        buf = C.create_string_buffer(n)
        assert lib().orc_get_state(self._h, buf, n) == 0
        return buf.raw

    def set_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        rc = lib().orc_set_state(self._h, buf, len(data))
        if rc != 0:
            raise ValueError(f"orc_set_state failed ({rc})")
        return self
