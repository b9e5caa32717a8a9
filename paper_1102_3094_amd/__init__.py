"""Python binding of the gfx950 lamellar-fluid library (``liblam.so``, C-ABI in include/lam.h).

This module only marshals arguments: device memory comes from PyTorch tensors, the HIP stream is
PyTorch's current stream, and every step of the method runs in the library's kernels.  There is
no fallback: if the built library is missing, ``load()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os

from .build import LIB_PATH

LAM_OK, LAM_EINVAL, LAM_EHIP, LAM_ESIZE, LAM_ENONFINITE, LAM_ESTATE, LAM_ECORRUPT = (
    0, -1, -2, -3, -4, -5, -6)
LAM_GUARD_BYTES = 256


class LamError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lam error {code}: {msg}")
        self.code = code


class lam_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("walls", C.c_int32), ("hydro", C.c_int32),
                ("tau", C.c_double), ("Gamma", C.c_double), ("b", C.c_double),
                ("kappa", C.c_double), ("c", C.c_double), ("Tc", C.c_double),
                ("T0", C.c_double), ("Tw", C.c_double), ("xi", C.c_double),
                ("n_phi_sub", C.c_int32), ("n_T_sub", C.c_int32), ("force_form", C.c_int32),
                ("pop_storage", C.c_int32), ("allow_unstable", C.c_int32),
                ("tile_hint", C.c_int32), ("body_force", C.c_double * 3)]


class lam_obs(C.Structure):
    _fields_ = [("mass_dev", C.c_double), ("mom", C.c_double * 3), ("phi_sum", C.c_double),
                ("max_u", C.c_double), ("mach", C.c_double), ("free_energy", C.c_double),
                ("step", C.c_int64), ("nonfinite", C.c_int32), ("reserved_", C.c_int32)]


EXPORTS = ("lam_workspace_bytes", "lam_create", "lam_substeps", "lam_init_fields", "lam_step",
           "lam_observables", "lam_structure_factor", "lam_orientation", "lam_get_fields",
           "lam_state_bytes", "lam_get_state", "lam_set_state", "lam_set_timing",
           "lam_kernel_times", "lam_last_error", "lam_destroy", "lam_set_fields",
           "lam_advance_temperature", "lam_structure_factor_static", "lam_launch_mode",
           "lam_check_guards", "lam_guard_layout",
           "lam_ensemble_workspace_bytes", "lam_ensemble_create", "lam_ensemble_member",
           "lam_ensemble_init_fields", "lam_ensemble_step", "lam_ensemble_tune",
           "lam_ensemble_sites", "lam_ensemble_last_error", "lam_ensemble_destroy")
LAM_K_LB, LAM_K_PHI, LAM_NK = 0, 1, 2

_lib = None


def load():
    """Load liblam.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1102_3094_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    pp = C.POINTER(lam_params)
    L.lam_workspace_bytes.argtypes = [pp, C.POINTER(C.c_size_t)]
    L.lam_create.argtypes = [pp, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.lam_substeps.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.lam_init_fields.argtypes = [vp, vp, vp, vp]
    L.lam_step.argtypes = [vp, C.c_int64]
    L.lam_observables.argtypes = [vp, C.POINTER(lam_obs)]
    L.lam_structure_factor.argtypes = [vp, dp, C.c_int32, dp, dp, dp]
    L.lam_orientation.argtypes = [vp, dp, C.c_int32, dp, dp]
    L.lam_structure_factor_static.argtypes = [vp, C.c_int32, C.c_int32, vp, dp, C.c_int32, dp,
                                              dp, dp]
    L.lam_get_fields.argtypes = [vp, vp, vp, vp, vp]
    L.lam_state_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.lam_get_state.argtypes = [vp, vp, C.c_size_t]
    L.lam_set_state.argtypes = [vp, vp, C.c_size_t]
    L.lam_check_guards.argtypes = [vp, C.POINTER(C.c_int32)]
    L.lam_guard_layout.argtypes = [pp, C.POINTER(C.c_size_t), C.c_int32, C.POINTER(C.c_int32)]
    L.lam_set_timing.argtypes = [vp, C.c_int32]
    L.lam_launch_mode.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_float),
                                  C.POINTER(C.c_float)]
    L.lam_kernel_times.argtypes = [vp, dp, C.POINTER(C.c_int64), C.c_int32]
    L.lam_last_error.argtypes = [vp]
    L.lam_set_fields.argtypes = [vp, vp, vp, vp]
    L.lam_advance_temperature.argtypes = [vp, C.c_int64]
    L.lam_last_error.restype = C.c_char_p
    L.lam_destroy.argtypes = [vp]
    L.lam_destroy.restype = None
    L.lam_ensemble_workspace_bytes.argtypes = [pp, C.c_int32, C.POINTER(C.c_size_t)]
    L.lam_ensemble_create.argtypes = [pp, C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.lam_ensemble_member.argtypes = [vp, C.c_int32, C.POINTER(vp)]
    L.lam_ensemble_init_fields.argtypes = [vp, C.POINTER(vp)]
    L.lam_ensemble_step.argtypes = [vp, C.c_int64]
    L.lam_ensemble_tune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.lam_ensemble_sites.argtypes = [vp, C.POINTER(C.c_int64)]
    L.lam_ensemble_last_error.argtypes = [vp]
    L.lam_ensemble_last_error.restype = C.c_char_p
    L.lam_ensemble_destroy.argtypes = [vp]
    L.lam_ensemble_destroy.restype = None
    _lib = L
    return L


def make_params(p: dict) -> lam_params:
    q = lam_params()
    q.dim = int(p["dim"])
    q.nx, q.ny = int(p["nx"]), int(p["ny"])
    q.nz = int(p.get("nz", 1)) if q.dim == 3 else 1
    q.walls = int(p.get("walls", 1))
    q.hydro = int(p.get("hydro", 1))
    for k in ("tau", "Gamma", "b", "kappa", "c", "Tc", "T0", "Tw", "xi"):
        setattr(q, k, float(p[k]))
    q.n_phi_sub = int(p.get("n_phi_sub", 0))
    q.n_T_sub = int(p.get("n_T_sub", 0))
    q.force_form = int(p.get("force_form", 0))
    q.pop_storage = int(p.get("pop_storage", 0))
    q.allow_unstable = int(p.get("allow_unstable", 0))
    q.tile_hint = int(p.get("tile_hint", 0))
    g = list(p.get("body_force", (0.0, 0.0, 0.0))) + [0.0, 0.0, 0.0]
    for k in range(3):
        q.body_force[k] = float(g[k])
    return q


def _check(rc: int, handle=None):
    if rc != LAM_OK:
        msg = load().lam_last_error(handle).decode(errors="replace")
        raise LamError(rc, msg)


def guard_layout(params: dict) -> list:
    """Byte offsets of the guard bands within the workspace of a parameter set (host only)."""
    q = make_params(params)
    n = C.c_int32()
    load().lam_guard_layout(C.byref(q), None, 0, C.byref(n))
    offs = (C.c_size_t * max(n.value, 1))()
    _check(load().lam_guard_layout(C.byref(q), offs, n.value, C.byref(n)))
    return list(offs[:n.value])


def workspace_bytes(params: dict) -> int:
    n = C.c_size_t()
    q = make_params(params)
    _check(load().lam_workspace_bytes(C.byref(q), C.byref(n)))
    return n.value


LAM_SK_STATIC_BYTES = 32 << 20


def structure_factor_static(phi, nbins: int, stream=None) -> dict:
    """S(k) of a 2D FP32 device field phi (ny, nx) through lam_structure_factor_static: no
    device memory is allocated; the scratch is the library's static device array.  The stream
    defaults to torch's current stream of phi's device."""
    import torch
    assert phi.is_cuda and phi.dtype == torch.float32 and phi.dim() == 2 and phi.is_contiguous()
    ny, nx = phi.shape
    with torch.cuda.device(phi.device):
        st = stream if stream is not None else torch.cuda.current_stream(phi.device)
        S = (C.c_double * nbins)()
        kp, Sp, km = C.c_double(), C.c_double(), C.c_double()
        _check(load().lam_structure_factor_static(C.c_void_p(phi.data_ptr()), nx, ny,
                                                  C.c_void_p(st.cuda_stream), S, nbins,
                                                  C.byref(kp), C.byref(Sp), C.byref(km)))
    return dict(S=list(S), k_peak=kp.value, S_peak=Sp.value, k_mean=km.value)


class Sim:
    """One simulation on one GPU.  Fields are torch tensors shaped (ny, nx) or (nz, ny, nx)."""

    @classmethod
    def _view(cls, handle, params: dict, device, stream):
        """A member of an ensemble: the ensemble owns the handle and the memory."""
        import torch
        self = cls.__new__(cls)
        self.params = dict(params)
        self.device = torch.device(device)
        self.dim = int(params["dim"])
        self.shape = (params["ny"], params["nx"])
        self.N = int(params["ny"]) * int(params["nx"])
        self.stream = stream
        self._h = handle
        self._owned = False
        return self

    def __init__(self, params: dict, device="cuda:0", stream=None):
        import torch
        L = load()
        self._owned = True
        self.params = dict(params)
        self.device = torch.device(device)
        self.dim = int(params["dim"])
        self.shape = ((params["ny"], params["nx"]) if self.dim == 2
                      else (params["nz"], params["ny"], params["nx"]))
        self.N = 1
        for s in self.shape:
            self.N *= int(s)
        self._p = make_params(params)
        nbytes = workspace_bytes(params)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(L.lam_create(C.byref(self._p), C.c_void_p(self.workspace.data_ptr()), nbytes,
                            C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None and getattr(self, "_owned", True):
            _lib.lam_destroy(h)
        self._h = None

    def _chk(self, rc):
        _check(rc, self._h)

    @property
    def substeps(self):
        a, b = C.c_int32(), C.c_int32()
        self._chk(load().lam_substeps(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def _dev(self, t, n):
        import torch
        if t is None:
            return None
        t = torch.as_tensor(t, dtype=torch.float32, device=self.device).contiguous()
        assert t.numel() == n, (t.shape, n)
        return t

    def init_fields(self, phi0, u0=None, n0=None):
        phi0 = self._dev(phi0, self.N)
        u0 = self._dev(u0, self.dim * self.N)
        n0 = self._dev(n0, self.N)
        self._keep = (phi0, u0, n0)
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
        self._chk(load().lam_init_fields(self._h, ptr(phi0), ptr(u0), ptr(n0)))
        return self

    def step(self, n: int = 1):
        self._chk(load().lam_step(self._h, int(n)))
        return self

    def set_fields(self, phi, u=None, n=None):
        """Replace phi and restart the populations from the equilibrium of (n, u); T and the
        step count are kept."""
        phi = self._dev(phi, self.N)
        u = self._dev(u, self.dim * self.N)
        n = self._dev(n, self.N)
        self._keep_set = (phi, u, n)
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
        self._chk(load().lam_set_fields(self._h, ptr(phi), ptr(u), ptr(n)))
        return self

    def advance_temperature(self, n: int):
        self._chk(load().lam_advance_temperature(self._h, int(n)))
        return self

    def fields_into(self, buf):
        """phi, u_x, u_y, T (and, for a buffer of five planes, the density n) of a 2D run into the
        planar FP32 device buffer buf [4 or 5][ny][nx]."""
        assert self.dim == 2 and buf.is_contiguous() and buf.numel() in (4 * self.N, 5 * self.N)
        p = buf.data_ptr()
        n = C.c_void_p(p + 16 * self.N) if buf.numel() == 5 * self.N else None
        self._chk(load().lam_get_fields(self._h, C.c_void_p(p), C.c_void_p(p + 4 * self.N), n,
                                        C.c_void_p(p + 12 * self.N)))
        return buf

    def observables(self, raise_nonfinite: bool = False) -> dict:
        o = lam_obs()
        rc = load().lam_observables(self._h, C.byref(o))
        if rc != LAM_ENONFINITE or raise_nonfinite:
            self._chk(rc)
        return dict(mass_dev=o.mass_dev, mom=list(o.mom)[:self.dim], phi_sum=o.phi_sum,
                    max_u=o.max_u, mach=o.mach, free_energy=o.free_energy, step=o.step,
                    nonfinite=o.nonfinite)

    def structure_factor(self, nbins: int) -> dict:
        S = (C.c_double * nbins)()
        kp, Sp, km = C.c_double(), C.c_double(), C.c_double()
        self._chk(load().lam_structure_factor(self._h, S, nbins, C.byref(kp), C.byref(Sp),
                                              C.byref(km)))
        return dict(S=list(S), k_peak=kp.value, S_peak=Sp.value, k_mean=km.value)

    def orientation(self, nbins: int = 18) -> dict:
        h = (C.c_double * nbins)()
        q = C.c_double()
        rows = (C.c_double * (self.params["ny"] if self.dim == 2 else self.params["nz"]))()
        self._chk(load().lam_orientation(self._h, h, nbins, C.byref(q), rows))
        return dict(hist=list(h), Q=q.value, Q_row=list(rows))

    def fields(self) -> dict:
        import torch
        phi = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        u = torch.empty((self.dim,) + tuple(self.shape), dtype=torch.float32, device=self.device)
        n = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        T = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        p = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
        self._chk(load().lam_get_fields(self._h, p(phi), p(u), p(n), p(T)))
        self.stream.synchronize()
        return dict(phi=phi, u=u, n=n, T=T)

    def state_bytes(self) -> int:
        n = C.c_size_t()
        self._chk(load().lam_state_bytes(self._h, C.byref(n)))
        return n.value

    def get_state(self):
        import torch
        buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        self._chk(load().lam_get_state(self._h, C.c_void_p(buf.data_ptr()), buf.numel()))
        self.stream.synchronize()
        return buf

    def set_state(self, buf):
        self._chk(load().lam_set_state(self._h, C.c_void_p(buf.data_ptr()), buf.numel()))
        return self

    def check_guards(self):
        """Raise LamError (code LAM_ECORRUPT, naming the region) if a guard band of the workspace
        was overwritten; synchronises."""
        bad = C.c_int32()
        self._chk(load().lam_check_guards(self._h, C.byref(bad)))
        return self

    def launch_mode(self) -> dict:
        """How lam_step launches: graphs -1 (not measured yet), 0 direct, 1 graph replays; the
        measured microseconds per step of each."""
        g, d, r = C.c_int32(), C.c_float(), C.c_float()
        self._chk(load().lam_launch_mode(self._h, C.byref(g), C.byref(d), C.byref(r)))
        return dict(graphs=g.value, direct_us=d.value, graph_us=r.value)

    def set_timing(self, enable: bool = True):
        self._chk(load().lam_set_timing(self._h, int(enable)))
        return self

    def kernel_times(self) -> dict:
        """{kernel class: (total ms, launches)} since the last call (synchronises)."""
        ms = (C.c_double * LAM_NK)()
        n = (C.c_int64 * LAM_NK)()
        self._chk(load().lam_kernel_times(self._h, ms, n, LAM_NK))
        return {"lb": (ms[LAM_K_LB], n[LAM_K_LB]), "phi": (ms[LAM_K_PHI], n[LAM_K_PHI])}

    def synchronize(self):
        self.stream.synchronize()


def _check_ens(rc: int, handle=None):
    if rc != LAM_OK:
        raise LamError(rc, load().lam_ensemble_last_error(handle).decode(errors="replace"))


class Ensemble:
    """Independent 2D simulations advanced together (one launch per kernel for all members).
    Runs on its own non-default stream so that step pairs are replayed from a HIP graph."""

    def __init__(self, members, device="cuda:0", stream=None):
        import torch
        L = load()
        self.members = [dict(m) for m in members]
        self.device = torch.device(device)
        arr = (lam_params * len(members))(*[make_params(m) for m in members])
        self._arr = arr
        n = C.c_size_t()
        _check_ens(L.lam_ensemble_workspace_bytes(arr, len(members), C.byref(n)))
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.workspace = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check_ens(L.lam_ensemble_create(arr, len(members), C.c_void_p(self.workspace.data_ptr()),
                                         n.value, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.sims = []
        for i, m in enumerate(self.members):
            sh = C.c_void_p()
            _check_ens(L.lam_ensemble_member(h, i, C.byref(sh)), h)
            self.sims.append(Sim._view(sh, m, self.device, self.stream))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            for s in getattr(self, "sims", []):
                s._h = None
            _lib.lam_ensemble_destroy(h)
        self._h = None

    @property
    def sites(self) -> int:
        n = C.c_int64()
        _check_ens(load().lam_ensemble_sites(self._h, C.byref(n)), self._h)
        return n.value

    def init_fields(self, phi0s):
        import torch
        ts = [torch.as_tensor(p, dtype=torch.float32, device=self.device).contiguous()
              for p in phi0s]
        self._keep = ts
        ptrs = (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])
        torch.cuda.current_stream(self.device).synchronize()
        _check_ens(load().lam_ensemble_init_fields(self._h, ptrs), self._h)
        return self

    def step(self, n: int = 1):
        _check_ens(load().lam_ensemble_step(self._h, int(n)), self._h)
        return self

    def tune(self, steps: int = 20) -> int:
        """Autotune before init_fields; returns the tile height (the persistent grid size is
        kept in self.workgroups)."""
        th, wg = C.c_int32(), C.c_int32()
        _check_ens(load().lam_ensemble_tune(self._h, int(steps), C.byref(th), C.byref(wg)),
                   self._h)
        self.workgroups = wg.value
        return th.value

    def synchronize(self):
        self.stream.synchronize()
