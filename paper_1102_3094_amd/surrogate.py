"""ctypes binding of the learned surrogate (include/lam_surrogate.h): argument marshalling only.
Every computation runs in the gfx950 kernels of liblam.so; torch supplies device memory and the
stream."""
from __future__ import annotations

import ctypes as C

from . import LAM_OK, LamError, load

SURROGATE_EXPORTS = ("lsn_param_count", "lsn_workspace_bytes", "lsn_create", "lsn_set_params",
                     "lsn_get_params", "lsn_forward", "lsn_advance", "lsn_make_target",
                     "lsn_zero_grad", "lsn_loss_backward", "lsn_loss_backward_ex", "lsn_get_grads", "lsn_adam",
                     "lsn_rollout", "lsn_set_limiter", "lsn_tune", "lsn_get_shapes", "lsn_set_shapes", "lsn_set_timing", "lsn_forward_time", "lsn_last_error",
                     "lsn_destroy")


class lsn_config(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("levels", C.c_int32),
                ("base_width", C.c_int32), ("training", C.c_int32),
                ("Tc", C.c_float), ("in_shift", C.c_float * 5), ("in_scale", C.c_float * 5),
                ("out_scale", C.c_float * 3)]


_bound = None


def lib():
    global _bound
    L = load()
    if _bound is L:
        return L
    vp, cp = C.c_void_p, C.POINTER(lsn_config)
    L.lsn_param_count.argtypes = [cp, C.POINTER(C.c_int64)]
    L.lsn_workspace_bytes.argtypes = [cp, C.POINTER(C.c_size_t)]
    L.lsn_create.argtypes = [cp, vp, C.c_size_t, vp, C.POINTER(vp)]
    for f in ("lsn_set_params", "lsn_get_params", "lsn_advance", "lsn_get_grads"):
        getattr(L, f).argtypes = [vp, vp]
    L.lsn_forward.argtypes = [vp, vp, vp]
    L.lsn_make_target.argtypes = [vp, vp, vp, vp]
    L.lsn_zero_grad.argtypes = [vp]
    L.lsn_loss_backward.argtypes = [vp, vp, vp, C.POINTER(C.c_double)]
    L.lsn_loss_backward_ex.argtypes = [vp, vp, vp, vp, vp, C.POINTER(C.c_double)]
    L.lsn_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float]
    L.lsn_rollout.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    L.lsn_set_limiter.argtypes = [vp, C.c_float]
    L.lsn_tune.argtypes = [vp, vp, C.c_int32]
    L.lsn_get_shapes.argtypes = [vp, C.POINTER(C.c_int32), C.c_int32]
    L.lsn_set_shapes.argtypes = [vp, C.POINTER(C.c_int32), C.c_int32]
    L.lsn_set_timing.argtypes = [vp, C.c_int32]
    L.lsn_forward_time.argtypes = [vp, C.POINTER(C.c_float)]
    L.lsn_last_error.argtypes = [vp]
    L.lsn_last_error.restype = C.c_char_p
    L.lsn_destroy.argtypes = [vp]
    L.lsn_destroy.restype = None
    _bound = L
    return L


def make_config(height, width, levels=4, base_width=32, training=False, Tc=1.0,
                in_shift=None, in_scale=None, out_scale=None) -> lsn_config:
    """Normalisation tuples have 5 inputs and 3 outputs; omitted ones are the identity."""
    in_shift = tuple(in_shift) if in_shift is not None else (0.0,) * 5
    in_scale = tuple(in_scale) if in_scale is not None else (1.0,) * 5
    out_scale = tuple(out_scale) if out_scale is not None else (1.0,) * 3
    if len(in_shift) != 5 or len(in_scale) != 5 or len(out_scale) != 3:
        raise ValueError("normalisation of 5 inputs and 3 outputs")
    c = lsn_config()
    c.height, c.width, c.levels, c.base_width = int(height), int(width), int(levels), int(base_width)
    c.training = int(bool(training))
    c.Tc = float(Tc)
    for i in range(5):
        c.in_shift[i] = float(in_shift[i])
        c.in_scale[i] = float(in_scale[i])
    for i in range(3):
        c.out_scale[i] = float(out_scale[i])
    return c


def _check(rc, handle=None):
    if rc != LAM_OK:
        raise LamError(rc, lib().lsn_last_error(handle).decode(errors="replace"))


def param_count(**cfg) -> int:
    n = C.c_int64()
    c = make_config(**cfg)
    _check(lib().lsn_param_count(C.byref(c), C.byref(n)))
    return n.value


class Surrogate:
    """U-Net surrogate on one GPU.  Fields are planar FP32 device tensors [NF, H, W] (phi, u_x,
    u_y, T); outputs and targets are [NOUT, H, W] (increments of phi, u_x, u_y).  NF = 4,
    NOUT = 3."""

    def __init__(self, height, width, device="cuda:0", stream=None, **cfg):
        import torch
        L = lib()
        self.device = torch.device(device)
        self.H, self.W = int(height), int(width)
        self.cfg = make_config(height, width, **cfg)
        self.NF, self.NOUT = 4, 3
        n = C.c_size_t()
        _check(L.lsn_workspace_bytes(C.byref(self.cfg), C.byref(n)))
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(L.lsn_create(C.byref(self.cfg), C.c_void_p(self.workspace.data_ptr()), n.value,
                            C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        k = C.c_int64()
        _check(L.lsn_param_count(C.byref(self.cfg), C.byref(k)))
        self.nparam = k.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _bound is not None:
            _bound.lsn_destroy(h)
        self._h = None

    def _chk(self, rc):
        _check(rc, self._h)

    def _t(self, x, shape):
        import torch
        t = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous()
        assert tuple(t.shape) == tuple(shape) or t.numel() == int(torch.tensor(shape).prod()), (t.shape, shape)
        return t

    def set_params(self, theta):
        t = self._t(theta, (self.nparam,))
        self._keep = t
        self._chk(lib().lsn_set_params(self._h, C.c_void_p(t.data_ptr())))
        return self

    def params(self):
        import torch
        out = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        self._chk(lib().lsn_get_params(self._h, C.c_void_p(out.data_ptr())))
        self.stream.synchronize()
        return out

    def forward(self, fields, out=None):
        import torch
        f = self._t(fields, (self.NF, self.H, self.W))
        if out is None:
            out = torch.empty((self.NOUT, self.H, self.W), dtype=torch.float32, device=self.device)
        self._chk(lib().lsn_forward(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(out.data_ptr())))
        return out

    def advance(self, fields):
        """In place on a contiguous [NF, H, W] FP32 device tensor."""
        assert fields.is_contiguous() and fields.dtype == torch_float32()
        assert fields.numel() == self.NF * self.H * self.W, fields.shape
        self._chk(lib().lsn_advance(self._h, C.c_void_p(fields.data_ptr())))
        return fields

    def make_target(self, earlier, later, out=None):
        import torch
        a = self._t(earlier, (self.NF, self.H, self.W))
        b = self._t(later, (self.NF, self.H, self.W))
        if out is None:
            out = torch.empty((self.NOUT, self.H, self.W), dtype=torch.float32, device=self.device)
        self._chk(lib().lsn_make_target(self._h, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                                        C.c_void_p(out.data_ptr())))
        return out

    def zero_grad(self):
        self._chk(lib().lsn_zero_grad(self._h))
        return self

    def loss_backward(self, fields, target, want_loss=True, out_grad=None, field_grad=None):
        """Adds the parameter gradient of the loss to the gradient buffer.  out_grad (optional,
        [NOUT, H, W]) is added to the loss gradient with respect to the output; field_grad
        (optional, contiguous FP32 [NF, H, W] device tensor) receives the gradient with respect
        to the fields."""
        f = self._t(fields, (self.NF, self.H, self.W))
        t = self._t(target, (self.NOUT, self.H, self.W))
        loss = C.c_double()
        if out_grad is None and field_grad is None:
            self._chk(lib().lsn_loss_backward(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(t.data_ptr()),
                                              C.byref(loss) if want_loss else None))
            return loss.value if want_loss else None
        g = None if out_grad is None else self._t(out_grad, (self.NOUT, self.H, self.W))
        if field_grad is not None:
            assert field_grad.is_contiguous() and field_grad.dtype == torch_float32()
            assert tuple(field_grad.shape) == (self.NF, self.H, self.W), field_grad.shape
        self._chk(lib().lsn_loss_backward_ex(
            self._h, C.c_void_p(f.data_ptr()), C.c_void_p(t.data_ptr()),
            None if g is None else C.c_void_p(g.data_ptr()),
            None if field_grad is None else C.c_void_p(field_grad.data_ptr()),
            C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def grads(self):
        import torch
        out = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        self._chk(lib().lsn_get_grads(self._h, C.c_void_p(out.data_ptr())))
        self.stream.synchronize()
        return out

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0):
        self._chk(lib().lsn_adam(self._h, lr, beta1, beta2, eps, grad_scale))
        return self

    def rollout(self, sim, fields_scratch, cycles, calls=10, steps_per_call=100, anchor_steps=100):
        """Surrogate-accelerated run of `sim` (a Sim on the same stream); fields_scratch is a
        contiguous [NF, H, W] FP32 device tensor."""
        assert fields_scratch.is_contiguous() and fields_scratch.numel() == self.NF * self.H * self.W
        self._chk(lib().lsn_rollout(self._h, sim._h, C.c_void_p(fields_scratch.data_ptr()),
                                    int(cycles), int(calls), int(steps_per_call), int(anchor_steps)))
        return sim

    def set_limiter(self, factor=1.05):
        """Order-parameter limiter of rollout(); factor <= 0 turns it off."""
        self._chk(lib().lsn_set_limiter(self._h, float(factor)))
        return self

    def tune(self, fields, reps=3):
        f = self._t(fields, (self.NF, self.H, self.W))
        self._chk(lib().lsn_tune(self._h, C.c_void_p(f.data_ptr()), int(reps)))
        return self.shapes()

    def shapes(self):
        """Tile-shape codes of the 3x3 layers in parameter order."""
        n = 4 * self.cfg.levels - 2
        codes = (C.c_int32 * n)()
        self._chk(lib().lsn_get_shapes(self._h, codes, n))
        return list(codes)

    def set_shapes(self, codes):
        """Tile-shape codes of the 3x3 layers in parameter order (0: the layer's default)."""
        n = 4 * self.cfg.levels - 2
        assert len(codes) == n, (len(codes), n)
        arr = (C.c_int32 * n)(*[int(c) for c in codes])
        self._chk(lib().lsn_set_shapes(self._h, arr, n))
        return self

    def set_timing(self, on=True):
        self._chk(lib().lsn_set_timing(self._h, int(bool(on))))
        return self

    def forward_time_ms(self) -> float:
        ms = C.c_float()
        self._chk(lib().lsn_forward_time(self._h, C.byref(ms)))
        return ms.value


def torch_float32():
    import torch
    return torch.float32
