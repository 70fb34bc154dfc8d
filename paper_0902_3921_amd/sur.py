"""ctypes binding of the surrogate network's C ABI (include/sur.h) in libhlb.so.

Argument marshalling only: the network runs in the library's HIP kernels.
Device arrays are torch tensors (float32, contiguous, NHWC [batch, height,
width, 3]); torch also provides the workspace and the stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import hlb

EXPORTS = ("sur_config_default", "sur_param_count", "sur_workspace_size", "sur_create", "sur_set_params",
           "sur_get_params", "sur_forward", "sur_loss_grad", "sur_adam_step", "sur_forward_timed",
           "sur_last_error", "sur_destroy")


class Config(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int), ("height", ctypes.c_int), ("width", ctypes.c_int),
                ("c0", ctypes.c_int), ("c1", ctypes.c_int), ("c2", ctypes.c_int),
                ("scale", ctypes.c_double * 3)]


_vp = ctypes.c_void_p
_sigs_done = False


def _lib():
    global _sigs_done
    lib = hlb.load()
    if not _sigs_done:
        st = ctypes.c_int
        cp = ctypes.POINTER(Config)
        fp = ctypes.POINTER(ctypes.c_float)
        dp = ctypes.POINTER(ctypes.c_double)
        sig = {
            "sur_config_default": (st, [cp]),
            "sur_param_count": (st, [cp, ctypes.POINTER(ctypes.c_size_t)]),
            "sur_workspace_size": (st, [cp, ctypes.POINTER(ctypes.c_size_t)]),
            "sur_create": (st, [ctypes.POINTER(_vp), cp, _vp, ctypes.c_size_t, _vp]),
            "sur_set_params": (st, [_vp, fp]),
            "sur_get_params": (st, [_vp, fp]),
            "sur_forward": (st, [_vp, _vp, _vp, ctypes.c_int]),
            "sur_loss_grad": (st, [_vp, _vp, _vp, ctypes.c_int, dp, fp]),
            "sur_adam_step": (st, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
            "sur_forward_timed": (st, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, dp, dp]),
            "sur_last_error": (ctypes.c_char_p, [_vp]),
            "sur_destroy": (st, [_vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _sigs_done = True
    return lib


def _check(status, net=None):
    if status != hlb.HLB_OK:
        raise hlb.HlbError(status, _lib().sur_last_error(net).decode())


def config(**kw) -> Config:
    c = Config()
    _check(_lib().sur_config_default(ctypes.byref(c)))
    for k, v in kw.items():
        if k == "scale":
            for i in range(3):
                c.scale[i] = float(v[i])
        else:
            setattr(c, k, int(v))
    return c


def param_count(**kw) -> int:
    n = ctypes.c_size_t()
    _check(_lib().sur_param_count(ctypes.byref(config(**kw)), ctypes.byref(n)))
    return n.value


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _dev(t):
    import torch

    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 device tensor")
    return ctypes.c_void_p(t.data_ptr())


class Surrogate:
    """The network of include/sur.h on the current HIP device."""

    def __init__(self, stream=None, **kw):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU")
        self.lib = _lib()
        self.cfg = config(**kw)
        n = ctypes.c_size_t()
        _check(self.lib.sur_workspace_size(ctypes.byref(self.cfg), ctypes.byref(n)))
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.nparam = param_count(**kw)
        net = _vp()
        _check(self.lib.sur_create(ctypes.byref(net), ctypes.byref(self.cfg),
                                   ctypes.c_void_p(self.workspace.data_ptr()), n.value,
                                   ctypes.c_void_p(self.stream.cuda_stream)))
        self.net = net

    def close(self):
        if getattr(self, "net", None):
            self.lib.sur_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.cfg.height, self.cfg.width, 3)

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if p.size != self.nparam:
            raise ValueError(f"expected {self.nparam} parameters")
        _check(self.lib.sur_set_params(self.net, _fptr(p)), self.net)

    def params(self) -> np.ndarray:
        p = np.empty(self.nparam, dtype=np.float32)
        _check(self.lib.sur_get_params(self.net, _fptr(p)), self.net)
        return p

    def forward(self, x, y=None):
        """y = network(x) for device tensors [batch, H, W, 3]; returns y."""
        import torch

        if y is None:
            y = torch.empty_like(x)
        _check(self.lib.sur_forward(self.net, _dev(x), _dev(y), x.shape[0]), self.net)
        return y

    def loss_grad(self, x, target, grads=False):
        loss = ctypes.c_double()
        g = np.empty(self.nparam, dtype=np.float32) if grads else None
        _check(self.lib.sur_loss_grad(self.net, _dev(x), _dev(target), x.shape[0], ctypes.byref(loss),
                                      None if g is None else _fptr(g)), self.net)
        return (loss.value, g) if grads else loss.value

    def loss_grad_async(self, x, target):
        _check(self.lib.sur_loss_grad(self.net, _dev(x), _dev(target), x.shape[0], None, None), self.net)

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(self.lib.sur_adam_step(self.net, lr, beta1, beta2, eps), self.net)

    def forward_timed(self, x, y, reps=10):
        ms = (ctypes.c_double * 2)()
        flops = ctypes.c_double()
        _check(self.lib.sur_forward_timed(self.net, _dev(x), _dev(y), x.shape[0], reps, ms, ctypes.byref(flops)),
               self.net)
        return float(ms[0]), float(ms[1]), float(flops.value)


def he_init(seed: int, **kw) -> np.ndarray:
    """Seeded initial parameters: He-normal weights (std sqrt(2 / fan_in)),
    zero biases, and a head scaled by 0.1 so the first prediction stays near
    the identity."""
    c = config(**kw)
    rng = np.random.default_rng(seed)
    c0, c1, c2 = c.c0, c.c1, c.c2
    layers = [(3, c0, 9), (c0, c0, 9), (c0, c1, 9), (c1, c1, 9), (c1, c2, 9), (c2, c2, 9), (c2 + c1, c1, 9),
              (c1, c1, 9), (c1 + c0, c0, 9), (c0, c0, 9), (c0, 3, 1)]
    out = []
    for i, (ci, co, taps) in enumerate(layers):
        w = rng.standard_normal(taps * ci * co) * np.sqrt(2.0 / (taps * ci))
        if i == len(layers) - 1:
            w *= 0.1
        out += [w, np.zeros(co)]
    return np.concatenate(out).astype(np.float32)
