"""Python binding of ``libhlb.so`` (the C ABI in ``include/hlb.h``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies the device workspace (one uint8 tensor) and
the stream; nothing here computes on the fields.  Loading fails loudly if the
library has not been built (``python -m paper_0902_3921_amd.build``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhlb.so")

HLB_OK, HLB_EINVAL, HLB_ESHAPE, HLB_EUNSTABLE, HLB_ENONFINITE, HLB_EHIP, HLB_ESTATE = 0, -1, -2, -3, -4, -5, -6
D2Q9, D3Q19 = 0, 1
F64, F32_SHIFTED = 0, 1
_STORAGE = {"f64": F64, "f32": F32_SHIFTED, F64: F64, F32_SHIFTED: F32_SHIFTED}

STATUS_NAMES = {0: "HLB_OK", -1: "HLB_EINVAL", -2: "HLB_ESHAPE", -3: "HLB_EUNSTABLE",
                -4: "HLB_ENONFINITE", -5: "HLB_EHIP", -6: "HLB_ESTATE"}

# every symbol include/hlb.h declares
EXPORTS = ("hlb_params_default", "hlb_check_params", "hlb_workspace_size", "hlb_workspace_size_params",
           "hlb_create",
           "hlb_set_params", "hlb_get_params", "hlb_init_fields", "hlb_set_state", "hlb_get_state",
           "hlb_step", "hlb_get_fields", "hlb_reduce", "hlb_drop_stats", "hlb_step_timed", "hlb_kernel_name", "hlb_time_kernels",
           "hlb_set_plan", "hlb_get_plan", "hlb_autotune", "hlb_last_error", "hlb_destroy", "hlb_version",
           "hlb_checkpoint_size", "hlb_save", "hlb_load", "hlb_create_noalloc",
           "hlb_batch_workspace_size", "hlb_batch_create", "hlb_batch_info", "hlb_batch_init_fields",
           "hlb_batch_step", "hlb_batch_step_timed", "hlb_batch_set_plan", "hlb_batch_get_plan", "hlb_batch_autotune",
           "hlb_batch_get_fields", "hlb_batch_reduce", "hlb_batch_last_error",
           "hlb_batch_destroy")


class HlbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("kappa", ctypes.c_double),
        ("tau", ctypes.c_double), ("gamma", ctypes.c_double),
        ("N", ctypes.c_double), ("Q", ctypes.c_double), ("cd_Q", ctypes.c_double),
        ("fd_substeps", ctypes.c_int), ("force_form", ctypes.c_int), ("advection", ctypes.c_int),
        ("cd_model", ctypes.c_int),
        ("g_ext", ctypes.c_double * 3), ("rho0", ctypes.c_double), ("tau_phi", ctypes.c_double),
    ]


class Drop(ctypes.Structure):
    _fields_ = [
        ("p_in", ctypes.c_double), ("phi_in", ctypes.c_double), ("n_in", ctypes.c_double),
        ("p_out", ctypes.c_double), ("phi_out", ctypes.c_double), ("n_out", ctypes.c_double),
        ("dp", ctypes.c_double), ("phi_sum", ctypes.c_double), ("radius", ctypes.c_double),
        ("count_in", ctypes.c_longlong), ("count_out", ctypes.c_longlong),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("phi_sum", ctypes.c_double), ("kinetic", ctypes.c_double),
        ("umax", ctypes.c_double), ("mom", ctypes.c_double * 3), ("step", ctypes.c_longlong),
        ("finite", ctypes.c_int), ("reserved", ctypes.c_int),
    ]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)


def load():
    """Load libhlb.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_0902_3921_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    sig = {
        "hlb_params_default": (st, [ctypes.POINTER(Params)]),
        "hlb_check_params": (st, [ctypes.c_int, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_int)]),
        "hlb_workspace_size": (st, [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_size_t)]),
        "hlb_workspace_size_params": (st, [ctypes.c_int] * 5 + [ctypes.POINTER(Params),
                                                                 ctypes.POINTER(ctypes.c_size_t)]),
        "hlb_create": (st, [ctypes.POINTER(_vp)] + [ctypes.c_int] * 5
                       + [ctypes.POINTER(Params), _vp, ctypes.c_size_t, _vp]),
        "hlb_create_noalloc": (st, [ctypes.POINTER(_vp)] + [ctypes.c_int] * 5 + [ctypes.POINTER(Params), _vp]),
        "hlb_set_params": (st, [_vp, ctypes.POINTER(Params)]),
        "hlb_get_params": (st, [_vp, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_int)]),
        "hlb_init_fields": (st, [_vp, _dp, _dp, _dp]),
        "hlb_set_state": (st, [_vp, _dp, _dp]),
        "hlb_get_state": (st, [_vp, _dp, _dp]),
        "hlb_step": (st, [_vp, ctypes.c_longlong]),
        "hlb_get_fields": (st, [_vp, _dp, _dp, _dp, _dp]),
        "hlb_reduce": (st, [_vp, ctypes.POINTER(Stats)]),
        "hlb_drop_stats": (st, [_vp, _dp, ctypes.c_double, ctypes.c_double, ctypes.POINTER(Drop)]),
        "hlb_step_timed": (st, [_vp, ctypes.c_longlong, _dp]),
        "hlb_kernel_name": (ctypes.c_char_p, [_vp, ctypes.c_int]),
        "hlb_time_kernels": (st, [_vp, ctypes.c_int, _dp]),
        "hlb_set_plan": (st, [_vp, ctypes.POINTER(ctypes.c_int)]),
        "hlb_get_plan": (st, [_vp, ctypes.POINTER(ctypes.c_int)]),
        "hlb_autotune": (st, [_vp, _dp]),
        "hlb_last_error": (ctypes.c_char_p, [_vp]),
        "hlb_destroy": (st, [_vp]),
        "hlb_version": (ctypes.c_char_p, []),
        "hlb_checkpoint_size": (st, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
        "hlb_save": (st, [_vp, _vp, ctypes.c_size_t]),
        "hlb_load": (st, [_vp, _vp, ctypes.c_size_t]),
        "hlb_batch_workspace_size": (st, [ctypes.c_int, ctypes.c_int, _ip, _ip, ctypes.POINTER(ctypes.c_size_t)]),
        "hlb_batch_create": (st, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _ip, _ip,
                                  ctypes.POINTER(Params), _vp, ctypes.c_size_t, _vp]),
        "hlb_batch_info": (st, [_vp, _ip, _ip, _ip]),
        "hlb_batch_init_fields": (st, [_vp, ctypes.c_int, _dp, _dp, _dp]),
        "hlb_batch_step": (st, [_vp, ctypes.c_longlong]),
        "hlb_batch_step_timed": (st, [_vp, ctypes.c_longlong, _dp]),
        "hlb_batch_set_plan": (st, [_vp, _ip]),
        "hlb_batch_get_plan": (st, [_vp, _ip]),
        "hlb_batch_autotune": (st, [_vp, _dp]),
        "hlb_batch_get_fields": (st, [_vp, ctypes.c_int, _dp, _dp, _dp, _dp]),
        "hlb_batch_reduce": (st, [_vp, ctypes.c_int, ctypes.POINTER(Stats)]),
        "hlb_batch_last_error": (ctypes.c_char_p, [_vp]),
        "hlb_batch_destroy": (st, [_vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, ctx=None):
    if status != HLB_OK:
        msg = load().hlb_last_error(ctx).decode()
        raise HlbError(status, msg)


def _bcheck(status: int, batch=None):
    if status != HLB_OK:
        msg = load().hlb_batch_last_error(batch).decode()
        raise HlbError(status, msg)


def lattice_of(shape) -> int:
    if len(shape) == 2:
        return D2Q9
    if len(shape) == 3:
        return D3Q19
    raise ValueError("lattice shape must be (ny, nx) or (nz, ny, nx)")


def _dims(shape):
    shape = tuple(int(s) for s in shape)
    return (shape[1], shape[0], 1) if len(shape) == 2 else (shape[2], shape[1], shape[0])


def params(**kw) -> Params:
    """hlb_params with the library defaults, then the given fields."""
    p = Params()
    _check(load().hlb_params_default(ctypes.byref(p)))
    for k, v in kw.items():
        if k in ("g_ext", "g"):
            for i in range(3):
                p.g_ext[i] = float(v[i]) if i < len(v) else 0.0
        elif k in ("m", "fd_substeps"):
            p.fd_substeps = int(v)
        else:
            if not hasattr(p, k):
                raise TypeError(f"unknown parameter {k}")
            setattr(p, k, type(getattr(p, k))(v))
    return p


def check_params(lattice: int, **kw) -> int:
    """Validate parameters on the host; returns the substep count m."""
    m = ctypes.c_int()
    _check(load().hlb_check_params(lattice, ctypes.byref(params(**kw)), ctypes.byref(m)))
    return m.value


def workspace_size(lattice: int, storage, nx: int, ny: int, nz: int = 1, p: Params = None) -> int:
    b = ctypes.c_size_t()
    if p is None:
        _check(load().hlb_workspace_size(lattice, _STORAGE[storage], nx, ny, nz, ctypes.byref(b)))
    else:
        _check(load().hlb_workspace_size_params(lattice, _STORAGE[storage], nx, ny, nz, ctypes.byref(p),
                                                ctypes.byref(b)))
    return b.value


def version() -> str:
    return load().hlb_version().decode()


def _f64(a, shape) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.size != int(np.prod(shape)):
        raise ValueError(f"expected {int(np.prod(shape))} values, got {a.size}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


class Sim:
    """One periodic simulation on the current HIP device.

    ``shape`` is ``(ny, nx)`` (D2Q9) or ``(nz, ny, nx)`` (D3Q19); ``storage``
    is ``"f64"`` or ``"f32"`` (populations stored as float deviations from
    w_i rho0).  Keyword arguments set ``hlb_params`` fields (``m`` is an alias
    of ``fd_substeps``).
    """

    def __init__(self, shape, storage="f32", stream=None, noalloc=False, **kw):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU")
        self.lib = load()
        self.shape = tuple(int(s) for s in shape)
        self.lattice = lattice_of(self.shape)
        self.d = 2 if self.lattice == D2Q9 else 3
        self.q = 9 if self.lattice == D2Q9 else 19
        self.storage = _STORAGE[storage]
        nx, ny, nz = _dims(self.shape)
        self.ns = nx * ny * nz
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._params = params(**kw)
        ctx = _vp()
        if noalloc:  # hlb_create_noalloc: the library's static workspace
            self.workspace = None
            _check(self.lib.hlb_create_noalloc(ctypes.byref(ctx), self.lattice, self.storage, nx, ny, nz,
                                               ctypes.byref(self._params), ctypes.c_void_p(self.stream.cuda_stream)))
        else:
            nbytes = workspace_size(self.lattice, self.storage, nx, ny, nz, self._params)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            _check(self.lib.hlb_create(ctypes.byref(ctx), self.lattice, self.storage, nx, ny, nz,
                                       ctypes.byref(self._params), ctypes.c_void_p(self.workspace.data_ptr()),
                                       nbytes, ctypes.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx

    # -- lifetime
    def close(self):
        if getattr(self, "ctx", None):
            self.lib.hlb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- parameters
    @property
    def m(self) -> int:
        m = ctypes.c_int()
        _check(self.lib.hlb_get_params(self.ctx, None, ctypes.byref(m)), self.ctx)
        return m.value

    def set_params(self, **kw):
        self._params = params(**kw)
        _check(self.lib.hlb_set_params(self.ctx, ctypes.byref(self._params)), self.ctx)

    # -- state
    def init(self, phi, n=None, u=None):
        phi = _f64(phi, self.shape)
        n = None if n is None else _f64(n, self.shape)
        u = None if u is None else _f64(u, (self.d,) + self.shape)
        _check(self.lib.hlb_init_fields(self.ctx, _ptr(phi), _ptr(n), _ptr(u)), self.ctx)
        return self

    def set_state(self, f, phi):
        f = _f64(f, (self.q,) + self.shape)
        phi = _f64(phi, self.shape)
        _check(self.lib.hlb_set_state(self.ctx, _ptr(f), _ptr(phi)), self.ctx)

    def state(self):
        f = np.empty((self.q,) + self.shape)
        phi = np.empty(self.shape)
        _check(self.lib.hlb_get_state(self.ctx, _ptr(f), _ptr(phi)), self.ctx)
        return f, phi

    # -- checkpoints
    def save(self) -> bytes:
        """The state, step counter and parameters as a checkpoint blob."""
        n = ctypes.c_size_t()
        _check(self.lib.hlb_checkpoint_size(self.ctx, ctypes.byref(n)), self.ctx)
        buf = ctypes.create_string_buffer(n.value)
        _check(self.lib.hlb_save(self.ctx, buf, n.value), self.ctx)
        return buf.raw

    def load(self, blob: bytes):
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        _check(self.lib.hlb_load(self.ctx, buf, len(blob)), self.ctx)
        self._params = Params()
        _check(self.lib.hlb_get_params(self.ctx, ctypes.byref(self._params), None), self.ctx)
        return self

    # -- stepping
    def step(self, nsteps: int = 1):
        _check(self.lib.hlb_step(self.ctx, int(nsteps)), self.ctx)
        return self

    def step_timed(self, nsteps: int):
        ms = (ctypes.c_double * 2)()
        _check(self.lib.hlb_step_timed(self.ctx, int(nsteps), ms), self.ctx)
        return float(ms[0]), float(ms[1])

    @property
    def plan(self):
        pl = (ctypes.c_int * 4)()
        _check(self.lib.hlb_get_plan(self.ctx, pl), self.ctx)
        return tuple(pl)

    def set_plan(self, kind, fuse=1, bw=128, seg=64):
        pl = (ctypes.c_int * 4)(kind, fuse, bw, seg)
        _check(self.lib.hlb_set_plan(self.ctx, pl), self.ctx)

    def autotune(self) -> float:
        us = ctypes.c_double()
        _check(self.lib.hlb_autotune(self.ctx, ctypes.byref(us)), self.ctx)
        return us.value

    def kernel_name(self, cls: int) -> str:
        return self.lib.hlb_kernel_name(self.ctx, cls).decode()

    def time_kernels(self, reps: int):
        """(us per collide-and-stream launch, us per first substep launch,
        us of all substep launches of a step, the same after a
        collide-and-stream launch as in a step); see hlb_time_kernels."""
        us = (ctypes.c_double * 4)()
        _check(self.lib.hlb_time_kernels(self.ctx, int(reps), us), self.ctx)
        return tuple(float(v) for v in us)

    # -- readout
    def fields(self):
        n = np.empty(self.shape)
        u = np.empty((self.d,) + self.shape)
        phi = np.empty(self.shape)
        mu = np.empty(self.shape)
        _check(self.lib.hlb_get_fields(self.ctx, _ptr(n), _ptr(u), _ptr(phi), _ptr(mu)), self.ctx)
        return {"n": n, "u": u, "phi": phi, "mu": mu}

    def drop_stats(self, centre, r_in, r_out):
        """hlb_drop_stats: bulk pressures, phi and n inside and outside a drop
        at ``centre`` (x, y[, z]), dp, the sum of phi and the equimolar radius."""
        c = (ctypes.c_double * 3)(*[float(v) for v in (list(centre) + [0.0, 0.0])[:3]])
        d = Drop()
        _check(self.lib.hlb_drop_stats(self.ctx, c, float(r_in), float(r_out), ctypes.byref(d)), self.ctx)
        return {k: getattr(d, k) for k, _ in Drop._fields_}

    def reduce(self, raise_on_error: bool = True):
        s = Stats()
        status = self.lib.hlb_reduce(self.ctx, ctypes.byref(s))
        out = {"mass": s.mass, "phi_sum": s.phi_sum, "kinetic": s.kinetic, "umax": s.umax,
               "mom": np.array(list(s.mom)[: self.d]), "step": s.step, "finite": bool(s.finite),
               "status": status}
        if raise_on_error and status != HLB_OK:
            _check(status, self.ctx)
        return out


def _ints(vals):
    return (ctypes.c_int * len(vals))(*[int(v) for v in vals])


def batch_workspace_size(storage, shapes) -> int:
    nx = _ints([s[1] for s in shapes])
    ny = _ints([s[0] for s in shapes])
    b = ctypes.c_size_t()
    _bcheck(load().hlb_batch_workspace_size(_STORAGE[storage], len(shapes), nx, ny, ctypes.byref(b)))
    return b.value


class Batch:
    """Independent periodic D2Q9 simulations advanced together.

    ``shapes`` is a list of ``(ny, nx)``; ``params`` a list of dicts of
    ``hlb_params`` fields, one per simulation (or one dict for all).
    """

    def __init__(self, shapes, params_list, storage="f32", stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU")
        self.lib = load()
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        if any(len(s) != 2 for s in self.shapes):
            raise ValueError("batch shapes are (ny, nx)")
        n = len(self.shapes)
        if isinstance(params_list, dict):
            params_list = [params_list] * n
        if len(params_list) != n:
            raise ValueError("one parameter set per simulation")
        self.storage = _STORAGE[storage]
        nx = _ints([s[1] for s in self.shapes])
        ny = _ints([s[0] for s in self.shapes])
        nbytes = batch_workspace_size(storage, self.shapes)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._params = (Params * n)(*[params(**kw) for kw in params_list])
        b = _vp()
        _bcheck(self.lib.hlb_batch_create(ctypes.byref(b), self.storage, n, nx, ny, self._params,
                                          ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                          ctypes.c_void_p(self.stream.cuda_stream)))
        self.b = b

    def __len__(self):
        return len(self.shapes)

    def close(self):
        if getattr(self, "b", None):
            self.lib.hlb_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def m(self):
        ms = (ctypes.c_int * len(self))()
        _bcheck(self.lib.hlb_batch_info(self.b, None, None, ms), self.b)
        return list(ms)

    @property
    def max_m(self) -> int:
        v = ctypes.c_int()
        _bcheck(self.lib.hlb_batch_info(self.b, None, ctypes.byref(v), None), self.b)
        return v.value

    def init(self, sim: int, phi, n=None, u=None):
        shape = self.shapes[sim]
        phi = _f64(phi, shape)
        n = None if n is None else _f64(n, shape)
        u = None if u is None else _f64(u, (2,) + shape)
        _bcheck(self.lib.hlb_batch_init_fields(self.b, int(sim), _ptr(phi), _ptr(n), _ptr(u)), self.b)
        return self

    def step(self, nsteps: int = 1):
        _bcheck(self.lib.hlb_batch_step(self.b, int(nsteps)), self.b)
        return self

    def step_timed(self, nsteps: int):
        ms = (ctypes.c_double * 2)()
        _bcheck(self.lib.hlb_batch_step_timed(self.b, int(nsteps), ms), self.b)
        return float(ms[0]), float(ms[1])

    @property
    def plan(self):
        """(lb_x, lb_y, substep kind, substeps per launch, substep x, substep y)."""
        return self._plan()[2:]

    @property
    def plan_index(self):
        """The (lb, substep) candidate indices of set_plan."""
        return self._plan()[:2]

    def _plan(self):
        pl = (ctypes.c_int * 8)()
        _bcheck(self.lib.hlb_batch_get_plan(self.b, pl), self.b)
        return tuple(pl)

    def set_plan(self, lb: int, ch: int):
        pl = (ctypes.c_int * 2)(lb, ch)
        _bcheck(self.lib.hlb_batch_set_plan(self.b, pl), self.b)

    def autotune(self):
        us = (ctypes.c_double * 2)()
        _bcheck(self.lib.hlb_batch_autotune(self.b, us), self.b)
        return float(us[0]), float(us[1])

    def fields(self, sim: int):
        shape = self.shapes[sim]
        n = np.empty(shape)
        u = np.empty((2,) + shape)
        phi = np.empty(shape)
        mu = np.empty(shape)
        _bcheck(self.lib.hlb_batch_get_fields(self.b, int(sim), _ptr(n), _ptr(u), _ptr(phi), _ptr(mu)), self.b)
        return {"n": n, "u": u, "phi": phi, "mu": mu}

    def reduce(self, sim: int, raise_on_error: bool = True):
        s = Stats()
        status = self.lib.hlb_batch_reduce(self.b, int(sim), ctypes.byref(s))
        out = {"mass": s.mass, "phi_sum": s.phi_sum, "kinetic": s.kinetic, "umax": s.umax,
               "mom": np.array(list(s.mom)[:2]), "step": s.step, "finite": bool(s.finite),
               "status": status}
        if raise_on_error and status != HLB_OK:
            _bcheck(status, self.b)
        return out
