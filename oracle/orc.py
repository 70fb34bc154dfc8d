"""ctypes binding of the FP64 CPU oracle (``orc.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use this module to compute the reference results the GPU
library is compared with.  The GPU library never imports it.

Array conventions (same as the GPU library's host interface):
  * a scalar field has the lattice shape, ``(ny, nx)`` in 2D or
    ``(nz, ny, nx)`` in 3D, C order, so x is the fastest index;
  * a vector field has shape ``(d, *lattice_shape)``;
  * populations have shape ``(q, *lattice_shape)`` with the velocity order of
    ``lattice(d)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c99", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    """Compile ``liborc.so`` next to its source with gcc."""
    cmd = ["gcc", *CFLAGS, "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("kappa", ctypes.c_double),
        ("tau", ctypes.c_double), ("gamma", ctypes.c_double),
        ("N", ctypes.c_double), ("Q", ctypes.c_double), ("cd_Q", ctypes.c_double),
        ("m", ctypes.c_int), ("force_form", ctypes.c_int), ("advection", ctypes.c_int),
        ("g", ctypes.c_double * 3),
        ("cd_model", ctypes.c_int), ("tau_phi", ctypes.c_double),
    ]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(OrcParams)]
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_set_params.argtypes = [ctypes.c_void_p, ctypes.POINTER(OrcParams)]
    lib.orc_init.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.orc_set_state.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.orc_get_state.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_longlong]
    lib.orc_fields.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
    lib.orc_reduce.argtypes = [ctypes.c_void_p, _dp]
    lib.orc_step_count.argtypes = [ctypes.c_void_p]
    lib.orc_step_count.restype = ctypes.c_longlong
    lib.orc_lattice.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int), _dp]
    lib.orc_grad.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, _dp, _dp]
    lib.orc_lap.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, _dp, _dp]
    lib.orc_feq.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp]
    lib.orc_source.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
    lib.orc_ch_advect.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
    lib.orc_ch_diffuse.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double] * 6 + [_dp, _dp, _dp]
    lib.orc_feq5.argtypes = [ctypes.c_double, ctypes.c_double, _dp, ctypes.c_double, _dp]
    lib.orc_get_h.argtypes = [ctypes.c_void_p, _dp]
    lib.orc_set_h.argtypes = [ctypes.c_void_p, _dp]
    lib.orc_drop_stats.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_threads.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dims(shape):
    shape = tuple(int(s) for s in shape)
    if len(shape) == 2:
        return 2, shape[1], shape[0], 1
    if len(shape) == 3:
        return 3, shape[2], shape[1], shape[0]
    raise ValueError("lattice shape must be (ny, nx) or (nz, ny, nx)")


def threads() -> int:
    return _load().orc_threads()


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def lattice(d: int):
    """Velocities ``e`` (q, 3) int and weights ``w`` (q,) of D2Q9 or D3Q19."""
    lib = _load()
    q = ctypes.c_int()
    e = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    lib.orc_lattice(d, ctypes.byref(q), e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _ptr(w))
    return e[: q.value].copy(), w[: q.value].copy()


def grad(field, N: float) -> np.ndarray:
    """Stencil gradient of Eq. xstencil (and its 3D generalisation)."""
    field = _f64(field)
    d, nx, ny, nz = _dims(field.shape)
    out = np.zeros((d,) + field.shape)
    _load().orc_grad(d, nx, ny, nz, float(N), _ptr(field), _ptr(out))
    return out


def lap(field, Q: float) -> np.ndarray:
    """Stencil Laplacian of Eq. laplstencil (and its 3D generalisation)."""
    field = _f64(field)
    d, nx, ny, nz = _dims(field.shape)
    out = np.zeros(field.shape)
    _load().orc_lap(d, nx, ny, nz, float(Q), _ptr(field), _ptr(out))
    return out


def feq(d: int, n: float, u) -> np.ndarray:
    u3 = np.zeros(3)
    u3[: len(u)] = u
    out = np.zeros(19)
    _load().orc_feq(d, float(n), _ptr(u3), _ptr(out))
    return out[: (9 if d == 2 else 19)].copy()


def source(d: int, tau: float, u, F) -> np.ndarray:
    u3 = np.zeros(3)
    u3[: len(u)] = u
    F3 = np.zeros(3)
    F3[: len(F)] = F
    out = np.zeros(19)
    _load().orc_source(d, float(tau), _ptr(u3), _ptr(F3), _ptr(out))
    return out[: (9 if d == 2 else 19)].copy()


def feq5(phi: float, mu: float, u, gamma_h: float) -> np.ndarray:
    """Equilibrium of the D2Q5 convection-diffusion populations."""
    u2 = np.zeros(2)
    u2[: len(u)] = u
    out = np.zeros(5)
    _load().orc_feq5(float(phi), float(mu), _ptr(u2), float(gamma_h), _ptr(out))
    return out


D2Q5 = (np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1]]), np.array([1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6]))


def ch_advect(phi, u, dt: float, mode: int = 0) -> np.ndarray:
    phi = _f64(phi)
    u = _f64(u)
    d, nx, ny, nz = _dims(phi.shape)
    assert u.shape == (d,) + phi.shape
    out = np.zeros(phi.shape)
    _load().orc_ch_advect(d, nx, ny, nz, float(dt), int(mode), _ptr(phi), _ptr(u), _ptr(out))
    return out


def ch_diffuse(h, phi, dt, gamma, a, b, kappa, cd_Q=1.0) -> np.ndarray:
    h = _f64(h)
    phi = _f64(phi)
    d, nx, ny, nz = _dims(phi.shape)
    out = np.zeros(phi.shape)
    _load().orc_ch_diffuse(d, nx, ny, nz, float(dt), float(gamma), float(a), float(b),
                           float(kappa), float(cd_Q), _ptr(h), _ptr(phi), _ptr(out))
    return out


def make_params(a=-0.1, b=0.1, kappa=0.1, tau=1.0, gamma=1.0, N=0.3, Q=2.5, cd_Q=1.0, m=1,
                force_form=1, advection=0, g=(0.0, 0.0, 0.0), cd_model=0, tau_phi=1.0) -> OrcParams:
    p = OrcParams()
    p.a, p.b, p.kappa, p.tau, p.gamma = a, b, kappa, tau, gamma
    p.N, p.Q, p.cd_Q = N, Q, cd_Q
    p.m, p.force_form, p.advection = int(m), int(force_form), int(advection)
    p.cd_model, p.tau_phi = int(cd_model), float(tau_phi)
    for k in range(3):
        p.g[k] = g[k] if k < len(g) else 0.0
    return p


class Oracle:
    """One periodic simulation advanced by the FP64 oracle."""

    def __init__(self, shape, **params):
        self.shape = tuple(int(s) for s in shape)
        self.d, nx, ny, nz = _dims(self.shape)
        self.q = 9 if self.d == 2 else 19
        self.params = make_params(**params)
        lib = _load()
        self._ctx = lib.orc_create(self.d, nx, ny, nz, ctypes.byref(self.params))
        if not self._ctx:
            raise ValueError("orc_create rejected the lattice or parameters")

    def __del__(self):
        if getattr(self, "_ctx", None):
            _load().orc_destroy(self._ctx)
            self._ctx = None

    def set_params(self, **params):
        self.params = make_params(**params)
        if _load().orc_set_params(self._ctx, ctypes.byref(self.params)) != 0:
            raise ValueError("orc_set_params rejected the parameters")

    def init(self, phi, n=None, u=None):
        phi = _f64(phi).reshape(self.shape)
        n = np.ones(self.shape) if n is None else _f64(n).reshape(self.shape)
        u = np.zeros((self.d,) + self.shape) if u is None else _f64(u).reshape((self.d,) + self.shape)
        _load().orc_init(self._ctx, _ptr(phi), _ptr(n), _ptr(u))
        return self

    def set_state(self, f, phi):
        f = _f64(f).reshape((self.q,) + self.shape)
        phi = _f64(phi).reshape(self.shape)
        _load().orc_set_state(self._ctx, _ptr(f), _ptr(phi))

    def state(self):
        f = np.zeros((self.q,) + self.shape)
        phi = np.zeros(self.shape)
        _load().orc_get_state(self._ctx, _ptr(f), _ptr(phi))
        return f, phi

    def h_state(self):
        """D2Q5 populations (5, *shape) of the convection-diffusion model."""
        h = np.zeros((5,) + self.shape)
        if _load().orc_get_h(self._ctx, _ptr(h)) != 0:
            raise ValueError("no D2Q5 populations (cd_model = 0)")
        return h

    def set_h(self, h):
        h = _f64(h).reshape((5,) + self.shape)
        if _load().orc_set_h(self._ctx, _ptr(h)) != 0:
            raise ValueError("no D2Q5 populations (cd_model = 0)")

    def step(self, nsteps: int = 1):
        if _load().orc_step(self._ctx, int(nsteps)) != 0:
            raise ValueError("orc_step failed")
        return self

    @property
    def t(self) -> int:
        return int(_load().orc_step_count(self._ctx))

    def fields(self):
        n = np.zeros(self.shape)
        u = np.zeros((self.d,) + self.shape)
        phi = np.zeros(self.shape)
        mu = np.zeros(self.shape)
        _load().orc_fields(self._ctx, _ptr(n), _ptr(u), _ptr(phi), _ptr(mu))
        return {"n": n, "u": u, "phi": phi, "mu": mu}

    def drop_stats(self, centre, r_in, r_out):
        """Bulk pressure, phi and n inside (distance < r_in) and outside
        (distance > r_out) a drop centred at ``centre`` (x, y[, z]), the sum
        of phi and the equimolar radius (see orc_drop_stats)."""
        c = np.zeros(3)
        c[: len(centre)] = centre
        out = np.zeros(10)
        _load().orc_drop_stats(self._ctx, _ptr(c), float(r_in), float(r_out), _ptr(out))
        return {"p_in": out[0], "phi_in": out[1], "n_in": out[2], "p_out": out[3], "phi_out": out[4],
                "n_out": out[5], "phi_sum": out[6], "radius": out[7], "count_in": int(out[8]),
                "count_out": int(out[9]), "dp": out[0] - out[3]}

    def reduce(self):
        out = np.zeros(8)
        _load().orc_reduce(self._ctx, _ptr(out))
        return {"mass": out[0], "phi_sum": out[1], "kinetic": out[2], "umax": out[3],
                "mom": out[4:4 + self.d].copy(), "finite": bool(out[7] == 1.0)}
