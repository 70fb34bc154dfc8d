"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers and lays out initial geometries (a drop,
a slab, a shear wave).  It holds none of the lattice Boltzmann or
convection-diffusion arithmetic: the order-parameter amplitude and interface
width of a drop are arguments, computed by the caller.

Every generator returns float64 numpy arrays in the lattice shape
``(ny, nx)`` or ``(nz, ny, nx)``, x fastest.
"""
from __future__ import annotations

import numpy as np


def spinodal(shape, seed: int, amp: float = 0.01) -> np.ndarray:
    """phi ~ U(-amp, amp), i.i.d. per site, from numpy's PCG64 with ``seed``."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, tuple(shape))


def _min_image(coord: np.ndarray, c: float, n: int) -> np.ndarray:
    d = coord - c
    return d - n * np.round(d / n)


def drop(shape, radius: float, phi0: float, width: float, center=None) -> np.ndarray:
    """A drop phi0*tanh((R - r)/width) on the periodic lattice.

    ``r`` is the minimum-image distance from ``center`` (default: the site
    nearest the middle, ``n // 2`` on every axis), so the drop has the
    lattice's mirror symmetries about its centre.
    ``width = 0`` gives a sharp drop (+phi0 for r < R, -phi0 outside, 0 on r = R).
    """
    shape = tuple(int(s) for s in shape)
    if center is None:
        center = tuple(n // 2 for n in shape)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    r2 = np.zeros(shape)
    for g, c, n in zip(grids, center, shape):
        r2 += _min_image(g, float(c), n) ** 2
    r = np.sqrt(r2)
    if width == 0:
        return phi0 * np.sign(radius - r)
    return phi0 * np.tanh((radius - r) / width)


def slab(shape, x0: float, x1: float, phi0: float, width: float, axis: int = -1) -> np.ndarray:
    """Two flat interfaces normal to ``axis`` at x0 < x1 (periodic): +phi0 inside.

    phi = phi0 * tanh((half - |x - mid|)/width), with mid and half the centre
    and half-thickness of the slab (minimum image), a smooth periodic slab;
    ``width = 0`` gives the sharp slab (0 on the two interface sites).
    """
    shape = tuple(int(s) for s in shape)
    n = shape[axis]
    x = np.arange(n, dtype=np.float64)
    if width == 0:
        prof = np.where((x > x0) & (x < x1), phi0, -phi0)
        prof = np.where((x == x0) | (x == x1), 0.0, prof)
    else:
        mid = 0.5 * (x0 + x1)
        half = 0.5 * (x1 - x0)
        dist = np.abs(_min_image(x, mid, n))
        prof = phi0 * np.tanh((half - dist) / width)
    bshape = [1] * len(shape)
    bshape[axis] = n
    return np.broadcast_to(prof.reshape(bshape), shape).copy()


def shear_wave(shape, amp: float, wave_axis: int = -2, vel_axis: int = -1, modes: int = 1):
    """Velocity field u_vel = amp*sin(2 pi modes x_wave / L) as (d, *shape)."""
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    n = shape[wave_axis]
    x = np.arange(n, dtype=np.float64)
    prof = amp * np.sin(2.0 * np.pi * modes * x / n)
    bshape = [1] * d
    bshape[wave_axis] = n
    u = np.zeros((d,) + shape)
    # component index counts x first: component 0 is along the last array axis
    comp = (d - 1) - (vel_axis % d)
    u[comp] = np.broadcast_to(prof.reshape(bshape), shape)
    return u


def uniform_velocity(shape, vel) -> np.ndarray:
    """A uniform velocity (components x, y[, z]) as (d, *shape)."""
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    u = np.zeros((d,) + shape)
    for k in range(d):
        u[k] = vel[k]
    return u


def batch_specs(nsim: int, seed: int, lmin: int = 64, lmax: int = 256):
    """Draws a batch of independent drop / flat-interface simulations.

    Simulation b has a square periodic lattice of side L ~ U{lmin..lmax}
    (integers), kappa ~ U(0.05, 0.2), tau ~ U(0.6, 1.5) and, with equal
    probability, either a drop of radius R ~ U(8, L/4) at a uniformly drawn
    centre or a slab with two flat interfaces, normal to x or y, of thickness
    ~ U(L/4, 3L/4) at a uniformly drawn offset.  Returns a list of dicts
    ``{"shape", "kappa", "tau", "kind", "radius", "center", "x0", "x1",
    "axis"}``; the caller turns a spec into phi with ``drop`` or ``slab``
    and the interface width of its own free energy.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(int(nsim)):
        L = int(rng.integers(lmin, lmax + 1))
        spec = {"shape": (L, L), "kappa": float(rng.uniform(0.05, 0.2)), "tau": float(rng.uniform(0.6, 1.5))}
        if rng.uniform() < 0.5:
            spec.update(kind="drop", radius=float(rng.uniform(8.0, L / 4.0)),
                        center=(float(rng.uniform(0, L)), float(rng.uniform(0, L))))
        else:
            thick = float(rng.uniform(L / 4.0, 3.0 * L / 4.0))
            x0 = float(rng.uniform(0, L - thick))
            spec.update(kind="slab", x0=x0, x1=x0 + thick, axis=int(rng.choice([-1, -2])))
        out.append(spec)
    return out
