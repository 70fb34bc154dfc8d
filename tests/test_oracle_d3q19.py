"""Pins of the oracle's coupled D3Q19 timestep (three-dimensional reading of
Secs. 2.1-2.3: D3Q19 velocities and weights, the 3x3x3 stencils with faces
and edges, the 7-point convection-diffusion Laplacian, upwinding per axis).

The paper is two-dimensional, so these pins come from what holds in any
dimension: streaming moves f^eq along e_i, BGK relaxes a uniform
non-equilibrium part by 1 - 1/tau, mass is conserved, the shear viscosity is
c_s^2 (tau - 1/2), a drop centred on a site keeps the cube's symmetries, a
flat interface relaxes to the discrete 1D fixed point of the
convection-diffusion step, and Laplace's law reads Delta p = 2 sigma / R for
a sphere (Sec. 2, Eq. surftens for sigma).
"""
import numpy as np
import pytest

import synth
from oracle import orc

BASE = dict(a=-0.1, b=0.1, kappa=0.1, tau=1.0, gamma=1.0)
ISO3 = dict(N=1.0 / 6.0, Q=1.0 / 3.0)
SC3 = dict(N=0.5, Q=1.0)
RNG = np.random.default_rng(1919)


def _phi_eq(a, b):
    return np.sqrt(-a / b)


def _w(a, kappa):
    return np.sqrt(-2.0 * kappa / a)


def test_d3q19_streaming_carries_equilibria_along_e_i():
    """Eq. forceevoleqn at tau = 1 with phi = 0 (no force): the populations
    after one step are f_i(r) = f_i^eq(n, u)(r - e_i), for all 19 i."""
    shape = (5, 6, 7)
    n = RNG.uniform(0.9, 1.1, shape)
    u = RNG.uniform(-0.02, 0.02, (3,) + shape)
    o = orc.Oracle(shape, **BASE, **ISO3, m=1)
    o.init(np.zeros(shape), n, u)
    o.step(1)
    f, _ = o.state()
    e, _ = orc.lattice(3)
    assert len(e) == 19
    for i in range(19):
        feq_i = np.zeros(shape)
        for idx in np.ndindex(shape):
            feq_i[idx] = orc.feq(3, n[idx], u[(slice(None),) + idx])[i]
        # arrays are (z, y, x): roll by (e_z, e_y, e_x)
        expect = np.roll(feq_i, shift=(e[i, 2], e[i, 1], e[i, 0]), axis=(0, 1, 2))
        np.testing.assert_allclose(f[i], expect, atol=1e-16)


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_d3q19_bgk_relaxation_of_a_uniform_nonequilibrium_part(tau):
    """Eq. evoleqn on a uniform lattice without force: the part of f
    orthogonal to the conserved moments decays by 1 - 1/tau per step."""
    shape = (4, 5, 6)
    n0, u0 = 0.97, np.array([0.01, -0.02, 0.015])
    feq = orc.feq(3, n0, u0)
    e, _ = orc.lattice(3)
    basis = np.stack([np.ones(19), e[:, 0], e[:, 1], e[:, 2]], 1).astype(float)
    v = RNG.standard_normal(19)
    v -= basis @ np.linalg.lstsq(basis, v, rcond=None)[0]
    delta = 1e-3 * v
    f0 = (feq + delta)[:, None, None, None] * np.ones((19,) + shape)
    o = orc.Oracle(shape, **{**BASE, "tau": tau}, **ISO3, m=1)
    o.set_state(f0, np.zeros(shape))
    o.step(1)
    f, _ = o.state()
    expect = (feq + (1 - 1 / tau) * delta)[:, None, None, None]
    np.testing.assert_allclose(f, np.broadcast_to(expect, f.shape), atol=1e-16)


@pytest.mark.parametrize("stencil", [ISO3, SC3])
def test_d3q19_drop_conserves_mass(stencil):
    """Collision conserves mass (sum f^eq = n, sum F_i = 0) and periodic
    streaming moves it: sum n over a coupled 3D drop run is constant."""
    shape = (14, 14, 14)
    phi = synth.drop(shape, 4, 1.0, np.sqrt(2.0))
    o = orc.Oracle(shape, **BASE, **stencil, m=10).init(phi)
    m0 = o.reduce()["mass"]
    o.step(150)
    r = o.reduce()
    assert r["finite"]
    assert abs(r["mass"] - m0) / m0 < 1e-13
    assert r["umax"] > 1e-6  # the force acted


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.5])
@pytest.mark.parametrize("wave_axis,vel_axis", [(-2, -1), (-3, -2), (-1, -3)])
def test_d3q19_shear_wave_viscosity(tau, wave_axis, vel_axis):
    """Shear viscosity nu = c_s^2 (tau - 1/2) (Sec. 2.1): a transverse wave
    decays as exp(-nu k^2 t).  Three orientations, so every axis carries
    the wave and every axis the velocity once; phi = 0 removes the force."""
    L = 64
    shape = [4, 4, 4]
    shape[wave_axis] = L
    shape = tuple(shape)
    u = synth.shear_wave(shape, 1e-4, wave_axis=wave_axis, vel_axis=vel_axis)
    comp = 2 - (vel_axis % 3)
    o = orc.Oracle(shape, **{**BASE, "tau": tau}, **ISO3, m=1)
    o.init(np.zeros(shape), np.ones(shape), u)
    s = np.sin(2 * np.pi * np.arange(L) / L)

    def amp():
        uc = o.fields()["u"][comp]
        prof = np.moveaxis(uc, wave_axis, 0)[:, 0, 0]
        return 2.0 * (prof * s).sum() / L

    o.step(50)
    t0, a0 = o.t, amp()
    o.step(600)
    t1, a1 = o.t, amp()
    rate = np.log(a0 / a1) / (t1 - t0)
    nu = (tau - 0.5) / 3.0
    k = 2 * np.pi / L
    assert abs(rate / (nu * k * k) - 1) < 0.01


@pytest.mark.parametrize("force_form", [1, 0])
def test_d3q19_drop_keeps_the_cube_symmetries(force_form):
    """A drop centred on a site: the D3Q19 lattice, the 3D stencils and the
    per-axis upwinding are invariant under the mirrors x -> 2c - x (and y,
    z) and the axis exchanges, so phi stays invariant and u* transforms as a
    vector, with either force form."""
    L = 16
    c = L // 2
    shape = (L, L, L)
    phi = synth.drop(shape, 4, 1.0, np.sqrt(2.0))
    o = orc.Oracle(shape, **BASE, **ISO3, m=10, force_form=force_form).init(phi)
    o.step(60)
    fl = o.fields()
    ph, u = fl["phi"], fl["u"]  # u[0] = u_x along array axis 2
    mir = (2 * c - np.arange(L)) % L
    np.testing.assert_allclose(ph, ph[:, :, mir], atol=1e-13)
    np.testing.assert_allclose(ph, ph[:, mir, :], atol=1e-13)
    np.testing.assert_allclose(ph, ph[mir, :, :], atol=1e-13)
    np.testing.assert_allclose(u[0], -u[0][:, :, mir], atol=1e-15)
    np.testing.assert_allclose(u[1], u[1][:, :, mir], atol=1e-15)
    np.testing.assert_allclose(u[2], -u[2][mir, :, :], atol=1e-15)
    # x <-> y exchange: swap array axes 1 and 2 and components 0 and 1
    np.testing.assert_allclose(ph, ph.transpose(0, 2, 1), atol=1e-13)
    np.testing.assert_allclose(u[0], u[1].transpose(0, 2, 1), atol=1e-15)
    # y <-> z exchange: swap array axes 0 and 1 and components 1 and 2
    np.testing.assert_allclose(ph, ph.transpose(1, 0, 2), atol=1e-13)
    np.testing.assert_allclose(u[1], u[2].transpose(1, 0, 2), atol=1e-15)
    assert np.abs(u).max() > 1e-6


def _newton_flat_profile(n, a, b, kappa, total):
    """Discrete 1D equilibrium of the convection-diffusion step:
    a p_i + b p_i^3 - kappa (p_{i+1} - 2 p_i + p_{i-1}) = mu_bar, sum p = total,
    by Newton (independent of the oracle)."""
    x = np.arange(n, dtype=float)
    p = _phi_eq(a, b) * np.tanh((n / 4 - np.abs(x - n / 2)) / _w(a, kappa))
    p += (total - p.sum()) / n
    mu = 0.0
    for _ in range(50):
        lap = np.roll(p, -1) - 2 * p + np.roll(p, 1)
        res = np.concatenate([a * p + b * p ** 3 - kappa * lap - mu, [p.sum() - total]])
        J = np.zeros((n + 1, n + 1))
        for i in range(n):
            J[i, i] = a + 3 * b * p[i] ** 2 + 2 * kappa
            J[i, (i + 1) % n] -= kappa
            J[i, (i - 1) % n] -= kappa
            J[i, n] = -1.0
        J[n, :n] = 1.0
        step = np.linalg.solve(J, -res)
        p += step[:n]
        mu += step[n]
        if np.abs(step).max() < 1e-15:
            break
    return p


@pytest.mark.parametrize("normal", [0, 1, 2])
def test_d3q19_flat_interface_reaches_the_discrete_fixed_point(normal):
    """A slab with flat interfaces normal to one axis (Sec. 3, first test,
    in 3D): it stays one-dimensional, relaxes to the 1D fixed point of the
    convection-diffusion step (the 7-point Laplacian acts as the 3-point
    one on such a profile), and the velocity vanishes."""
    a, b, kappa = BASE["a"], BASE["b"], BASE["kappa"]
    L = 32
    shape = [3, 3, 3]
    shape[2 - normal] = L
    shape = tuple(shape)
    phi = synth.slab(shape, L / 4, 3 * L / 4, _phi_eq(a, b), _w(a, kappa), axis=2 - normal)
    o = orc.Oracle(shape, **BASE, **ISO3, m=10).init(phi)
    o.step(3000)
    fl = o.fields()
    prof = np.moveaxis(fl["phi"], 2 - normal, 0)
    line = prof[:, 0, 0]
    assert np.abs(prof - line[:, None, None]).max() < 1e-12
    ref = _newton_flat_profile(L, a, b, kappa, line.sum())
    assert np.abs(line - ref).max() < 1e-9
    assert np.abs(fl["u"]).max() < 1e-10


def _bulk_pressure(n, phi, a, b):
    """Eq. diagpress without gradient terms: n c_s^2 + a/2 phi^2 + 3b/4 phi^4."""
    return n / 3.0 + a / 2 * phi ** 2 + 3 * b / 4 * phi ** 4


@pytest.mark.slow
def test_d3q19_laplace_law_for_spheres():
    """Laplace's law for a sphere, Delta p = 2 sigma / R (twice the 2D
    value; sigma of Eq. surftens), from relaxed drops of radius 8 and 10 in
    a 24^3 box with the mu-first force and the standard stencil.  The bulk
    pressures are those of Eq. diagpress at the drop centre and at the
    farthest corner, the radius the equimolar one.  Each drop gives
    Delta p R / 2 sigma within 5% of 1 (a circle's sigma / R would give 1/2),
    and the flow has died down.  Smaller drops in this box dissolve into the
    bulk."""
    a, b, kappa = BASE["a"], BASE["b"], BASE["kappa"]
    sigma = 2.0 / 3.0 * np.sqrt(2 * a * a * kappa / b)
    L = 24
    c = L // 2
    shape = (L, L, L)
    for R in (8.0, 10.0):
        phi = synth.drop(shape, R, _phi_eq(a, b), _w(a, kappa))
        o = orc.Oracle(shape, **BASE, **SC3, m=10, force_form=0).init(phi)
        o.step(1200)
        fl = o.fields()
        phi_in, phi_out = fl["phi"][c, c, c], fl["phi"][0, 0, 0]
        dp = (_bulk_pressure(fl["n"][c, c, c], phi_in, a, b)
              - _bulk_pressure(fl["n"][0, 0, 0], phi_out, a, b))
        vol = (fl["phi"].sum() - phi_out * L ** 3) / (phi_in - phi_out)
        radius = np.cbrt(3.0 * vol / (4.0 * np.pi))
        assert abs(radius / R - 1) < 0.05
        assert abs(dp * radius / (2 * sigma) - 1) < 0.05
        assert np.abs(fl["u"]).max() < 1e-5  # relaxed: the force is balanced
