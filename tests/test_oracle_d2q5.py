"""Pins of the oracle's D2Q5 convection-diffusion model: the alternative
Sec. 2 names for the convection-diffusion equation (Eq. convdiffeqn solved
by a lattice Boltzmann scheme on a five-velocity lattice instead of by the
finite differences of Sec. 2.3).

Reading (the paper names the model and its memory saving only): populations
h_i on c_0 = 0 and the four axis vectors, weights 1/3 and 1/6; equilibrium
with sum h^eq = phi, sum h^eq c = phi u* and sum h^eq c c = Gamma_h mu I;
BGK relaxation with tau_phi; mobility Gamma = Gamma_h (tau_phi - 1/2); mu
with the convection-diffusion Laplacian.  The pins: the equilibrium moments,
exact conservation of total phi, the closed form of one step at
tau_phi = 1 (a centred forward-Euler step of Eq. convdiffeqn), the
diffusivity Gamma a of a decaying cosine for several tau_phi, the flat
interface's discrete fixed point, and Galilean advection of a drop.
"""
import numpy as np
import pytest

import synth
from oracle import orc

RNG = np.random.default_rng(55)
PAPER = dict(a=-1e-3, b=1e-3, kappa=3e-3, gamma=5.0, tau=1.0, N=0.3, Q=2.5)
CS = np.sqrt(1.0 / 3.0)


def test_d2q5_equilibrium_moments():
    """sum h^eq = phi, sum h^eq c = phi u, sum h^eq c c = Gamma_h mu I."""
    c, _ = orc.D2Q5
    for _ in range(20):
        phi, mu = RNG.uniform(-1, 1), RNG.uniform(-0.1, 0.1)
        u = RNG.uniform(-0.1, 0.1, 2)
        gh = RNG.uniform(0.1, 20.0)
        h = orc.feq5(phi, mu, u, gh)
        assert abs(h.sum() - phi) < 1e-15
        np.testing.assert_allclose(h @ c, phi * u, atol=1e-16)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", h, c, c), gh * mu * np.eye(2), atol=1e-14 * gh)


def _paper_drop(shape, R, **kw):
    a, b, kappa = PAPER["a"], PAPER["b"], PAPER["kappa"]
    phi = synth.drop(shape, R, np.sqrt(-a / b), np.sqrt(-2 * kappa / a))
    return orc.Oracle(shape, **{**PAPER, **kw}, m=1, cd_model=1).init(phi)


@pytest.mark.parametrize("tau_phi", [0.8, 1.0, 1.6])
def test_d2q5_conserves_total_phi_exactly(tau_phi):
    """Collision conserves the zeroth moment and periodic streaming moves it,
    so sum phi stays at its initial value to rounding (unlike the paper's
    non-conservative finite-difference advection)."""
    o = _paper_drop((40, 48), 10, tau_phi=tau_phi)
    s0 = o.reduce()["phi_sum"]
    o.step(600)
    r = o.reduce()
    assert r["finite"]
    assert abs(r["phi_sum"] - s0) < 1e-13 * 40 * 48
    assert r["umax"] > 1e-7


def test_d2q5_at_unit_relaxation_is_a_centred_euler_step():
    """At tau_phi = 1 the post-collision populations are h^eq, so one step is
    phi_1(r) = sum_i h_i^eq(r - c_i) = phi + Gamma L(mu) - D_c(phi u*): the
    explicit Euler step of Eq. convdiffeqn with the 5-point Laplacian and the
    centred divergence (Gamma_h = 2 Gamma), mu = a phi + b phi^3 - kappa L phi."""
    shape = (20, 24)
    a, b, kappa, gamma = -0.1, 0.1, 0.1, 0.05
    phi = synth.drop(shape, 6, 1.0, np.sqrt(2.0)) + RNG.uniform(-0.05, 0.05, shape)
    u0 = RNG.uniform(-0.02, 0.02, (2,) + shape)
    o = orc.Oracle(shape, a=a, b=b, kappa=kappa, gamma=gamma, tau=0.9, N=0.3, Q=2.5, m=1, cd_model=1,
                   tau_phi=1.0).init(phi, None, u0)
    ustar = o.fields()["u"]
    phi0 = o.fields()["phi"]

    def L(f):
        return np.roll(f, 1, 0) + np.roll(f, -1, 0) + np.roll(f, 1, 1) + np.roll(f, -1, 1) - 4 * f

    mu = a * phi0 + b * phi0 ** 3 - kappa * L(phi0)
    jx, jy = phi0 * ustar[0], phi0 * ustar[1]
    div = (np.roll(jx, -1, 1) - np.roll(jx, 1, 1)) / 2 + (np.roll(jy, -1, 0) - np.roll(jy, 1, 0)) / 2
    expect = phi0 + gamma * L(mu) - div
    o.step(1)
    np.testing.assert_allclose(o.fields()["phi"], expect, atol=2e-15)


@pytest.mark.parametrize("tau_phi", [0.8, 1.0, 1.7])
def test_d2q5_diffusivity_is_gamma_a(tau_phi):
    """With a > 0 (one phase), kappa = 0 and a small cosine, Eq. convdiffeqn
    reduces to diffusion with coefficient Gamma a: the mode decays as
    exp(-Gamma a k^2 t), whatever tau_phi (Gamma_h adapts), within 1%."""
    L = 128
    shape = (4, L)
    a, gamma = 0.05, 0.5
    x = np.arange(L)
    phi = 1e-6 * np.broadcast_to(np.cos(2 * np.pi * x / L), shape)
    o = orc.Oracle(shape, a=a, b=0.1, kappa=0.0, gamma=gamma, tau=1.0, N=0.3, Q=2.5, m=1, cd_model=1,
                   tau_phi=tau_phi).init(phi)
    c = np.cos(2 * np.pi * x / L)

    def amp():
        return 2.0 * (o.fields()["phi"][0] * c).sum() / L

    o.step(50)
    t0, a0 = o.t, amp()
    o.step(3000)
    t1, a1 = o.t, amp()
    rate = np.log(a0 / a1) / (t1 - t0)
    k = 2 * np.pi / L
    assert abs(rate / (gamma * a * k * k) - 1) < 0.01


def _newton_flat_profile(n, a, b, kappa, total):
    """Discrete 1D equilibrium a p + b p^3 - kappa (p_{i+1} - 2 p_i + p_{i-1})
    = mu_bar with sum p = total, by Newton (independent of the oracle)."""
    x = np.arange(n, dtype=float)
    w = np.sqrt(-2 * kappa / a)
    p = np.sqrt(-a / b) * np.tanh((n / 4 - np.abs(x - n / 2)) / w)
    p += (total - p.sum()) / n
    mu = 0.0
    for _ in range(60):
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


def test_d2q5_flat_interface_reaches_the_discrete_fixed_point():
    """A flat slab at the paper's parameters relaxes to the state where mu
    (with the 5-point Laplacian) is uniform, which Newton finds
    independently; the flow dies down."""
    a, b, kappa = PAPER["a"], PAPER["b"], PAPER["kappa"]
    L = 32
    shape = (3, L)
    phi = synth.slab(shape, L / 4, 3 * L / 4, 1.0, np.sqrt(-2 * kappa / a), axis=1)
    o = orc.Oracle(shape, **PAPER, m=1, cd_model=1, tau_phi=1.0).init(phi)
    o.step(40000)
    fl = o.fields()
    prof = fl["phi"][0]
    assert np.abs(fl["phi"] - prof).max() < 1e-12
    ref = _newton_flat_profile(L, a, b, kappa, prof.sum())
    assert np.abs(prof - ref).max() < 1e-8
    assert np.abs(fl["u"]).max() < 1e-10


def test_d2q5_drop_is_carried_by_a_uniform_flow():
    """Galilean advection (Sec. 3): at the paper's parameters a drop in a
    uniform flow u0 moves with u0, within 1%."""
    L = 64
    shape = (L, L)
    u0 = np.array([0.01, 0.005])
    a, b, kappa = PAPER["a"], PAPER["b"], PAPER["kappa"]
    phi = synth.drop(shape, 16, np.sqrt(-a / b), np.sqrt(-2 * kappa / a))
    o = orc.Oracle(shape, **PAPER, m=1, cd_model=1, tau_phi=1.0)
    o.init(phi, np.ones(shape), synth.uniform_velocity(shape, u0))
    ang = 2 * np.pi * np.arange(L) / L

    def centre():
        wgt = np.clip(o.fields()["phi"], 0, None)
        out = []
        for axis in (1, 0):
            prof = wgt.sum(axis=1 - axis)
            out.append(np.arctan2((prof * np.sin(ang)).sum(), (prof * np.cos(ang)).sum()) * L / (2 * np.pi))
        return np.array(out)

    o.step(200)
    c0, t0 = centre(), o.t
    o.step(1000)
    c1, t1 = centre(), o.t
    np.testing.assert_allclose((c1 - c0) / (t1 - t0), u0, rtol=0.01)


@pytest.mark.slow
def test_d2q5_spurious_velocity_matches_the_finite_difference_model():
    """The D2Q5 model and the paper's finite-difference step solve the same
    equation, so at the Table I setup (D = 64 drop in 128^2, tau = 1, the
    optimal stencil) their spurious velocities agree: |u*_max|/c_s within 5%
    of the printed 3.65e-5 for both after 10,000 steps."""
    o = _paper_drop((128, 128), 32, tau_phi=1.0)
    o.step(10000)
    assert abs(o.reduce()["umax"] / CS / 3.65e-5 - 1) < 0.05
