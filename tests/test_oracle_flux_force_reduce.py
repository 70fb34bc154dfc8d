"""Pins of three oracle parts against what the paper and the mathematics fix:
the flux-form advection (the conservative option beside Eq. adv), the
uniform body force G = n g of the drop-advection test (Sec. 3), and the FP64
global diagnostics (mass, sum of phi, kinetic energy, momentum, max |u*|).

None of these retypes the oracle's formula.  The advection pins use exact
translation at Courant number one, the upwind symbol, the continuity of a
uniform field, positivity and the direction in which mass leaves a spike,
and first-order consistency with -d(u phi)/dx.  The body force pins use
Newton's second law on the lattice, which Eqs. newvel and latticeforceterm
make exact.  The diagnostics are checked against sums of the fields that the
test itself built.
"""
import itertools

import numpy as np
import pytest

from oracle import orc

RNG = np.random.default_rng(903921)
BASE = dict(a=-0.1, b=0.1, kappa=0.1, tau=1.0, gamma=1.0, N=0.3, Q=2.5)


def _wave(shape, k):
    grids = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    phase = sum(kk * g for kk, g in zip(k, reversed(grids)))
    return np.cos(phase), np.sin(phase)


def _axis_roll(field, shift, axis_comp, d):
    """Roll a lattice field by ``shift`` sites along component axis
    ``axis_comp`` (0 = x, the last array axis)."""
    return np.roll(field, shift, axis=d - 1 - axis_comp)


# ------------------------------------------------------- flux-form advection
@pytest.mark.parametrize("shape", [(16, 20), (8, 10, 12)])
def test_flux_advection_uniform_u_is_the_upwind_scheme(shape):
    """With uniform u the face velocity is u itself, so the flux form is the
    first-order upwind scheme: on exp(i k.r) it multiplies by
    1 - dt sum_a u_a (1 - exp(-i k_a)) for u_a > 0 and
    1 - dt sum_a u_a (exp(i k_a) - 1) for u_a < 0 (Eqs. backdiff, fordiff)."""
    d = len(shape)
    dt = 0.41
    for _ in range(4):
        k = [2 * np.pi * RNG.integers(0, n) / n for n in reversed(shape)]
        for signs in itertools.product([1, -1], repeat=d):
            vel = np.array([0.017 * s * (a + 1) for a, s in enumerate(signs)])
            u = np.zeros((d,) + shape)
            for a in range(d):
                u[a] = vel[a]
            sym = sum(vel[a] * ((1 - np.exp(-1j * k[a])) if vel[a] > 0 else (np.exp(1j * k[a]) - 1))
                      for a in range(d))
            c, s = _wave(shape, k)
            expect = (1 - dt * sym) * (c + 1j * s)
            np.testing.assert_allclose(orc.ch_advect(c, u, dt, 1), expect.real, atol=1e-15)
            np.testing.assert_allclose(orc.ch_advect(s, u, dt, 1), expect.imag, atol=1e-15)


@pytest.mark.parametrize("shape", [(12, 18), (6, 8, 10)])
def test_flux_advection_unit_courant_number_is_an_exact_shift(shape):
    """At |u| dt = 1 along one axis the upwind flux moves every value exactly
    one site downstream: h(r) = phi(r - sign(u) 1_a), the exact solution of
    the advection equation (up to the rounding of phi - (phi - phi_up))."""
    d = len(shape)
    phi = RNG.standard_normal(shape)
    for a in range(d):
        for sgn in (1, -1):
            u = np.zeros((d,) + shape)
            u[a] = 0.5 * sgn
            out = orc.ch_advect(phi, u, 2.0, 1)
            np.testing.assert_allclose(out, _axis_roll(phi, sgn, a, d), rtol=0, atol=1e-15)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("shape", [(14, 22), (6, 10, 8)])
def test_uniform_phi_follows_continuity_with_the_centred_divergence(mode, shape):
    """A uniform phi = c in a non-uniform flow changes only through
    -c div u.  In both forms that divergence is the centred difference of
    Eq. centrdiff: the face velocities (u_i + u_{i+1})/2 of the flux form
    differ across a site by (u_{i+1} - u_{i-1})/2, whatever the upwind
    choice.  A face velocity taken at one side of the face gives a one-sided
    divergence instead and fails this."""
    d = len(shape)
    u = RNG.uniform(-0.05, 0.05, (d,) + shape)
    c, dt = 0.83, 0.3
    div = np.zeros(shape)
    for a in range(d):
        div += (_axis_roll(u[a], -1, a, d) - _axis_roll(u[a], 1, a, d)) / 2
    out = orc.ch_advect(np.full(shape, c), u, dt, mode)
    np.testing.assert_allclose(out, c * (1 - dt * div), atol=1e-15)


def test_flux_advection_moves_a_spike_downstream_through_its_face():
    """Upwinding in flux form: a unit spike at site i0 can lose mass only
    through the face whose velocity points away from it, to the neighbour
    on that side, and the amount is dt times that face velocity, the mean of
    the two sites' velocities.  Checked for both signs on every axis."""
    shape = (9, 11, 13)
    d = 3
    i0 = (4, 5, 6)  # (z, y, x)
    dt = 0.7
    for a in range(d):
        for sgn in (1, -1):
            u = np.zeros((d,) + shape)
            u[a] = sgn * RNG.uniform(0.01, 0.2, shape)
            phi = np.zeros(shape)
            phi[i0] = 1.0
            out = orc.ch_advect(phi, u, dt, 1)
            ax = d - 1 - a
            down = list(i0)
            down[ax] += sgn
            down = tuple(down)
            up = list(i0)
            up[ax] -= sgn
            up = tuple(up)
            face_v = 0.5 * (abs(u[a][i0]) + abs(u[a][down]))
            assert out[down] == pytest.approx(dt * face_v, rel=1e-14)
            assert out[i0] == pytest.approx(1 - dt * face_v, rel=1e-14)
            assert out[up] == 0.0
            rest = out.copy()
            rest[down] = rest[i0] = 0.0
            assert np.all(rest == 0.0)


def test_flux_advection_keeps_a_nonnegative_field_nonnegative():
    """The upwind flux form is monotone: every new value is a combination
    of old ones with non-negative coefficients when dt (|v_in| + |v_out|)
    <= 1, so an indicator field with random mixed-sign velocity stays
    non-negative (a downwind face value makes a site next to a jump
    negative)."""
    shape = (32, 32)
    phi = (RNG.uniform(size=shape) < 0.3).astype(float)
    u = RNG.uniform(-0.4, 0.4, (2,) + shape)
    out = orc.ch_advect(phi, u, 0.6, 1)
    assert out.min() >= 0.0
    assert abs(out.sum() - phi.sum()) < 1e-12


def test_flux_advection_is_consistent_to_first_order():
    """(h - phi)/dt approximates -d(u phi)/dx - d(v phi)/dy for smooth
    fields with an error that halves when the lattice spacing halves (the
    sites are refined, the fields kept).  A value taken from the wrong site
    gives an O(1) error and fails this."""
    errs = []
    for L in (32, 64, 128):
        h = 1.0 / L
        x = (np.arange(L) + 0.0) * h
        X, Y = np.meshgrid(x, x, indexing="xy")  # arrays (y, x)
        tp = 2 * np.pi
        phi = 1.2 + np.sin(tp * X) * np.cos(tp * Y)
        ux = 0.3 + 0.2 * np.cos(tp * (X + 2 * Y))
        uy = -0.25 + 0.1 * np.sin(tp * X)
        dphidx = tp * np.cos(tp * X) * np.cos(tp * Y)
        dphidy = -tp * np.sin(tp * X) * np.sin(tp * Y)
        duxdx = -0.2 * tp * np.sin(tp * (X + 2 * Y))
        duydy = 0.0
        exact = -(ux * dphidx + phi * duxdx + uy * dphidy + phi * duydy)
        # one lattice time unit lasting h makes the lattice velocity equal
        # to u; the physical rate is then the lattice change per unit / h
        dt = 0.5
        out = orc.ch_advect(phi, np.stack([ux, uy]), dt, 1)
        rate = (out - phi) / dt / h
        errs.append(np.abs(rate - exact).max())
    assert errs[0] < 2.0
    assert 1.6 < errs[0] / errs[1] < 2.4
    assert 1.6 < errs[1] / errs[2] < 2.4


# ---------------------------------------------------------------- body force
@pytest.mark.parametrize("shape,g", [((8, 12), (1e-5, -2e-5)), ((6, 5, 7), (3e-6, 1e-5, -4e-6))])
def test_body_force_accelerates_a_uniform_fluid(shape, g):
    """Sec. 3, drop advection, with phi = 0 (so the only force is G = n g):
    a uniform fluid stays uniform and, because Eq. newvel adds F/2 and the
    forcing term of Eq. latticeforceterm adds (1 - 1/2tau) F to the
    momentum, its measured velocity is u*(t) = u0 + g (t + 1/2) exactly, for
    any tau."""
    d = len(shape)
    u0 = np.array([0.01, -0.004, 0.002][:d])
    for tau in (0.7, 1.0, 1.6):
        o = orc.Oracle(shape, **{**BASE, "tau": tau}, m=1, g=tuple(g) + (0.0,) * (3 - d))
        o.init(np.zeros(shape), np.ones(shape), np.broadcast_to(u0.reshape((d,) + (1,) * d),
                                                                  (d,) + shape))
        for t in (0, 1, 7, 40):
            o.step(t - o.t)
            fl = o.fields()
            expect = u0 + np.array(g) * (t + 0.5)
            for a in range(d):
                np.testing.assert_allclose(fl["u"][a], expect[a], rtol=0, atol=1e-15)
            np.testing.assert_allclose(fl["n"], 1.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("shape", [(16, 18), (6, 8, 10)])
def test_body_force_momentum_grows_by_total_force(shape):
    """Newton's second law on the lattice: with G = n g and phi = 0 the
    total momentum sum n u* grows by M g per step (M = sum n is conserved),
    and starts at sum n u0 + M g/2, for a non-uniform n and u0.  Adding g
    without the factor n, or leaving G out of u*, breaks this."""
    d = len(shape)
    g = np.array([2e-5, -1e-5, 5e-6][:d])
    n0 = RNG.uniform(0.9, 1.1, shape)
    u0 = RNG.uniform(-0.02, 0.02, (d,) + shape)
    o = orc.Oracle(shape, **{**BASE, "tau": 0.8}, m=1, g=tuple(g) + (0.0,) * (3 - d))
    o.init(np.zeros(shape), n0, u0)
    M = n0.sum()
    p0 = (n0 * u0).reshape(d, -1).sum(1)
    for t in (0, 1, 25, 120):
        o.step(t - o.t)
        r = o.reduce()
        np.testing.assert_allclose(r["mom"], p0 + M * g * (t + 0.5), rtol=0, atol=1e-12 * M)
        assert abs(r["mass"] - M) < 1e-12 * M


# --------------------------------------------------------------- diagnostics
@pytest.mark.parametrize("shape", [(10, 14), (5, 6, 7)])
def test_reduce_matches_sums_of_the_fields_it_was_given(shape):
    """The diagnostics of a hand-built state: with phi = 0 and g = 0 there is
    no force, f = f^eq(n, u) gives back n and u* = u exactly, so the mass is
    sum n, the kinetic energy sum n |u|^2 / 2, the momentum sum n u and the
    largest speed max |u|.  A missing 1/2, a missing n or a wrong component
    fails this."""
    d = len(shape)
    n = RNG.uniform(0.8, 1.3, shape)
    u = RNG.uniform(-0.05, 0.05, (d,) + shape)
    o = orc.Oracle(shape, **BASE, m=1).init(np.zeros(shape), n, u)
    r = o.reduce()
    speed2 = (u ** 2).sum(0)
    assert r["mass"] == pytest.approx(n.sum(), rel=1e-14)
    assert r["kinetic"] == pytest.approx(0.5 * (n * speed2).sum(), rel=1e-13)
    np.testing.assert_allclose(r["mom"], (n * u).reshape(d, -1).sum(1), rtol=1e-12, atol=1e-15)
    assert r["umax"] == pytest.approx(np.sqrt(speed2.max()), rel=1e-14)
    assert r["phi_sum"] == 0.0 and r["finite"]


def test_reduce_of_a_coupled_state_agrees_with_its_fields():
    """With a drop (phi, F != 0) the diagnostics are the sums of the read
    fields n and u* at the same time, and the sum of phi."""
    import synth

    shape = (24, 24)
    u0 = synth.uniform_velocity(shape, (0.01, -0.02))
    o = orc.Oracle(shape, **BASE, m=5).init(synth.drop(shape, 6, 1.0, np.sqrt(2.0)), None, u0)
    o.step(30)
    fl = o.fields()
    r = o.reduce()
    speed2 = (fl["u"] ** 2).sum(0)
    assert r["mass"] == pytest.approx(fl["n"].sum(), rel=1e-14)
    assert r["phi_sum"] == pytest.approx(fl["phi"].sum(), rel=1e-14, abs=1e-12)
    assert r["kinetic"] == pytest.approx(0.5 * (fl["n"] * speed2).sum(), rel=1e-12)
    np.testing.assert_allclose(r["mom"], (fl["n"] * fl["u"]).reshape(2, -1).sum(1), rtol=1e-12)
    assert r["umax"] == pytest.approx(np.sqrt(speed2.max()), rel=1e-14)
    assert r["umax"] > 1e-3


@pytest.mark.parametrize("shape", [(12, 16), (6, 7, 8)])
def test_reduce_is_invariant_under_a_periodic_shift(shape):
    """The lattice is periodic, so shifting the whole state (populations and
    phi) by a lattice vector changes no global diagnostic beyond the
    rounding of the summation order."""
    d = len(shape)
    import synth

    phi = synth.drop(shape, min(shape) / 4, 1.0, np.sqrt(2.0))
    n = RNG.uniform(0.95, 1.05, shape)
    u = RNG.uniform(-0.01, 0.01, (d,) + shape)
    o = orc.Oracle(shape, **BASE, m=5).init(phi, n, u)
    o.step(3)
    f, ph = o.state()
    r0 = o.reduce()
    shift = tuple(int(s) for s in RNG.integers(1, min(shape), d))
    axes = tuple(range(d))
    o2 = orc.Oracle(shape, **BASE, m=5)
    o2.set_state(np.roll(f, shift, axis=tuple(a + 1 for a in axes)), np.roll(ph, shift, axis=axes))
    r1 = o2.reduce()
    for key in ("mass", "phi_sum", "kinetic", "umax"):
        assert r1[key] == pytest.approx(r0[key], rel=1e-12, abs=1e-13)
    np.testing.assert_allclose(r1["mom"], r0["mom"], rtol=1e-10, atol=1e-14)


def test_reduce_flags_a_non_finite_state():
    shape = (8, 8)
    o = orc.Oracle(shape, **BASE, m=1).init(np.zeros(shape))
    f, ph = o.state()
    ph[3, 4] = np.nan
    o.set_state(f, ph)
    assert not o.reduce()["finite"]
    ph[3, 4] = 0.0
    f[2, 1, 1] = np.inf
    o.set_state(f, ph)
    assert not o.reduce()["finite"]
