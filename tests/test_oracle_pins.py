"""Pins of the FP64 oracle's building blocks against what the paper and the
mathematics fix independently of the oracle's own formulas.

Each test names the passage it follows.  None of them retypes the oracle's
formula: they check moment identities, Fourier symbols of the stencils,
Taylor coefficients on polynomials, exact amplification factors, and
conservation / symmetry invariants.
"""
import itertools

import numpy as np
import pytest

from oracle import orc

RNG = np.random.default_rng(20240902)


# ---------------------------------------------------------------- lattices
@pytest.mark.parametrize("d", [2, 3])
def test_lattice_isotropy(d):
    """Sec. 2.1: the weights make the lattice tensors isotropic up to rank 4
    with c_s^2 = 1/3, which is what Eqs. consmass, consimp and secmoment need."""
    e, w = orc.lattice(d)
    e = e[:, :d].astype(float)
    cs2 = 1.0 / 3.0
    assert len(w) == (9 if d == 2 else 19)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia->a", w, e), 0.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, e, e), cs2 * np.eye(d), atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", w, e, e, e), 0.0, atol=1e-16)
    I = np.eye(d)
    iso4 = cs2 ** 2 * (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
                       + np.einsum("ad,bc->abcd", I, I))
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e), iso4, atol=1e-16)
    # speeds: |e| = 1 for the axis links, sqrt(2) for the diagonals (Sec. 2.1)
    speeds = np.sqrt((e ** 2).sum(1))
    assert set(np.round(speeds ** 2).astype(int)) == ({0, 1, 2})
    # velocities come in opposite pairs
    for ei in e:
        assert any(np.all(ej == -ei) for ej in e)


# ------------------------------------------------------- equilibrium, forcing
@pytest.mark.parametrize("d", [2, 3])
def test_feq_moments(d):
    """Eqs. consmass, consimp, secmoment: sum f^eq = n, sum f^eq e = n u,
    sum f^eq e e = n c_s^2 I + n u u."""
    e, _ = orc.lattice(d)
    e = e[:, :d].astype(float)
    for _ in range(20):
        n = RNG.uniform(0.5, 2.0)
        u = RNG.uniform(-0.1, 0.1, d)
        f = orc.feq(d, n, u)
        assert abs(f.sum() - n) < 1e-15 * n * 4
        np.testing.assert_allclose(f @ e, n * u, atol=1e-16 * 8)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", f, e, e),
                                   n / 3.0 * np.eye(d) + n * np.outer(u, u), atol=1e-15)


@pytest.mark.parametrize("d", [2, 3])
def test_source_moments(d):
    """Eq. momentsforceterm with the coefficients of Eq. coeff:
    sum F_i = A = 0, sum F_i e = B = (1 - 1/2tau) F,
    sum F_i e e = (C + C^T)/2 = (1 - 1/2tau)(u F + F u)."""
    e, _ = orc.lattice(d)
    e = e[:, :d].astype(float)
    for _ in range(20):
        tau = RNG.uniform(0.55, 5.0)
        u = RNG.uniform(-0.1, 0.1, d)
        F = RNG.uniform(-1e-2, 1e-2, d)
        S = orc.source(d, tau, u, F)
        c = 1.0 - 0.5 / tau
        assert abs(S.sum()) < 1e-17
        np.testing.assert_allclose(S @ e, c * F, atol=1e-17)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", S, e, e),
                                   c * (np.outer(u, F) + np.outer(F, u)), atol=1e-17)


# ------------------------------------------------------------------ stencils
def _wave(shape, k):
    """exp(i k.r) on the lattice as (cos, sin) fields; k indexed (kx, ky[, kz])."""
    grids = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    # grids[-1] is x, grids[-2] is y, grids[-3] is z
    phase = sum(kk * g for kk, g in zip(k, reversed(grids)))
    return np.cos(phase), np.sin(phase)


def _modes(shape, count):
    out = []
    for _ in range(count):
        out.append([2 * np.pi * RNG.integers(0, n) / n for n in reversed(shape)])
    return out


@pytest.mark.parametrize("shape", [(16, 24), (8, 12, 10)])
@pytest.mark.parametrize("N", [0.5, 1.0 / 3.0, 0.3, 7.0 / 12.0])
def test_grad_fourier_symbol(shape, N):
    """Eq. xstencil: on exp(i k.r) the x-stencil gives
    2i sin(kx) [N + 2M cos(ky)] in 2D (2N + 4M = 1), and with the 3D rule
    2i sin(kx) [N + 2M (cos ky + cos kz)] (2N + 8M = 1); y and z by
    transposition."""
    d = len(shape)
    M = (1 - 2 * N) / 4 if d == 2 else (1 - 2 * N) / 8
    for k in _modes(shape, 6):
        c, s = _wave(shape, k)
        gc = orc.grad(c, N)
        gs = orc.grad(s, N)
        for a in range(d):
            others = [k[b] for b in range(d) if b != a]
            sym = 2 * np.sin(k[a]) * (N + 2 * M * sum(np.cos(kb) for kb in others))
            # D(cos) = -sym sin, D(sin) = sym cos
            np.testing.assert_allclose(gc[a], -sym * s, atol=1e-13)
            np.testing.assert_allclose(gs[a], sym * c, atol=1e-13)


@pytest.mark.parametrize("shape", [(16, 24), (8, 12, 10)])
@pytest.mark.parametrize("Q", [1.0, 2.0 / 3.0, 2.5, 1.0 / 3.0])
def test_lap_fourier_symbol(shape, Q):
    """Eq. laplstencil: symbol 2Q(cos kx + cos ky) + 4R cos kx cos ky - 4(Q+R)
    with Q + 2R = 1 in 2D; in 3D 2Q sum cos + 4R sum_{pairs} cos cos
    - (6Q + 12R) with Q + 4R = 1."""
    d = len(shape)
    R = (1 - Q) / 2 if d == 2 else (1 - Q) / 4
    for k in _modes(shape, 6):
        c, s = _wave(shape, k)
        cs = [np.cos(kk) for kk in k]
        pairs = sum(cs[i] * cs[j] for i, j in itertools.combinations(range(d), 2))
        centre = 4 * (Q + R) if d == 2 else 6 * Q + 12 * R
        sym = 2 * Q * sum(cs) + 4 * R * pairs - centre
        np.testing.assert_allclose(orc.lap(c, Q), sym * c, atol=1e-13)
        np.testing.assert_allclose(orc.lap(s, Q), sym * s, atol=1e-13)


def _poly_field(shape, fn, origin):
    """fn(x, y) evaluated on the lattice with coordinates relative to origin."""
    ny, nx = shape
    y, x = np.meshgrid(np.arange(ny, dtype=float) - origin[1],
                       np.arange(nx, dtype=float) - origin[0], indexing="ij")
    return fn(x, y)


@pytest.mark.parametrize("N,Q", [(0.5, 1.0), (0.3, 2.5), (1 / 3, 2 / 3), (7 / 12, 7 / 6)])
def test_stencil_taylor_coefficients(N, Q):
    """Sec. 3 (expansions before and after Eq. (39)):
    d_Dx = d_x + (1/6) d_x^3 + ((1-2N)/2) d_x d_y^2 + ...,
    lap_D = lap + (1/12)(d_x^4 + d_y^4) + ((1-Q)/2) d_x^2 d_y^2 + ...
    (the printed d_x^2 d_y^3 is read as d_x^2 d_y^2, the only fourth-order
    mixed term), and their product has mixed coefficients
    [1/6 + (1-2N)/2 + (1-Q)/2] d_x^3 d_y^2 and [1/12 + (1-2N)/2] d_x d_y^4,
    both zero at N = 7/12, Q = 7/6.  Finite stencils are exact on
    polynomials, so these are equalities at a site away from the wrap."""
    shape = (16, 16)
    o = (8, 8)

    def at(field):
        return field[o[1], o[0]]

    def gx(f):
        return orc.grad(f, N)[0]

    def L(f):
        return orc.lap(f, Q)

    P = lambda fn: _poly_field(shape, fn, o)  # noqa: E731
    # gradient: exact derivative is zero at the origin for these monomials
    assert abs(at(gx(P(lambda x, y: x ** 3))) - 1.0) < 1e-12            # (1/6)*6
    assert abs(at(gx(P(lambda x, y: x * y ** 2))) - (1 - 2 * N)) < 1e-12  # ((1-2N)/2)*2
    assert abs(at(gx(P(lambda x, y: y ** 2 * x + x)) ) - (1 + (1 - 2 * N))) < 1e-12
    # y derivative is the transpose
    assert abs(at(orc.grad(P(lambda x, y: y * x ** 2), N)[1]) - (1 - 2 * N)) < 1e-12
    assert abs(at(orc.grad(P(lambda x, y: x * y ** 2), N)[1])) < 1e-12
    # Laplacian
    assert abs(at(L(P(lambda x, y: x ** 4))) - 2.0) < 1e-11             # (1/12)*24
    assert abs(at(L(P(lambda x, y: x ** 2 * y ** 2))) - 2 * (1 - Q)) < 1e-11  # ((1-Q)/2)*4
    assert abs(at(L(P(lambda x, y: x ** 2 + y ** 2))) - 4.0) < 1e-12     # exact lap
    # composite d_Dx lap_D on fifth-degree monomials
    c32 = 1 / 6 + (1 - 2 * N) / 2 + (1 - Q) / 2
    c14 = 1 / 12 + (1 - 2 * N) / 2
    assert abs(at(gx(L(P(lambda x, y: x ** 3 * y ** 2)))) - 12 * c32) < 1e-9
    assert abs(at(gx(L(P(lambda x, y: x * y ** 4)))) - 24 * c14) < 1e-9
    assert abs(at(gx(L(P(lambda x, y: x ** 5)))) - 30.0) < 1e-9         # (1/4)*120
    if (N, Q) == (7 / 12, 7 / 6):
        assert abs(c32) < 1e-15 and abs(c14) < 1e-15


@pytest.mark.parametrize("N,Q", [(0.5, 1.0), (0.3, 2.5), (0.3, 3.0)])
def test_stencils_collapse_on_1d_profiles(N, Q):
    """Sec. 2.2: with 2N + 4M = 1 and Q + 2R = 1 the 3x3 stencils acting on a
    field that depends on x only reduce to the 3-point central difference and
    Laplacian, whatever N and Q are (consistency)."""
    prof = RNG.standard_normal(20)
    f = np.broadcast_to(prof, (12, 20)).copy()
    central = (np.roll(prof, -1) - np.roll(prof, 1)) / 2
    lap3 = np.roll(prof, -1) - 2 * prof + np.roll(prof, 1)
    np.testing.assert_allclose(orc.grad(f, N)[0], np.broadcast_to(central, f.shape), atol=1e-14)
    np.testing.assert_allclose(orc.grad(f, N)[1], 0.0, atol=1e-14)
    np.testing.assert_allclose(orc.lap(f, Q), np.broadcast_to(lap3, f.shape), atol=1e-13)


# -------------------------------------------------- convection-diffusion step
@pytest.mark.parametrize("shape", [(16, 20), (8, 10, 12)])
def test_advection_upwind_amplification(shape):
    """Eqs. adv, backdiff, fordiff with uniform u: D_c u = 0 and the upwind
    difference has symbol 1 - exp(-ik) for u > 0 and exp(ik) - 1 for u < 0,
    so h = phi - dt sum_a u_a sym_a phi exactly."""
    d = len(shape)
    dt = 0.37
    for k in _modes(shape, 4):
        for signs in itertools.product([1, -1], repeat=d):
            vel = np.array([0.013 * s * (a + 1) for a, s in enumerate(signs)])
            c, s = _wave(shape, k)
            u = np.zeros((d,) + shape)
            for a in range(d):
                u[a] = vel[a]
            sym = 0j
            for a in range(d):
                if vel[a] > 0:
                    sym += vel[a] * (1 - np.exp(-1j * k[a]))
                else:
                    sym += vel[a] * (np.exp(1j * k[a]) - 1)
            g = 1 - dt * sym
            z = c + 1j * s
            expect = g * z
            np.testing.assert_allclose(orc.ch_advect(c, u, dt), expect.real, atol=1e-15)
            np.testing.assert_allclose(orc.ch_advect(s, u, dt), expect.imag, atol=1e-15)


def test_advection_divergence_term():
    """Eqs. adv and centrdiff: with phi uniform the upwind term vanishes and
    h = phi (1 - dt D_c u_x), D_c cos(k x) = -sin(k) sin(k x)."""
    shape = (10, 32)
    kx = 2 * np.pi * 3 / 32
    x = np.arange(32, dtype=float)
    u = np.zeros((2,) + shape)
    u[0] = 0.01 * np.cos(kx * x)
    phi = np.full(shape, 0.7)
    dt = 0.2
    expect = 0.7 * (1 - dt * 0.01 * (-np.sin(kx) * np.sin(kx * x)))
    np.testing.assert_allclose(orc.ch_advect(phi, u, dt), np.broadcast_to(expect, shape), atol=1e-16)


@pytest.mark.parametrize("shape,cdQ", [((16, 20), 1.0), ((16, 20), 2 / 3), ((8, 10, 12), 1.0),
                                      ((8, 10, 12), 1 / 3)])
def test_diffusion_linear_amplification(shape, cdQ):
    """Eq. diff about phi = 0 (cubic term O(eps^3)): a Fourier mode of
    amplitude eps is multiplied by 1 + dt Gamma (a s - kappa s^2), s the
    Laplacian symbol (standard stencil: 2 sum cos k - 2d)."""
    d = len(shape)
    a, b, kappa, gamma, dt = -0.1, 0.1, 0.1, 1.0, 0.2
    eps = 1e-9
    R = (1 - cdQ) / 2 if d == 2 else (1 - cdQ) / 4
    for k in _modes(shape, 5):
        c, _ = _wave(shape, k)
        cs = [np.cos(kk) for kk in k]
        pairs = sum(cs[i] * cs[j] for i, j in itertools.combinations(range(d), 2))
        centre = 4 * (cdQ + R) if d == 2 else 6 * cdQ + 12 * R
        s = 2 * cdQ * sum(cs) + 4 * R * pairs - centre
        g = 1 + dt * gamma * (a * s - kappa * s * s)
        phi = eps * c
        out = orc.ch_diffuse(phi, phi, dt, gamma, a, b, kappa, cdQ)
        np.testing.assert_allclose(out, g * phi, atol=1e-15 * eps * max(1.0, abs(g)) * 10)


def test_diffusion_cubic_uses_pre_advection_phi():
    """Eq. diff: the cubic term is b lap (phi^n)^3 with the value before the
    advection half-step, the a and kappa terms act on phi^{n+1/2}.  Choosing
    (phi^n)^3 = cos(kx) isolates it: out(h, phi) - out(h, 0) =
    dt Gamma b s cos(kx)."""
    shape = (6, 24)
    kx = 2 * np.pi * 5 / 24
    x = np.arange(24, dtype=float)
    c = np.broadcast_to(np.cos(kx * x), shape).copy()
    phi = np.cbrt(c)
    h = RNG.standard_normal(shape)
    a, b, kappa, gamma, dt = -0.1, 0.1, 0.1, 1.0, 0.2
    s = 2 * np.cos(kx) - 2
    diff = (orc.ch_diffuse(h, phi, dt, gamma, a, b, kappa)
            - orc.ch_diffuse(h, np.zeros(shape), dt, gamma, a, b, kappa))
    np.testing.assert_allclose(diff, dt * gamma * b * s * c, atol=1e-15)


@pytest.mark.parametrize("mode", [0, 1])
def test_diffusion_conserves_and_flux_advection_conserves(mode):
    """Eq. diff is a discrete divergence (the Laplacian weights sum to zero),
    so sum phi is conserved to roundoff; the flux-form advection (mode 1) is
    conservative as well, the paper's form (mode 0) is not in general."""
    shape = (24, 20)
    phi = RNG.uniform(-1, 1, shape)
    h = RNG.uniform(-1, 1, shape)
    out = orc.ch_diffuse(h, phi, 0.2, 1.0, -0.1, 0.1, 0.1)
    assert abs(out.sum() - h.sum()) < 1e-12
    u = RNG.uniform(-0.05, 0.05, (2,) + shape)
    adv = orc.ch_advect(phi, u, 0.2, mode)
    if mode == 1:
        assert abs(adv.sum() - phi.sum()) < 1e-12
    else:
        assert abs(adv.sum() - phi.sum()) > 1e-6
