"""The paper's printed results, reproduced with the HIP library.

Sec. 3 gives two quantitative experiments on the circular drop at the
paper's parameters (-a = b = 1e-3, kappa = -3a, Gamma = 5, Delta x =
Delta t = 1):
  * Table I: the maximum spurious velocity |u*_max|/c_s of an equilibrated
    drop of diameter 64 in a 128^2 lattice with the optimal stencil (N, Q)
    for each tau, about ten times below the standard stencil (Fig. 4);
  * the drop advected by a body force G = n (g_x, 0) acting until t = 500 in
    a 256 x 128 lattice: the centre-of-mass velocity equals the fluid
    velocity at the centre of mass, and the drop keeps its shape.
The printed Table I is the fixture tests/golden/table1.txt.
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

CS = np.sqrt(1.0 / 3.0)
PAPER = dict(a=-1e-3, b=1e-3, kappa=3e-3, gamma=5.0)
W = np.sqrt(6.0)  # sqrt(-2 kappa / a)


@pytest.fixture(scope="module")
def hlb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0902_3921_amd import hlb as mod

    mod.load()
    return mod


def _table1():
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "table1.txt"))
    return [(float(r[0]), float(r[1]), float(r[2]), float(r[3])) for r in rows]


@pytest.mark.parametrize("row", _table1(), ids=lambda r: f"tau{r[0]}")
def test_table1_spurious_velocities(hlb, row):
    """Every row of Table I within 5% after 60,000 steps (the slowest rows,
    tau = 5 and 10, relax over tens of thousands of steps), and the
    standard stencil N = 1/2, Q = 1 between 5 and 15 times higher (the
    factor of about ten of Fig. 4)."""
    tau, N, Q, ref = row
    phi = synth.drop((128, 128), 32, 1.0, W)
    vals = {}
    for label, (n_, q_) in (("OC", (N, Q)), ("SC", (0.5, 1.0))):
        sim = hlb.Sim((128, 128), "f64", **PAPER, tau=tau, N=n_, Q=q_)
        assert sim.m == 1
        sim.init(phi)
        sim.step(60000)
        r = sim.reduce()
        assert r["finite"]
        vals[label] = r["umax"] / CS
    print(f"tau={tau}: OC {vals['OC']:.4e} (Table I {ref:.4e}), SC/OC {vals['SC'] / vals['OC']:.2f}", flush=True)
    assert abs(vals["OC"] / ref - 1) < 0.05
    assert 5 < vals["SC"] / vals["OC"] < 15


def _shape_measures(f, shape):
    """Centre of mass of the nodes inside the drop (phi > 0); the horizontal
    and vertical diameters from the interpolated phi = 0 crossings through
    it; the ratio sqrt(Ixx / Iyy) of the second moments of phi > 0 about the
    centre (a shape measure that does not depend on the interface profile at
    two points); and the fluid velocity there."""
    ph = f["phi"]
    ny, nx = shape
    wgt = np.clip(ph, 0, None)
    ang = 2 * np.pi * np.arange(nx) / nx
    prof = wgt.sum(axis=0)
    cx = (np.arctan2((prof * np.sin(ang)).sum(), (prof * np.cos(ang)).sum()) * nx / (2 * np.pi)) % nx
    cy = (wgt.sum(axis=1) * np.arange(ny)).sum() / wgt.sum()

    def width(line):
        # the drop never reaches the lattice edge here, so the inside is one run
        idx = np.nonzero(line > 0)[0]
        lo, hi = idx[0], idx[-1]
        left = lo - line[lo] / (line[lo] - line[lo - 1])
        right = hi + line[hi] / (line[hi] - line[hi + 1])
        return right - left

    dx = width(ph[int(round(cy)) % ny])
    dy = width(ph[:, int(round(cx)) % nx])
    X = (np.arange(nx) - cx + nx / 2) % nx - nx / 2
    Y = np.arange(ny) - cy
    mom = np.sqrt((wgt * X[None, :] ** 2).sum() / (wgt * Y[:, None] ** 2).sum())
    ux = f["u"][0][int(round(cy)) % ny, int(round(cx)) % nx]
    return cx, cy, dx / dy, mom, ux


def _advected_drop(hlb, gx, kappa=PAPER["kappa"], t_end=3000):
    prm = dict(PAPER, kappa=kappa)
    w = np.sqrt(-2 * prm["kappa"] / prm["a"])
    shape = (128, 256)
    eq = hlb.Sim(shape, "f64", **prm, tau=1.0, N=0.3, Q=2.5)
    eq.init(synth.drop(shape, 32, 1.0, w, center=(64, 128)))
    eq.step(5000)
    f0, p0 = eq.state()
    eq.close()
    sim = hlb.Sim(shape, "f64", **prm, tau=1.0, N=0.3, Q=2.5, g_ext=(gx, 0.0))
    sim.set_state(f0, p0)
    hist = []
    for t in range(0, t_end + 1, 100):
        if t == 500:
            sim.set_params(**prm, tau=1.0, N=0.3, Q=2.5, g_ext=(0.0, 0.0))
        hist.append((t,) + _shape_measures(sim.fields(), shape))
        if t < t_end:
            sim.step(100)
    sim.close()
    return np.array(hist), shape


@pytest.mark.parametrize("gx", [1e-5, 3e-5, 5e-5])
def test_drop_advection_galilean(hlb, gx):
    """Sec. 3, drop advection: an equilibrated drop of diameter 64 in
    256 x 128, optimal stencil, body force G = n (g_x, 0) until t = 500.
    Afterwards the centre of mass moves with the fluid velocity at the
    centre of mass (v_CM = v_f within 1%), and the fluid moves with the
    momentum the force gave it.  The paper's shape statements are tested in
    test_drop_advection_shape."""
    h, shape = _advected_drop(hlb, gx)
    xs = np.unwrap(h[:, 1] * 2 * np.pi / shape[1]) * shape[1] / (2 * np.pi)
    vcm = np.diff(xs) / 100.0
    after = h[:, 0][1:] > 1000
    v_cm = vcm[after].mean()
    v_f = h[1:, 5][after].mean()
    print(f"g_x={gx}: v_CM={v_cm:.5e} v_f={v_f:.5e}; D_x/D_y - 1 every 500 steps "
          f"{np.round(h[::5, 3] - 1, 4).tolist()}; moment ratio - 1 {np.round(h[::5, 4] - 1, 4).tolist()}",
          flush=True)
    assert abs(v_cm / v_f - 1) < 0.01
    assert abs(v_f / (gx * 500) - 1) < 0.05  # momentum given by the force, n ~ 1


def test_drop_advection_shape(hlb):
    """Sec. 3, drop advection, shape: the paper states that the diameter
    ratio stays within 3% of 1, that a faster drop is slightly deformed, and
    that the deformation becomes negligible with a larger surface tension
    (larger kappa).  The paper gives neither the diameters' definition nor
    the time window, so two definitions are used over t <= 3000: the phi = 0
    crossings through the centre (D_x / D_y) and the second moments of
    phi > 0 (sqrt(Ixx / Iyy)).
      - At g_x = 1e-5 both stay within the paper's 3%.
      - The deformation grows with the speed: at g_x = 1e-5, 3e-5, 5e-5 the
        largest deviation of either measure increases.
      - The second-moment deformation at g_x = 3e-5 drops by at least a
        factor 2 when kappa is four times larger (the paper's remark); the
        phi = 0 crossings do not respond to kappa, so their growth is a
        property of the advected interface profile, not of the shape.
    The g_x = 3e-5 deviations themselves (3.8% and 3.4%) exceed the quoted
    3%; see the readings of the paper."""
    dev = {}
    for gx in (1e-5, 3e-5, 5e-5):
        h, _ = _advected_drop(hlb, gx)
        dev[gx] = (np.abs(h[:, 3] - 1).max(), np.abs(h[:, 4] - 1).max())
    h4, _ = _advected_drop(hlb, 3e-5, kappa=4 * PAPER["kappa"])
    dev_k4 = (np.abs(h4[:, 3] - 1).max(), np.abs(h4[:, 4] - 1).max())
    print(f"max deviations (crossings, moments): {dev}; kappa x 4 at 3e-5: {dev_k4}", flush=True)
    assert max(dev[1e-5]) < 0.03
    for k in (0, 1):
        assert dev[1e-5][k] < dev[3e-5][k] < dev[5e-5][k]
    assert dev_k4[1] < 0.5 * dev[3e-5][1]
