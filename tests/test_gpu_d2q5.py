"""The D2Q5 convection-diffusion model (the alternative Sec. 2 names for
Eq. convdiffeqn) on the GPU, compared element by element with the FP64
oracle's D2Q5 model on the same seeded inputs, at the paper's parameters
(the regime where a whole lattice Boltzmann step of phi is stable).

Tolerances as for the finite-difference model: FP64 differs from the oracle
only in summation order and fused multiply-adds; FP32 storage within 1e-5
after 1000 steps."""
import numpy as np
import pytest

import synth
from oracle import orc

pytestmark = pytest.mark.gpu

PAPER = dict(a=-1e-3, b=1e-3, kappa=3e-3, tau=1.0, gamma=5.0, N=0.3, Q=2.5)
CS = np.sqrt(1.0 / 3.0)


@pytest.fixture(scope="module")
def hlb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0902_3921_amd import hlb as mod

    mod.load()
    return mod


def _drop(shape, R, params=PAPER):
    a, b, kappa = params["a"], params["b"], params["kappa"]
    return synth.drop(shape, R, np.sqrt(-a / b), np.sqrt(-2 * kappa / a))


def _pair(hlb, shape, storage, phi, n=None, u=None, tau_phi=1.0, **kw):
    params = dict(PAPER, **kw)
    gpu = hlb.Sim(shape, storage, cd_model=1, tau_phi=tau_phi, **params).init(phi, n, u)
    ora = orc.Oracle(shape, m=1, cd_model=1, tau_phi=tau_phi, **params).init(phi, n, u)
    return gpu, ora


def _maxdiff(gpu, ora):
    g, o = gpu.fields(), ora.fields()
    return {k: float(np.abs(g[k] - o[k]).max()) for k in ("n", "u", "phi", "mu")}


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_d2q5_init_matches(hlb, storage):
    """t = 0: f = f^eq(n0, u0), h = h^eq(phi0, mu0, u0) and phi = sum h."""
    shape = (37, 52)
    rng = np.random.default_rng(5)
    phi = _drop(shape, 10) + rng.uniform(-0.02, 0.02, shape)
    u = rng.uniform(-0.01, 0.01, (2,) + shape)
    gpu, ora = _pair(hlb, shape, storage, phi, None, u)
    d = _maxdiff(gpu, ora)
    assert max(d.values()) < (1e-14 if storage == "f64" else 3e-7), d


@pytest.mark.parametrize("tau_phi", [1.0, 0.8, 1.7])
@pytest.mark.parametrize("variant", [dict(), dict(force_form=0), dict(N=0.5, Q=1.0, g=(2e-6, -1e-6)),
                                     dict(cd_Q=2.0 / 3.0)], ids=["paper", "mu_first", "standard_body_force",
                                                                 "iso_laplacian"])
def test_d2q5_parity_fp64_ragged(hlb, tau_phi, variant):
    """A ragged 70 x 45 lattice (no multiple of the 64 x 8 tile), 300 steps:
    every relaxation time, both force forms, the body force and the
    9-point Laplacian inside mu agree with the oracle to rounding."""
    shape = (45, 70)
    u0 = np.zeros((2,) + shape)
    u0[0] = 0.005
    gpu, ora = _pair(hlb, shape, "f64", _drop(shape, 14), None, u0, tau_phi=tau_phi, **variant)
    gpu.step(300)
    ora.step(300)
    d = _maxdiff(gpu, ora)
    assert max(d.values()) < 1e-12, d


def test_d2q5_drop_128_fp64_and_fp32_1000_steps(hlb):
    """The D = 64 drop in 128^2 of Table I (tau = 1, the optimal stencil),
    1000 steps: FP64 within 1e-11, FP32 shifted storage within 1e-5."""
    shape = (128, 128)
    phi = _drop(shape, 32)
    ora = orc.Oracle(shape, m=1, cd_model=1, tau_phi=1.0, **PAPER).init(phi)
    ora.step(1000)
    o = ora.fields()
    for storage, tol in (("f64", 1e-11), ("f32", 1e-5)):
        gpu = hlb.Sim(shape, storage, cd_model=1, tau_phi=1.0, **PAPER).init(phi)
        gpu.step(1000)
        g = gpu.fields()
        d = {k: float(np.abs(g[k] - o[k]).max()) for k in ("phi", "u", "n")}
        print(f"D2Q5 {storage} 1000 steps: {d}", flush=True)
        assert d["phi"] < tol and d["u"] < tol, d
        gpu.close()


def test_d2q5_tiny_lattices(hlb):
    """Lattices smaller than the tile and the stencil reach (wrapping onto
    themselves) agree with the oracle."""
    rng = np.random.default_rng(9)
    for shape in ((1, 1), (2, 3), (5, 4), (3, 9)):
        phi = rng.uniform(-0.5, 0.5, shape)
        gpu, ora = _pair(hlb, shape, "f64", phi, tau_phi=1.3)
        gpu.step(25)
        ora.step(25)
        d = _maxdiff(gpu, ora)
        assert max(d.values()) < 1e-12, (shape, d)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_d2q5_conserves_total_phi(hlb, storage):
    """The D2Q5 model conserves sum phi exactly (the collision keeps the
    zeroth moment, streaming moves it): to 1e-12 relative in FP64 over 2000
    steps; FP32 only rounds."""
    shape = (96, 96)
    gpu = hlb.Sim(shape, storage, cd_model=1, **PAPER).init(_drop(shape, 24))
    r0 = gpu.reduce()
    gpu.step(2000)
    r1 = gpu.reduce()
    drift = abs(r1["phi_sum"] - r0["phi_sum"]) / np.abs(gpu.fields()["phi"]).sum()
    print(f"D2Q5 {storage}: relative sum-phi drift {drift:.3e}", flush=True)
    assert drift < (1e-12 if storage == "f64" else 1e-6)
    assert r1["finite"] and abs(r1["mass"] / r0["mass"] - 1) < 1e-9


def test_d2q5_spurious_velocity_table1(hlb):
    """At the Table I setup (tau = 1, N = 0.3, Q = 2.5) the D2Q5 model's
    spurious velocity equals the finite-difference model's: |u*_max|/c_s
    within 5% of the printed 3.65e-5 after 20,000 steps (FP64)."""
    shape = (128, 128)
    gpu = hlb.Sim(shape, "f64", cd_model=1, **PAPER).init(_drop(shape, 32))
    gpu.step(20000)
    v = gpu.reduce()["umax"] / CS
    print(f"D2Q5 |u*max|/c_s = {v:.4e} (Table I, finite differences: 3.65e-5)", flush=True)
    assert abs(v / 3.65e-5 - 1) < 0.05


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_d2q5_checkpoint_and_state_rules(hlb, storage):
    """A checkpoint holds the D2Q5 populations: a resumed run is bit for bit
    the uninterrupted one.  hlb_set_state (no populations h) and a change of
    cd_model are refused."""
    shape = (40, 56)
    a = hlb.Sim(shape, storage, cd_model=1, **PAPER).init(_drop(shape, 12))
    a.step(9)
    blob = a.save()
    a.step(13)
    fa = a.fields()
    b = hlb.Sim(shape, storage, cd_model=1, tau_phi=1.4, **PAPER)
    b.load(blob)
    assert b.reduce()["step"] == 9
    b.step(13)
    fb = b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    with pytest.raises(hlb.HlbError) as e:
        b.set_state(*b.state())
    assert e.value.status == hlb.HLB_EINVAL
    with pytest.raises(hlb.HlbError) as e:
        b.set_params(**PAPER)  # cd_model 0
    assert e.value.status == hlb.HLB_EINVAL
    fd = hlb.Sim(shape, storage, **PAPER)
    with pytest.raises(hlb.HlbError) as e:
        fd.load(blob)
    assert e.value.status == hlb.HLB_ESHAPE


def test_d2q5_kernel_names_and_timing(hlb):
    shape = (256, 256)
    s = hlb.Sim(shape, "f32", cd_model=1, **PAPER).init(_drop(shape, 64))
    assert s.kernel_name(0) == "hlb::k_lb5<float, 64, 8>"
    assert s.kernel_name(1) == "hlb::k_phi5<float>"
    s.step(2)
    before = s.fields()
    us = s.time_kernels(5)
    assert all(v > 0 for v in us[:3])  # us[3] is a difference of two timings
    after = s.fields()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    assert s.autotune() == 0.0
