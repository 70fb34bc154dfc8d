"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Both sides start from the same seeded host arrays and are compared element
by element.  Tolerances:
  * FP64 storage: the two sides differ only in summation order and FMA
    contraction, so the difference stays at a few hundred ulps of the
    fields even after 1000 steps of a dissipative run;
  * FP32 storage: max |dphi|, |du| <= 1e-5 after 1000 steps of the 128^2
    drop (the target stated for this workload); shorter runs in proportion.
"""
import ctypes

import numpy as np
import pytest

import synth
from oracle import orc

pytestmark = pytest.mark.gpu

BASE = dict(a=-0.1, b=0.1, kappa=0.1, tau=1.0, gamma=1.0)
PAPER = dict(a=-1e-3, b=1e-3, kappa=3e-3, tau=1.0, gamma=5.0)
OC, ISO, SC = (0.3, 2.5), (1.0 / 3.0, 2.0 / 3.0), (0.5, 1.0)


@pytest.fixture(scope="module")
def hlb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0902_3921_amd import hlb as mod

    mod.load()
    return mod


def _pair(hlb, shape, storage, phi, n=None, u=None, m=None, **kw):
    """A GPU simulation and an oracle simulation from the same inputs."""
    d = len(shape)
    lattice = 0 if d == 2 else 1
    if m is None:
        m = hlb.check_params(lattice, **kw)
    gpu = hlb.Sim(shape, storage, m=m, **kw)
    gpu.init(phi, n, u)
    ora = orc.Oracle(shape, m=m, **kw)
    ora.init(phi, n, u)
    return gpu, ora


def _maxdiff(gpu, ora):
    g, o = gpu.fields(), ora.fields()
    return {k: float(np.abs(g[k] - o[k]).max()) for k in ("n", "u", "phi", "mu")}


def _drop(shape, R, params):
    a, b, kappa = params["a"], params["b"], params["kappa"]
    return synth.drop(shape, R, np.sqrt(-a / b), np.sqrt(-2 * kappa / a))


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_init_and_readout_match(hlb, storage):
    """t = 0: f = f^eq(n0, u0) (Eq. espdistrfunc) and the readout of n, u*
    (Eq. newvel), phi and mu (Eq. chempot)."""
    shape = (45, 70)
    rng = np.random.default_rng(7)
    phi = _drop(shape, 12, BASE) + rng.uniform(-0.01, 0.01, shape)
    n = rng.uniform(0.95, 1.05, shape)
    u = rng.uniform(-0.01, 0.01, (2,) + shape)
    gpu, ora = _pair(hlb, shape, storage, phi, n, u, **BASE, N=0.3, Q=2.5)
    d = _maxdiff(gpu, ora)
    tol = 1e-14 if storage == "f64" else 2e-7
    assert max(d.values()) < tol, d
    f_g, phi_g = gpu.state()
    f_o, phi_o = ora.state()
    assert np.abs(f_g - f_o).max() < (1e-15 if storage == "f64" else 1e-7)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_state_roundtrip(hlb, storage):
    shape = (13, 17)
    rng = np.random.default_rng(3)
    w = orc.lattice(2)[1]
    f = w[:, None, None] * rng.uniform(0.9, 1.1, (9,) + shape)
    phi = rng.uniform(-1, 1, shape)
    gpu = hlb.Sim(shape, storage, **BASE)
    gpu.set_state(f, phi)
    f2, phi2 = gpu.state()
    # f64: f - w rho0 + w rho0 rounds once; f32: float deviations and phi
    tol = 1e-16 if storage == "f64" else 1e-7
    assert np.abs(f2 - f).max() < tol
    if storage == "f64":
        assert np.array_equal(phi2, phi)
    else:
        assert np.abs(phi2 - phi).max() < 1e-7


def test_drop_128_fp64_1000_steps(hlb):
    """The 128^2 drop (R = 20, a = -0.1, b = 0.1, kappa = 0.1, tau = 1,
    Gamma = 1, paper stencil N = 0.3, Q = 2.5, m = 5) in FP64 storage agrees
    with the oracle after 1000 steps."""
    shape = (128, 128)
    phi = _drop(shape, 20, BASE)
    gpu, ora = _pair(hlb, shape, "f64", phi, **BASE, N=0.3, Q=2.5)
    assert gpu.m == 5
    gpu.step(1000)
    ora.step(1000)
    d = _maxdiff(gpu, ora)
    print("fp64 drop 1000 steps max diffs", d, flush=True)
    assert d["phi"] < 1e-11 and d["u"] < 1e-12 and d["n"] < 1e-12, d


@pytest.mark.parametrize("stencil", [OC, SC, ISO], ids=["paper", "standard", "isotropic"])
def test_drop_128_fp32_1000_steps(hlb, stencil):
    """Same workload with FP32 shifted populations: max |dphi|, |du| <= 1e-5,
    with the paper's optimal stencil, the standard one and the isotropic
    one (N = 1/3, Q = 2/3)."""
    shape = (128, 128)
    phi = _drop(shape, 20, BASE)
    gpu, ora = _pair(hlb, shape, "f32", phi, **BASE, N=stencil[0], Q=stencil[1])
    gpu.step(1000)
    ora.step(1000)
    d = _maxdiff(gpu, ora)
    print(f"fp32 drop 1000 steps, N = {stencil[0]:.4f}, Q = {stencil[1]:.4f}: max diffs", d, flush=True)
    assert d["phi"] <= 1e-5 and d["u"] <= 1e-5, d


@pytest.mark.parametrize("stencil", [OC, ISO, SC])
@pytest.mark.parametrize("force_form", [1, 0])
@pytest.mark.parametrize("advection", [0, 1])
def test_variants_fp64_ragged(hlb, stencil, force_form, advection):
    """Every stencil preset, both force forms and both advection forms on a
    ragged 70 x 45 lattice (not a multiple of any tile), 60 steps."""
    shape = (45, 70)
    phi = _drop(shape, 14, BASE)
    u0 = np.zeros((2,) + shape)
    u0[0] = 0.01
    kw = dict(BASE, N=stencil[0], Q=stencil[1], force_form=force_form, advection=advection)
    gpu, ora = _pair(hlb, shape, "f64", phi, None, u0, **kw)
    gpu.step(60)
    ora.step(60)
    d = _maxdiff(gpu, ora)
    assert max(d.values()) < 1e-12, d


@pytest.mark.parametrize("cd_Q,m", [(1.0, 5), (2.0 / 3.0, 3), (1.0, 8)])
def test_ch_laplacian_and_substeps(hlb, cd_Q, m):
    shape = (40, 64)
    phi = synth.spinodal(shape, seed=11)
    gpu, ora = _pair(hlb, shape, "f64", phi, m=m, **BASE, N=0.3, Q=2.5, cd_Q=cd_Q)
    gpu.step(50)
    ora.step(50)
    d = _maxdiff(gpu, ora)
    assert max(d.values()) < 1e-12, d


def test_paper_parameters_m1(hlb):
    """The paper's parameters (-a = b = 1e-3, kappa = 3e-3, Gamma = 5), m = 1."""
    shape = (64, 64)
    phi = _drop(shape, 16, PAPER)
    gpu, ora = _pair(hlb, shape, "f64", phi, **PAPER, N=0.3, Q=2.5)
    assert gpu.m == 1
    gpu.step(300)
    ora.step(300)
    d = _maxdiff(gpu, ora)
    assert d["phi"] < 1e-14 and d["u"] < 1e-15 and d["n"] < 1e-13, d


@pytest.mark.parametrize("storage,steps,tol", [("f64", 100, 1e-11), ("f32", 50, 1e-5)])
def test_spinodal_short_horizon(hlb, storage, steps, tol):
    """Spinodal decomposition from phi ~ U(-0.01, 0.01): unstable modes grow
    roundoff, so trajectories are compared at short horizons only."""
    shape = (64, 64)
    phi = synth.spinodal(shape, seed=0)
    gpu, ora = _pair(hlb, shape, storage, phi, **BASE, N=0.3, Q=2.5)
    gpu.step(steps)
    ora.step(steps)
    d = _maxdiff(gpu, ora)
    assert d["phi"] < tol and d["u"] < tol, d


@pytest.mark.parametrize("storage,steps,tol", [("f64", 100, 1e-11), ("f32", 50, 1e-5)])
@pytest.mark.parametrize("cd_Q", [1.0, 1 / 3], ids=["lap7", "lap19"])
def test_d3q19_spinodal_short_horizon(hlb, storage, steps, tol, cd_Q):
    """D3Q19 spinodal decomposition on 32^3 (the 3D workload's stencils),
    with the autotuned substep plan, at the same short horizons as in 2D."""
    shape = (32, 32, 32)
    phi = synth.spinodal(shape, seed=0)
    gpu, ora = _pair(hlb, shape, storage, phi, **BASE, N=1 / 6, Q=1 / 3, cd_Q=cd_Q)
    gpu.autotune()
    gpu.step(steps)
    ora.step(steps)
    d = _maxdiff(gpu, ora)
    assert d["phi"] < tol and d["u"] < tol, (gpu.plan, d)


@pytest.mark.parametrize("shape", [(18, 20, 24), (7, 9, 33)])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_d3q19_drop(hlb, shape, storage):
    """D3Q19 with the 3D stencils: a drop on ragged lattices, 12 steps."""
    phi = _drop(shape, 5, BASE)
    u0 = np.zeros((3,) + shape)
    u0[2] = 0.005
    gpu, ora = _pair(hlb, shape, storage, phi, None, u0, **BASE, N=1 / 6, Q=1 / 3)
    assert gpu.m == 10
    gpu.step(12)
    ora.step(12)
    d = _maxdiff(gpu, ora)
    tol = 1e-12 if storage == "f64" else 2e-6
    assert max(d.values()) < tol, d


def test_reduce_matches_oracle(hlb):
    shape = (48, 80)
    phi = _drop(shape, 15, BASE)
    gpu, ora = _pair(hlb, shape, "f64", phi, **BASE, N=0.3, Q=2.5)
    gpu.step(40)
    ora.step(40)
    rg, ro = gpu.reduce(), ora.reduce()
    assert rg["finite"] and ro["finite"] and rg["step"] == 40
    for k in ("mass", "phi_sum"):
        assert abs(rg[k] - ro[k]) < 1e-10 * abs(ro[k]) + 1e-12, k
    assert abs(rg["kinetic"] - ro["kinetic"]) < 1e-12 * max(1.0, ro["kinetic"]) + 1e-16
    assert abs(rg["umax"] - ro["umax"]) < 1e-13
    np.testing.assert_allclose(rg["mom"], ro["mom"], atol=1e-12)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_tiny_and_degenerate_lattices(hlb, storage):
    """Lattices smaller than the stencil reach (periodic images overlap), with
    the default plan, the one-substep tiles and the fused tiles (whose staged
    box wraps many times; widths 4 and 8 take its 16-byte path in FP32)."""
    tol = 1e-13 if storage == "f64" else 2e-6
    for shape in [(1, 1), (2, 3), (5, 1), (3, 4), (4, 4), (4, 8)]:
        for plan in [None, (0, 1, 128, 64), (2, 5, 16, 0), (2, 3, 64, 1024)]:
            if storage == "f64" and plan == (2, 3, 64, 1024):
                continue  # exceeds the LDS in FP64
            rng = np.random.default_rng(sum(shape))
            phi = rng.uniform(-0.5, 0.5, shape)
            gpu, ora = _pair(hlb, shape, storage, phi, **BASE, N=0.3, Q=2.5)
            if plan is not None:
                gpu.set_plan(*plan)
            gpu.step(7)
            ora.step(7)
            d = _maxdiff(gpu, ora)
            assert max(d.values()) < tol, (shape, plan, d)


@pytest.mark.parametrize("cd_Q", [1.0, 1 / 3], ids=["lap7", "lap19"])
def test_tiny_d3q19_lattices(hlb, cd_Q):
    """D3Q19 lattices of one to three sites per axis (every stencil reach is
    a periodic image), with the tiled and the z-marching substep kernels."""
    for shape in [(1, 1, 1), (1, 2, 3), (2, 3, 1)]:
        for plan in [(0, 1, 128, 64), (1, 1, 256, 2), (1, 1, 512, 1)]:
            rng = np.random.default_rng(sum(shape) + 1)
            phi = rng.uniform(-0.5, 0.5, shape)
            gpu, ora = _pair(hlb, shape, "f64", phi, **BASE, N=1 / 6, Q=1 / 3, cd_Q=cd_Q)
            gpu.set_plan(*plan)
            gpu.step(5)
            ora.step(5)
            d = _maxdiff(gpu, ora)
            assert max(d.values()) < 1e-13, (shape, plan, d)


def test_zero_steps_and_counter(hlb):
    shape = (16, 16)
    gpu = hlb.Sim(shape, "f32", **BASE)
    gpu.init(np.zeros(shape))
    gpu.step(0)
    assert gpu.reduce()["step"] == 0
    gpu.step(3)
    assert gpu.reduce()["step"] == 3


def test_nonfinite_state_is_reported(hlb):
    """A state that overflows float storage is caught by the reduction, and
    the context then refuses to step until it is re-initialised."""
    shape = (16, 16)
    gpu = hlb.Sim(shape, "f32", **BASE)
    f = np.full((9,) + shape, 1e300)
    gpu.set_state(f, np.zeros(shape))
    r = gpu.reduce(raise_on_error=False)
    assert r["status"] == hlb.HLB_ENONFINITE and not r["finite"]
    with pytest.raises(hlb.HlbError) as ei:
        gpu.step(1)
    assert ei.value.status == hlb.HLB_ESTATE
    gpu.init(np.zeros(shape))
    gpu.step(1)
    assert gpu.reduce()["finite"]


def test_nonfinite_or_nonpositive_initial_fields_are_rejected(hlb):
    """hlb_init_fields checks its host arrays: a NaN or infinity anywhere, or
    a density that is not positive, returns HLB_ENONFINITE, and a rejected
    call leaves the context usable."""
    shape = (16, 16)
    gpu = hlb.Sim(shape, "f32", **BASE)
    bad_phi = np.zeros(shape)
    bad_phi[3, 5] = np.nan
    bad_u = np.zeros((2,) + shape)
    bad_u[1, 2, 2] = np.inf
    for args in [(bad_phi,), (np.zeros(shape), None, bad_u), (np.zeros(shape), np.zeros(shape)),
                 (np.zeros(shape), -np.ones(shape))]:
        with pytest.raises(hlb.HlbError) as ei:
            gpu.init(*args)
        assert ei.value.status == hlb.HLB_ENONFINITE
    gpu.init(np.zeros(shape))
    gpu.step(2)
    assert gpu.reduce()["finite"]


@pytest.mark.parametrize("plan", [(0, 1, 128, 64), (1, 5, 64, 7), (1, 5, 128, 16), (1, 5, 256, 40),
                                  (1, 2, 64, 9), (1, 3, 128, 100), (1, 1, 64, 1),
                                  (2, 5, 32, 0), (2, 5, 16, 0), (2, 2, 32, 0), (2, 3, 16, 256), (2, 1, 16, 0),
                                  (2, 2, 32, 512), (2, 2, 16, 1024), (2, 3, 48, 1024), (2, 5, 48, 512),
                                  (2, 1, 48, 256), (2, 3, 64, 1024), (2, 5, 64, 1024), (2, 5, 64, 256)])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("nx", [150, 152])
def test_substep_plans_agree(hlb, plan, storage, nx):
    """Every execution plan of the convection-diffusion substeps (one launch
    per substep, fused y-marching launches of several substeps with various
    block shapes, fused tiles of edge 16 to 64 with 256 to 1024 threads)
    computes the same step: ragged 150 x 83 and 152 x 83 lattices, m = 5
    split into fused launches of plan[1] substeps.  The fused tiles stage
    rows in 16-byte vectors where nx is a multiple of the vector width (152
    in both storages, 150 in FP64) and element by element otherwise."""
    if storage == "f64" and plan[0] == 1 and plan[2] == 256:
        pytest.skip("needs float storage (LDS size)")
    if plan[0] != 2 and nx == 152:
        pytest.skip("the second width matters only for the fused tiles")
    if plan[0] == 2:
        es = 8 if storage == "f64" else 4
        v, h = 16 // es, 3 * plan[1]
        ha = -(-h // v) * v
        if 4 * (plan[2] + 2 * h) * (plan[2] + 2 * ha) * es > 163840:
            pytest.skip("the staged tile exceeds a CU's LDS in this storage")
    shape = (83, nx)
    phi = _drop(shape, 20, BASE) + synth.spinodal(shape, seed=5, amp=0.02)
    u0 = np.zeros((2,) + shape)
    u0[0], u0[1] = 0.01, -0.007
    # both advection forms across the plans (fused tiles: by tile edge)
    advection = (plan[2] // 16) % 2 if plan[0] == 2 else plan[3] % 2
    gpu, ora = _pair(hlb, shape, storage, phi, None, u0, **BASE, N=0.3, Q=2.5, advection=advection)
    gpu.set_plan(*plan)
    assert gpu.plan == plan
    gpu.step(40)
    ora.step(40)
    d = _maxdiff(gpu, ora)
    tol = 1e-12 if storage == "f64" else 2e-6
    assert max(d.values()) < tol, (plan, d)


@pytest.mark.parametrize("plan", [(2, 3, 64, 1024), (2, 3, 32, 256), (2, 1, 16, 0), (2, 2, 48, 512),
                                  (2, 3, 16, 1024)])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("nx", [150, 152])
def test_fused_tiles_isotropic_laplacian(hlb, plan, storage, nx):
    """The fused tiles with the 9-point convection-diffusion Laplacian
    (cd_Q = 2/3, the isotropic one, for which the stability bound gives
    m = 3) against the oracle on ragged 150 x 83 and 152 x 83 lattices:
    its diagonal neighbours come from the neighbouring lanes' row vectors
    above and below, or from LDS at row ends and wavefront edges."""
    es = 8 if storage == "f64" else 4
    v, h = 16 // es, 3 * plan[1]
    ha = -(-h // v) * v
    if 4 * (plan[2] + 2 * h) * (plan[2] + 2 * ha) * es > 163840:
        pytest.skip("the staged tile exceeds a CU's LDS in this storage")
    shape = (83, nx)
    phi = _drop(shape, 20, BASE) + synth.spinodal(shape, seed=6, amp=0.02)
    u0 = np.zeros((2,) + shape)
    u0[0], u0[1] = -0.006, 0.009
    gpu, ora = _pair(hlb, shape, storage, phi, None, u0, **BASE, N=0.3, Q=2.5, cd_Q=2 / 3,
                     advection=plan[2] // 16 % 2)
    assert gpu.m == 3
    gpu.set_plan(*plan)
    gpu.step(40)
    ora.step(40)
    d = _maxdiff(gpu, ora)
    tol = 1e-12 if storage == "f64" else 2e-6
    assert max(d.values()) < tol, (plan, d)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_fused_plan_on_lattices_smaller_than_the_halo(hlb, storage):
    """The fused kernel's strip and march wrap around lattices narrower or
    shorter than its halo (3 rows per fused substep), with widths that are
    and are not multiples of the fused tile's vector width."""
    for shape in [(7, 9), (40, 5), (3, 100), (40, 8), (9, 12)]:
        for plan in [(1, 5, 64, 4), (2, 5, 16, 0), (2, 3, 64, 1024)]:
            if storage == "f64" and plan == (2, 3, 64, 1024):
                continue  # exceeds the LDS in FP64
            phi = synth.spinodal(shape, seed=sum(shape), amp=0.3)
            gpu, ora = _pair(hlb, shape, storage, phi, **BASE, N=0.3, Q=2.5)
            gpu.set_plan(*plan)
            gpu.step(6)
            ora.step(6)
            d = _maxdiff(gpu, ora)
            assert max(d.values()) < (1e-13 if storage == "f64" else 2e-6), (shape, plan, d)


def test_invalid_plans_rejected(hlb):
    gpu = hlb.Sim((32, 32), "f64", **BASE)
    for bad in [(3, 1, 64, 8), (1, 6, 128, 8), (1, 5, 96, 8), (1, 5, 256, 8), (1, 1, 64, 0), (1, 5, 32, 8),
                (2, 4, 16, 0), (2, 5, 64, 0), (2, 5, 48, 0), (2, 2, 32, 300), (2, 2, 32, 2048)]:
        with pytest.raises(hlb.HlbError) as e:
            gpu.set_plan(*bad)
        assert e.value.status == hlb.HLB_EINVAL
    g3 = hlb.Sim((8, 8, 8), "f32", **BASE)
    for bad in [(1, 5, 128, 8), (1, 1, 128, 8), (1, 2, 512, 8)]:
        with pytest.raises(hlb.HlbError):
            g3.set_plan(*bad)
    g3d = hlb.Sim((8, 8, 8), "f64", **BASE)
    with pytest.raises(hlb.HlbError):
        g3d.set_plan(1, 1, 1024, 8)
    g3w = hlb.Sim((8, 8, 8), "f32", **BASE, cd_Q=1 / 3)
    g3w.set_plan(1, 1, 512, 8)
    with pytest.raises(hlb.HlbError):
        g3w.set_plan(1, 1, 1024, 8)
    g2 = hlb.Sim((32, 32), "f32", **BASE, cd_Q=2 / 3)
    assert g2.plan[0] == 0
    with pytest.raises(hlb.HlbError):
        g2.set_plan(1, 3, 128, 8)


def test_autotune_keeps_state_and_parity(hlb):
    shape = (256, 256)
    phi = synth.spinodal(shape, seed=2)
    gpu, ora = _pair(hlb, shape, "f32", phi, **BASE, N=0.3, Q=2.5)
    gpu.step(5)
    ora.step(5)
    before = gpu.state()
    us = gpu.autotune()
    after = gpu.state()
    assert us > 0
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    gpu.step(20)
    ora.step(20)
    d = _maxdiff(gpu, ora)
    assert d["phi"] < 1e-5 and d["u"] < 1e-5, (gpu.plan, d)


@pytest.mark.parametrize("plan", [(0, 1, 128, 64), (1, 1, 256, 5), (1, 1, 512, 7), (1, 1, 1024, 16)])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("advection", [0, 1])
@pytest.mark.parametrize("cd_Q", [1.0, 1 / 3], ids=["lap7", "lap19"])
def test_d3q19_substep_plans_agree(hlb, plan, storage, advection, cd_Q):
    """The 3D z-marching substep kernels (block shapes 16x16, 32x16, 64x16,
    various segment heights; the 7-point convection-diffusion Laplacian,
    m = 10, and the isotropic 19-point one, m = 3) and the tiled kernel give
    the oracle's step on a ragged 70 x 37 x 21 lattice."""
    if storage == "f64" and plan[2] > 512:
        pytest.skip("bw = 1024 needs float storage")
    if cd_Q != 1.0 and plan[2] > 512:
        pytest.skip("the 19-point march takes at most 512 threads (registers)")
    shape = (21, 37, 70)
    phi = _drop(shape, 8, BASE) + synth.spinodal(shape, seed=9, amp=0.02)
    u0 = np.zeros((3,) + shape)
    u0[0], u0[1], u0[2] = 0.004, -0.006, 0.005
    gpu, ora = _pair(hlb, shape, storage, phi, None, u0, **BASE, N=1 / 6, Q=1 / 3, advection=advection, cd_Q=cd_Q)
    gpu.set_plan(*plan)
    gpu.step(4)
    ora.step(4)
    d = _maxdiff(gpu, ora)
    tol = 1e-12 if storage == "f64" else 2e-6
    assert max(d.values()) < tol, (plan, d)


@pytest.mark.parametrize("cd_Q", [1.0, 1 / 3], ids=["lap7", "lap19"])
def test_d3q19_march_thin_lattices(hlb, cd_Q):
    """z-marching with fewer planes than its halo, and x-y tiles wider than
    the lattice (periodic images)."""
    for shape in [(3, 12, 40), (9, 5, 6), (1, 8, 8)]:
        phi = synth.spinodal(shape, seed=sum(shape), amp=0.3)
        gpu, ora = _pair(hlb, shape, "f64", phi, **BASE, N=1 / 6, Q=1 / 3, cd_Q=cd_Q)
        gpu.set_plan(1, 1, 256, 2)
        gpu.step(3)
        ora.step(3)
        d = _maxdiff(gpu, ora)
        assert max(d.values()) < 1e-13, (shape, d)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_checkpoint_resume_bit_exact(hlb, storage):
    """hlb_save / hlb_load: a run resumed from a checkpoint (into a context
    created with other parameters, which the checkpoint's replace) is bit
    for bit the uninterrupted run, and the step counter comes back."""
    shape = (48, 80)
    phi = _drop(shape, 12, BASE)
    a = hlb.Sim(shape, storage, **BASE, N=0.3, Q=2.5)
    a.init(phi)
    a.step(7)
    blob = a.save()
    a.step(9)
    fa, sa = a.fields(), a.state()
    b = hlb.Sim(shape, storage, **dict(BASE, tau=0.7), N=0.5, Q=1.0)
    b.load(blob)
    assert b.reduce()["step"] == 7
    assert abs(b._params.tau - 1.0) < 1e-15 and abs(b._params.N - 0.3) < 1e-15
    b.step(9)
    fb, sb = b.fields(), b.state()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1])
    lib = hlb.load()
    other = hlb.Sim((48, 81), storage, **BASE)
    with pytest.raises(hlb.HlbError) as e:
        other.load(blob)
    assert e.value.status == hlb.HLB_ESHAPE
    with pytest.raises(hlb.HlbError) as e:
        b.load(b"not a checkpoint" * 8)
    assert e.value.status == hlb.HLB_EINVAL
    with pytest.raises(hlb.HlbError) as e:
        b.load(blob[: len(blob) // 2])
    assert e.value.status == hlb.HLB_EINVAL
    buf = ctypes.create_string_buffer(16)
    assert lib.hlb_save(b.ctx, buf, 16) == hlb.HLB_EINVAL


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_checkpoint_keeps_the_plan(hlb, storage):
    """Plans agree only up to rounding order, so a checkpoint carries the
    substep plan: a run saved under a non-default plan (here a 2 + 2 + 1
    march, and the autotuned plan) and resumed in a fresh context, which
    starts with the default plan, is bit for bit the uninterrupted run."""
    shape = (64, 96)
    phi = _drop(shape, 14, BASE)
    for plan in ((1, 2, 64, 16), None):
        a = hlb.Sim(shape, storage, **BASE, N=0.3, Q=2.5)
        a.init(phi)
        if plan is None:
            a.autotune()
        else:
            a.set_plan(*plan)
        a.step(5)
        blob = a.save()
        saved_plan = a.plan
        a.step(11)
        fa = a.fields()
        b = hlb.Sim(shape, storage, **BASE, N=0.3, Q=2.5)
        b.load(blob)
        assert b.plan == saved_plan
        b.step(11)
        fb = b.fields()
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), (plan, k)
        a.close()
        b.close()


def test_kernel_names_and_timing_leave_the_state_alone(hlb):
    """hlb_kernel_name gives the profiler's names of the instantiations a
    step launches, and hlb_time_kernels neither changes the state nor the
    step counter: a run with timings in between equals one without."""
    shape = (96, 128)
    phi = _drop(shape, 20, BASE)
    a = hlb.Sim(shape, "f32", **BASE, N=0.3, Q=2.5)
    b = hlb.Sim(shape, "f32", **BASE, N=0.3, Q=2.5)
    for s in (a, b):
        s.init(phi)
        s.set_plan(2, 5, 32, 256)
    assert a.kernel_name(0) == "hlb::k_lb<hlb::D2Q9, float, 64, 8, 1>"
    assert a.kernel_name(1) == "hlb::k_ch_tile<float, 5, 32, false, 256, false>"
    a.step(3)
    us = a.time_kernels(5)
    assert all(u > 0 for u in us) and us[2] >= 0.9 * us[1]  # one launch per step here
    a.step(4)
    b.step(7)
    assert a.reduce()["step"] == 7
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    a.set_plan(1, 2, 64, 16)
    assert a.kernel_name(1) == "hlb::k_ch_march<float, 2, 64, false>"
    a.set_plan(0, 1, 128, 64)
    assert a.kernel_name(1) == "hlb::k_ch<hlb::D2Q9, float, 64, 16, 1, true>"
    c = hlb.Sim((16, 16, 16), "f32", **BASE, N=1 / 6, Q=1 / 3, advection=1)
    c.set_plan(1, 1, 512, 8)
    assert c.kernel_name(0) == "hlb::k_lb<hlb::D3Q19, float, 64, 4, 4>"
    assert c.kernel_name(1) == "hlb::k_ch_march3<float, 32, 16, true>"


TILE2_PLANS = [(3, 5, 64, 1024), (3, 5, 48, 1024), (3, 5, 32, 1024), (3, 5, 32, 512), (3, 3, 64, 1024),
               (3, 3, 48, 512), (3, 2, 32, 512), (3, 2, 64, 1024), (3, 1, 32, 1024), (3, 1, 64, 512)]


def _tile2_or_skip(hlb, gpu, plan):
    try:
        gpu.set_plan(*plan)
    except hlb.HlbError as e:
        pytest.skip(f"not a valid plan here: {e}")
    assert gpu.plan == plan


@pytest.mark.parametrize("plan", TILE2_PLANS)
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("nx", [150, 152])
@pytest.mark.parametrize("advection", [0, 1])
def test_fixed_mapping_fused_tiles_agree(hlb, plan, storage, nx, advection):
    """The fused tiles with a fixed vector-to-thread mapping (plan kind 3:
    phi, h and the potential in registers, the advection half-step as five
    precomputed coefficients per site) against the oracle on ragged
    150 x 83 and 152 x 83 lattices, both advection forms, m = 5 in fused
    launches of plan[1] substeps.  A plan is skipped only where its staged
    box exceeds the LDS or three vectors per thread."""
    shape = (83, nx)
    phi = _drop(shape, 20, BASE) + synth.spinodal(shape, seed=7, amp=0.02)
    u0 = np.zeros((2,) + shape)
    u0[0], u0[1] = 0.012, -0.008
    gpu, ora = _pair(hlb, shape, storage, phi, None, u0, **BASE, N=0.3, Q=2.5, advection=advection)
    _tile2_or_skip(hlb, gpu, plan)
    gpu.step(40)
    ora.step(40)
    d = _maxdiff(gpu, ora)
    tol = 1e-12 if storage == "f64" else 2e-6
    assert max(d.values()) < tol, (plan, d)


@pytest.mark.parametrize("plan", [(3, 3, 64, 1024), (3, 3, 32, 512), (3, 1, 48, 1024)])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_fixed_mapping_fused_tiles_isotropic_laplacian(hlb, plan, storage):
    """Plan kind 3 with the 9-point convection-diffusion Laplacian
    (cd_Q = 2/3, m = 3), whose diagonal neighbours come from the
    neighbouring lanes' rows above and below or from LDS."""
    shape = (83, 150)
    phi = _drop(shape, 20, BASE) + synth.spinodal(shape, seed=8, amp=0.02)
    u0 = np.zeros((2,) + shape)
    u0[0], u0[1] = -0.006, 0.009
    gpu, ora = _pair(hlb, shape, storage, phi, None, u0, **BASE, N=0.3, Q=2.5, cd_Q=2 / 3, advection=plan[2] % 2)
    assert gpu.m == 3
    _tile2_or_skip(hlb, gpu, plan)
    gpu.step(40)
    ora.step(40)
    d = _maxdiff(gpu, ora)
    tol = 1e-12 if storage == "f64" else 2e-6
    assert max(d.values()) < tol, (plan, d)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_fixed_mapping_fused_tiles_on_small_lattices(hlb, storage):
    """Plan kind 3 on lattices narrower or shorter than its staged box (the
    box wraps several times), with widths that are and are not multiples of
    the vector width."""
    for shape in [(7, 9), (40, 5), (3, 100), (40, 8), (9, 12), (1, 1)]:
        for plan in [(3, 5, 32, 1024), (3, 3, 64, 1024), (3, 1, 32, 512)]:
            phi = synth.spinodal(shape, seed=sum(shape) + 1, amp=0.3)
            gpu, ora = _pair(hlb, shape, storage, phi, **BASE, N=0.3, Q=2.5)
            try:
                gpu.set_plan(*plan)
            except hlb.HlbError:
                continue  # beyond the LDS or the register budget in this storage
            gpu.step(6)
            ora.step(6)
            d = _maxdiff(gpu, ora)
            assert max(d.values()) < (1e-13 if storage == "f64" else 2e-6), (shape, plan, d)
