"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every function include/hlb.h declares, and parameter validation
behaves as documented (all of it runs before any device call)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hlb():
    from paper_0902_3921_amd import build, hlb as mod

    if not os.path.exists(build.LIB):
        build.build()
    mod.load()
    return mod


def _declared():
    names = set()
    for h in ("hlb.h", "sur.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b((?:hlb|sur)_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_exports_every_declared_symbol(hlb):
    from paper_0902_3921_amd import sur

    declared = _declared()
    assert set(declared) == set(hlb.EXPORTS) | set(sur.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", hlb.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT ((?:hlb|sur)_[a-z_]+)$", out, flags=re.M))
    assert set(declared) <= exported, set(declared) - exported
    for name in declared:
        assert getattr(hlb.load(), name)


def test_defaults(hlb):
    p = hlb.params()
    assert (p.a, p.b, p.kappa, p.tau, p.gamma) == (-0.1, 0.1, 0.1, 1.0, 1.0)
    assert (p.N, p.Q, p.cd_Q, p.fd_substeps, p.force_form, p.advection, p.rho0) == (0.3, 2.5, 1.0, 0, 1, 0, 1.0)
    assert hlb.version().startswith("hlb")


def test_substep_selection(hlb):
    """Sec. 2.3, Delta t_LB = m Delta t_FD: the automatic m is the smallest one
    with Gamma dt (kappa s^2 + a_eff s) <= 1.8 (s = 8 for the 5-point, 12 for
    the 7-point Laplacian, 16/3 for the isotropic 9/19-point ones)."""
    assert hlb.check_params(hlb.D2Q9) == 5
    assert hlb.check_params(hlb.D3Q19) == 10
    assert hlb.check_params(hlb.D2Q9, cd_Q=2 / 3) == 3
    assert hlb.check_params(hlb.D3Q19, cd_Q=1 / 3) == 3
    assert hlb.check_params(hlb.D2Q9, a=-1e-3, b=1e-3, kappa=3e-3, gamma=5.0) == 1
    assert hlb.check_params(hlb.D2Q9, kappa=0.2) == 8
    assert hlb.check_params(hlb.D2Q9, m=4) == 4  # rate/m = 2: the marginal bound is allowed
    with pytest.raises(hlb.HlbError) as e:
        hlb.check_params(hlb.D2Q9, m=3)
    assert e.value.status == hlb.HLB_EUNSTABLE


@pytest.mark.parametrize("bad", [dict(tau=0.5), dict(tau=0.2), dict(b=0.0), dict(kappa=-1e-3), dict(gamma=-1.0),
                                 dict(rho0=0.0), dict(force_form=2), dict(advection=3), dict(cd_model=2), dict(tau_phi=0.4),
                                 dict(m=-1), dict(a=float("nan")), dict(g_ext=(0, 0, 1e-5)),
                                 dict(cd_Q=-1.0)])
def test_invalid_parameters(hlb, bad):
    with pytest.raises(hlb.HlbError) as e:
        hlb.check_params(hlb.D2Q9, **bad)
    assert e.value.status == hlb.HLB_EINVAL


def test_workspace_size_and_shape_errors(hlb):
    ns = 1024 * 1024
    b = hlb.workspace_size(hlb.D2Q9, "f32", 1024, 1024, 1)
    # two population copies, two phi, u*, double staging, reduction partials
    assert b >= (2 * 9 + 2 + 2) * 4 * ns + 5 * 8 * ns
    assert hlb.workspace_size(hlb.D2Q9, "f64", 1024, 1024, 1) > b
    for dims in [(0, 4, 1), (4, -1, 1), (4, 4, 2)]:
        with pytest.raises(hlb.HlbError) as e:
            hlb.workspace_size(hlb.D2Q9, "f32", *dims)
        assert e.value.status == hlb.HLB_ESHAPE
    with pytest.raises(hlb.HlbError) as e:
        hlb.workspace_size(hlb.D3Q19, "f32", 2048, 2048, 1024)
    assert e.value.status == hlb.HLB_ESHAPE
    with pytest.raises(hlb.HlbError):
        hlb.workspace_size(7, "f32", 4, 4, 1)


def test_create_rejects_before_touching_the_device(hlb):
    """Invalid shapes, parameters and a missing workspace are rejected on
    the host (no HIP call is made)."""
    lib = hlb.load()
    ctx = ctypes.c_void_p()
    p = hlb.params()
    st = lib.hlb_create(ctypes.byref(ctx), 0, 1, 16, 16, 1, ctypes.byref(p), None, 0, None)
    assert st == hlb.HLB_ESHAPE and not ctx.value
    assert b"workspace" in lib.hlb_last_error(None)
    p.tau = 0.4
    st = lib.hlb_create(ctypes.byref(ctx), 0, 1, 16, 16, 1, ctypes.byref(p), None, 0, None)
    assert st == hlb.HLB_EINVAL
    assert b"tau" in lib.hlb_last_error(None)


def test_batch_workspace_size_and_shape_errors(hlb):
    shapes = [(64, 64), (96, 128), (7, 5)]
    b = hlb.batch_workspace_size("f32", shapes)
    sites = sum(ny * nx for ny, nx in shapes)
    # per simulation: two population copies, two phi and u*, all float
    assert b >= (2 * 9 + 2 + 2) * 4 * sites
    assert hlb.batch_workspace_size("f64", shapes) > b
    for bad in ([(0, 4)], [(4, 4), (4, -2)]):
        with pytest.raises(hlb.HlbError) as e:
            hlb.batch_workspace_size("f32", bad)
        assert e.value.status == hlb.HLB_ESHAPE
    with pytest.raises(hlb.HlbError) as e:
        hlb.batch_workspace_size("f32", [])
    assert e.value.status == hlb.HLB_EINVAL


def test_batch_create_rejects_before_touching_the_device(hlb):
    """A batch names the simulation whose parameters are invalid, and a
    missing workspace is rejected, all on the host."""
    lib = hlb.load()
    b = ctypes.c_void_p()
    nx = (ctypes.c_int * 2)(16, 32)
    ny = (ctypes.c_int * 2)(16, 8)
    ps = (hlb.Params * 2)(hlb.params(), hlb.params(tau=0.4))
    st = lib.hlb_batch_create(ctypes.byref(b), 1, 2, nx, ny, ps, None, 0, None)
    assert st == hlb.HLB_EINVAL and not b.value
    assert b"simulation 1" in lib.hlb_batch_last_error(None)
    ps[1] = hlb.params()
    st = lib.hlb_batch_create(ctypes.byref(b), 1, 2, nx, ny, ps, None, 0, None)
    assert st == hlb.HLB_ESHAPE and not b.value
    assert b"workspace" in lib.hlb_batch_last_error(None)


def test_surrogate_parameter_count_and_config_checks(hlb):
    """The library's parameter layout has the oracle's size for several
    widths, and invalid configurations are rejected on the host."""
    from oracle import unet
    from paper_0902_3921_amd import sur

    for widths in ((32, 64, 128), (8, 16, 24), (5, 7, 3)):
        c0, c1, c2 = widths
        assert sur.param_count(c0=c0, c1=c1, c2=c2) == unet.param_count(c0, c1, c2)
    lib = sur._lib()
    n = ctypes.c_size_t()
    for bad in (dict(height=30), dict(width=0), dict(batch=0), dict(c1=0)):
        c = sur.config(**bad)
        assert lib.sur_workspace_size(ctypes.byref(c), ctypes.byref(n)) == hlb.HLB_EINVAL
    c = sur.config(batch=4, height=64, width=64)
    assert lib.sur_workspace_size(ctypes.byref(c), ctypes.byref(n)) == hlb.HLB_OK
    # activations and gradients at full resolution alone: 4 images x 64 x 64 x (3 + 3 + 32 + 96 + ...) floats
    assert n.value > 4 * 64 * 64 * (2 * 3 + 2 * 32 + 2 * 96) * 4
    net = ctypes.c_void_p()
    assert lib.sur_create(ctypes.byref(net), ctypes.byref(c), None, 0, None) == hlb.HLB_ESHAPE
    assert b"workspace" in lib.sur_last_error(None)


def test_d2q5_model_parameters(hlb):
    """The D2Q5 convection-diffusion alternative (cd_model 1): D2Q9 only, no
    substeps, and the explicit bound of a whole LB step (m = 1): accepted at
    the paper's parameters (Sec. 3), HLB_EUNSTABLE at a = -0.1, kappa = 0.1,
    Gamma = 1; its two population buffers enlarge the workspace."""
    paper = dict(a=-1e-3, b=1e-3, kappa=3e-3, gamma=5.0, cd_model=1)
    assert hlb.check_params(hlb.D2Q9, **paper) == 1
    assert hlb.check_params(hlb.D2Q9, **paper, tau_phi=0.8) == 1
    with pytest.raises(hlb.HlbError) as e:
        hlb.check_params(hlb.D2Q9, cd_model=1)
    assert e.value.status == hlb.HLB_EUNSTABLE
    for bad in (dict(fd_substeps=2), dict(tau_phi=0.5)):
        with pytest.raises(hlb.HlbError) as e:
            hlb.check_params(hlb.D2Q9, **paper, **bad)
        assert e.value.status == hlb.HLB_EINVAL
    with pytest.raises(hlb.HlbError) as e:
        hlb.check_params(hlb.D3Q19, **paper)
    assert e.value.status == hlb.HLB_EINVAL
    p = hlb.params(**paper)
    assert p.tau_phi == 0.0 and hlb.params().cd_model == 0
    for storage, es in (("f32", 4), ("f64", 8)):
        base = hlb.workspace_size(hlb.D2Q9, storage, 96, 80, 1)
        assert hlb.workspace_size(hlb.D2Q9, storage, 96, 80, 1, hlb.params()) == base
        with5 = hlb.workspace_size(hlb.D2Q9, storage, 96, 80, 1, p)
        assert 2 * 5 * 96 * 80 * es <= with5 - base < 2 * 5 * 96 * 80 * es + 512
