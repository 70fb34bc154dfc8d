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
    text = open(os.path.join(ROOT, "include", "hlb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hlb_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(hlb):
    declared = _declared()
    assert set(declared) == set(hlb.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", hlb.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (hlb_[a-z_]+)$", out, flags=re.M))
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
                                 dict(rho0=0.0), dict(force_form=2), dict(advection=3), dict(reserved=1),
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
