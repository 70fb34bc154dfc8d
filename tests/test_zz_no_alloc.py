"""hlb_create_noalloc (for callers that cannot allocate device memory): a
context over the library's static device array computes exactly what a
context over a caller workspace computes, on two calls in a row (the second
with a smaller lattice), and the documented limits hold."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

BASE = dict(a=-0.1, b=0.1, kappa=0.1, tau=1.0, gamma=1.0, N=0.3, Q=2.5)


@pytest.fixture(scope="module")
def hlb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0902_3921_amd import hlb as mod

    mod.load()
    return mod


def _run(hlb, shape, storage, steps, noalloc, **kw):
    d = len(shape)
    phi = synth.drop(shape, min(shape) / 4, 1.0, np.sqrt(2.0))
    u0 = synth.uniform_velocity(shape, (0.01, -0.005, 0.002)[:d])
    sim = hlb.Sim(shape, storage, noalloc=noalloc, **kw)
    sim.init(phi, None, u0)
    sim.step(steps)
    out = sim.fields()
    f, ph = sim.state()
    red = sim.reduce()
    sim.close()
    return out, f, ph, red


@pytest.mark.parametrize("first,second", [
    (((160, 224), "f32"), ((48, 80), "f64")),
    (((24, 20, 28), "f32"), ((9, 14, 11), "f32")),
])
def test_noalloc_context_matches_a_workspace_context(hlb, first, second):
    for shape, storage in (first, second):  # two calls in a row, the second smaller
        kw = dict(BASE) if len(shape) == 2 else dict(BASE, N=1 / 6, Q=1 / 3)
        ref = _run(hlb, shape, storage, 37, False, **kw)
        got = _run(hlb, shape, storage, 37, True, **kw)
        for k in ref[0]:
            assert np.array_equal(ref[0][k], got[0][k]), (shape, k)
        assert np.array_equal(ref[1], got[1]) and np.array_equal(ref[2], got[2])
        for k in ("mass", "phi_sum", "kinetic", "umax"):
            assert ref[3][k] == got[3][k], (shape, k)


def test_noalloc_limits(hlb):
    lib = hlb.load()
    ctx = ctypes.c_void_p()
    p = hlb.params(**BASE)
    # a lattice whose workspace exceeds the static array is rejected with a message
    st = lib.hlb_create_noalloc(ctypes.byref(ctx), hlb.D2Q9, hlb.F32_SHIFTED, 1024, 1024, 1, ctypes.byref(p), None)
    assert st == hlb.HLB_ESHAPE and not ctx.value
    assert b"static array" in lib.hlb_last_error(None)
    # one live context per device; destroying it frees the array
    a = hlb.Sim((32, 32), "f32", noalloc=True, **BASE)
    st = lib.hlb_create_noalloc(ctypes.byref(ctx), hlb.D2Q9, hlb.F32_SHIFTED, 16, 16, 1, ctypes.byref(p), None)
    assert st == hlb.HLB_ESTATE and not ctx.value
    a.close()
    b = hlb.Sim((16, 16), "f32", noalloc=True, **BASE)
    b.init(np.zeros((16, 16)))
    b.step(2)
    assert b.reduce()["step"] == 2
    b.close()
