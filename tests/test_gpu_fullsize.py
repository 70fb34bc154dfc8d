"""Parity with the FP64 oracle at the benchmark's full sizes, in the launch
configuration the benchmark times (the autotuned plan of the same
lattice), over a short horizon: spinodal decomposition amplifies rounding
differences, so pointwise comparison is meaningful only over a few tens of
steps (reading C19).  Every output site is compared.  FP32 shifted storage:
max |dphi|, |du|, |dn| <= 2e-6 (the 128^2 drop's 1e-5 over 1000 steps is the
stated target; these runs are 2 to 20 steps long).
"""
import numpy as np
import pytest

from oracle import orc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hlb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0902_3921_amd import hlb as mod

    mod.load()
    return mod


@pytest.mark.parametrize("name,steps,stencil", [
    ("d2q9_spinodal_1024", 20, None),
    ("d2q9_spinodal_1024", 20, "standard"),
    ("d2q9_spinodal_4096", 4, None),
    ("d3q19_spinodal_256", 2, None),
])
def test_benchmark_workload_full_size(hlb, name, steps, stencil):
    import bench

    shape, storage, kw, desc = bench.WORKLOADS[name]
    if stencil == "standard":
        kw = dict(kw, **bench.STANDARD_STENCIL)
    phi0 = bench.make_inputs(name, shape)
    sim = hlb.Sim(shape, storage, **kw)
    sim.init(phi0)
    sim.autotune()
    print(f"{name} ({stencil or 'paper'} stencil): plan {sim.plan}, m = {sim.m}, {steps} steps", flush=True)
    sim.step(steps)
    g = sim.fields()
    sim.close()
    o = orc.Oracle(shape, m=hlb.check_params(0 if len(shape) == 2 else 1, **kw), **kw)
    o.init(phi0)
    o.step(steps)
    r = o.fields()
    d = {k: float(np.abs(g[k] - r[k]).max()) for k in ("n", "u", "phi")}
    print(f"max differences {d}", flush=True)
    assert max(d.values()) <= 2e-6, d
