"""Host-side logic of bench.py (no GPU): the one-GPU contract, the
algorithmic bytes behind the roofline figures, the traffic lookup from the
committed rocprofv3 summaries, and the validity of every workload's
parameters under the library's own checks."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("d,q,es,lb,ch,step", [
    (2, 9, 4, 84, 16, 80),     # D2Q9 FP32: 18 population moves + phi + u*; CH phi, u*, phi'; minimum 80
    (2, 9, 8, 168, 32, 160),   # D2Q9 FP64
    (3, 19, 4, 168, 20, 160),  # D3Q19 FP32
    (3, 19, 8, 336, 40, 320),  # D3Q19 FP64
])
def test_algorithmic_bytes_per_lattice_update(d, q, es, lb, ch, step):
    assert bench.algorithmic_bytes(d, q, es) == (lb, ch, step)


def test_measured_traffic_from_committed_profiles():
    """Each committed summary lists its dominant kernel with FETCH_SIZE and
    WRITE_SIZE; the lookup scales them by the copy calibration, and returns
    None for a kernel it does not list or a workload without a summary."""
    t = bench.measured_traffic("d2q9_spinodal_4096", "hlb::k_lb<hlb::D2Q9, float, ...>")
    if t is None:
        pytest.skip("the committed summary was taken on other library sources")
    alg = 84 * 4096 * 4096
    assert 0.95 * alg < t < 1.2 * alg  # within a few percent of the algorithmic bytes at 4096^2
    assert bench.measured_traffic("d2q9_spinodal_4096", "hlb::no_such_kernel<float>") is None
    assert bench.measured_traffic("no_such_workload", "hlb::k_lb<hlb::D2Q9, float, ...>") is None


@pytest.mark.parametrize("name", [n for n, w in bench.WORKLOADS.items() if w[0] is not None])
def test_workload_parameters_pass_the_library_checks(name):
    from paper_0902_3921_amd import hlb

    shape, storage, kw, desc = bench.WORKLOADS[name]
    m = hlb.check_params(0 if len(shape) == 2 else 1, **kw)
    assert m >= 1
    phi = bench.make_inputs(name, shape)
    assert phi.shape == tuple(shape) and np.isfinite(phi).all()


def test_batch_workload_recipe():
    specs, params, phis = bench.batch_workload()
    assert len(specs) == len(params) == len(phis) == 512
    assert all(64 <= sp["shape"][0] <= 256 and sp["shape"][0] == sp["shape"][1] for sp in specs)
    assert all(phi.shape == sp["shape"] for sp, phi in zip(specs, phis))
    assert sum(sp["shape"][0] * sp["shape"][1] for sp in specs) == 14_766_734
