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


def test_profile_figures_match_the_exact_instantiation(tmp_path, monkeypatch):
    """The traffic and the kernel-trace duration come from the summary rows
    of exactly the dominant kernel's instantiation, not from other
    instantiations of the same template (autotuning candidates), and only
    from a summary taken on the current library sources."""
    from paper_0902_3921_amd import build

    prof = tmp_path / "profiles"
    prof.mkdir()
    rows = [
        f"library source hash: {build.source_hash()}",
        "| kernel | calls | avg us | min us | max us | % time |",
        "|---|---|---|---|---|---|",
        "| hlb::k_ch_tile<float, 5, 64, false, 1024, false> | 40 | 19.50 | 18.0 | 21.0 | 40.0 |",
        "| hlb::k_ch_tile<float, 5, 64, false, 512, false> | 4 | 22.00 | 21.0 | 23.0 | 1.0 |",
        "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB |",
        "|---|---|---|---|",
        "| hlb::k_ch_tile<float, 5, 64, false, 1024, false> | 10 | 7000.0 | 4096.0 |",
        "| hlb::k_ch_tile<float, 5, 64, false, 512, false> | 4 | 9000.0 | 4096.0 |",
    ]
    (prof / "w.md").write_text("\n".join(rows) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    t, us = bench.profile_figures("w", "hlb::k_ch_tile<float, 5, 64, false, 1024, false>")
    assert us == 19.5
    assert t == 7000.0 * 1024 * bench.FETCH_SCALE + 4096.0 * 1024 * bench.WRITE_SCALE
    assert bench.profile_figures("w", "hlb::k_ch_tile<float, 5, 64>") == (None, None)
    assert bench.profile_figures("missing", "x") == (None, None)
    (prof / "w.md").write_text("\n".join(["library source hash: 0000"] + rows[1:]) + "\n")
    assert bench.profile_figures("w", "hlb::k_ch_tile<float, 5, 64, false, 1024, false>") == (None, None)


@pytest.mark.parametrize("m,plan,seq", [
    (5, (2, 5, 64, 1024), [5]), (5, (1, 2, 128, 64), [2, 2, 1]), (5, (0, 1, 128, 64), [1] * 5),
    (10, (1, 1, 1024, 52), [1] * 10), (4, (2, 5, 32, 256), [3, 1]), (8, (2, 5, 32, 256), [5, 3]),
])
def test_launch_sequence(m, plan, seq):
    assert bench.launch_sequence(m, plan) == seq


def test_mall_residency():
    assert bench.state_bytes((1024, 1024), "f32") < bench.MALL_BYTES
    assert bench.state_bytes((4096, 4096), "f32") > bench.MALL_BYTES
    assert bench.state_bytes((256, 256, 256), "f32") > bench.MALL_BYTES


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
