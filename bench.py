"""Benchmark of the hybrid lattice Boltzmann timestep on one MI355X.

A step is one full timestep of the method: the force + collide-and-stream
kernel and the m convection-diffusion substeps.  The default workload is the
D2Q9 spinodal decomposition on a 1024 x 1024 periodic lattice with FP32
shifted populations (a = -0.1, b = 0.1, kappa = 0.1, tau = 1, Gamma = 1,
m = 5, the paper's stencil N = 0.3, Q = 2.5), phi ~ U(-0.01, 0.01) from
seed 0, n = 1, u = 0; the standard stencil (N = 1/2, Q = 1) is timed beside
it, and the 256^3 D3Q19 spinodal (m = 10) is measured as a sub-record.
Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
N_CU, CLOCK_HZ = 256, 2.4e9  # MI355X compute units and peak engine clock
# rocprofv3 counter scale, from a 1 GiB device copy (1 GiB read, 1 GiB written)
# that reads FETCH_SIZE = 524,300 KiB and WRITE_SIZE = 1,048,576 KiB
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0

BASE = dict(a=-0.1, b=0.1, kappa=0.1, tau=1.0, gamma=1.0)
# the paper's parameters (Sec. 3): -a = b = 1e-3, kappa = 3e-3, Gamma = 5, m = 1
PAPER = dict(a=-1e-3, b=1e-3, kappa=3e-3, tau=1.0, gamma=5.0)
PAPER_STENCIL = dict(N=0.3, Q=2.5)
STANDARD_STENCIL = dict(N=0.5, Q=1.0)

WORKLOADS = {
    # name: (shape, storage, stencil, description)
    "d2q9_spinodal_1024": ((1024, 1024), "f32", dict(BASE, **PAPER_STENCIL),
                           "D2Q9 spinodal 1024x1024 periodic, FP32 shifted populations"),
    # at the paper's parameters, where the D2Q5 convection-diffusion model is
    # stable; it is timed beside the finite-difference model (m = 1)
    "d2q9_spinodal_1024_paper": ((1024, 1024), "f32", dict(PAPER, **PAPER_STENCIL),
                                 "D2Q9 spinodal 1024x1024 periodic at the paper's parameters, FP32 shifted "
                                 "populations"),
    "d2q9_spinodal_4096": ((4096, 4096), "f32", dict(BASE, **PAPER_STENCIL),
                           "D2Q9 spinodal 4096x4096 periodic, FP32 shifted populations"),
    "d2q9_drop_128_f64": ((128, 128), "f64", dict(BASE, **PAPER_STENCIL),
                          "D2Q9 drop R=20 128x128 periodic, FP64"),
    "d3q19_spinodal_256": ((256, 256, 256), "f32", dict(BASE, N=1 / 6, Q=1 / 3),
                           "D3Q19 spinodal 256^3 periodic, FP32 shifted populations"),
    # the same with the isotropic 19-point convection-diffusion Laplacian
    # (Q = 1/3, R = 1/6), whose smaller largest eigenvalue allows m = 3
    "d3q19_spinodal_256_iso": ((256, 256, 256), "f32", dict(BASE, N=1 / 6, Q=1 / 3, cd_Q=1 / 3),
                               "D3Q19 spinodal 256^3 periodic, isotropic CH Laplacian (m = 3), "
                               "FP32 shifted populations"),
    # shape None: a batch of independent simulations (batch_workload)
    "d2q9_batch_512": (None, "f32", dict(BASE, **PAPER_STENCIL),
                       "512 independent D2Q9 drop/slab simulations, L ~ U{64..256}, kappa ~ U(0.05, 0.2), "
                       "tau ~ U(0.6, 1.5), FP32 shifted populations, one batch"),
}


def batch_workload(nsim=512, seed=0):
    """The batched workload: specs from synth.batch_specs (square lattices of
    side L ~ U{64..256}, kappa ~ U(0.05, 0.2), tau ~ U(0.6, 1.5), a drop of
    radius ~ U(8, L/4) or a slab with two flat interfaces), a = -0.1,
    b = 0.1, Gamma = 1, the paper's stencil N = 0.3, Q = 2.5, and the
    equilibrium tanh profile of amplitude sqrt(-a/b) = 1 and width
    sqrt(-2 kappa/a).  Returns (specs, params, phis)."""
    import numpy as np

    import synth

    specs = synth.batch_specs(nsim, seed)
    params, phis = [], []
    for s in specs:
        p = dict(BASE, kappa=s["kappa"], tau=s["tau"], **PAPER_STENCIL)
        w = np.sqrt(-2 * s["kappa"] / p["a"])
        if s["kind"] == "drop":
            phi = synth.drop(s["shape"], s["radius"], 1.0, w, center=s["center"])
        else:
            phi = synth.slab(s["shape"], s["x0"], s["x1"], 1.0, w, axis=s["axis"])
        params.append(p)
        phis.append(phi)
    return specs, params, phis


def algorithmic_bytes(d: int, q: int, es: int):
    """Bytes per lattice update that each kernel must move (and the whole
    step's minimum): the collide-and-stream kernel reads and writes every
    population once, reads phi and writes u*; a convection-diffusion substep
    reads phi and u* and writes phi; the whole step at its minimum reads and
    writes every population and phi once."""
    lb = (2 * q + 1 + d) * es
    ch = (2 + d) * es
    step_min = (2 * q + 2) * es
    return lb, ch, step_min


def make_inputs(name, shape):
    import numpy as np

    import synth

    if "drop" in name:
        a, b, kappa = BASE["a"], BASE["b"], BASE["kappa"]
        return synth.drop(shape, 20, np.sqrt(-a / b), np.sqrt(-2 * kappa / a))
    return synth.spinodal(shape, seed=0)


def launch_sequence(m: int, plan) -> list:
    """Substeps of each convection-diffusion launch of one step under a plan
    (kind, fuse, bw, seg): one per launch for kind 0 and for D3Q19; kind 1
    fuses up to `fuse`; kinds 2 and 3 fuse 1, 2, 3 or 5 (4 runs as 3)."""
    kind, fuse = plan[0], plan[1]
    out, done = [], 0
    while done < m:
        k = 1 if kind == 0 else min(fuse, m - done)
        if kind in (2, 3) and k == 4:
            k = 3
        out.append(k)
        done += k
    return out


def state_bytes(shape, storage) -> int:
    """Device bytes of the state a step touches: two population buffers, two
    phi buffers and u*."""
    d = len(shape)
    q = 9 if d == 2 else 19
    es = 8 if storage == "f64" else 4
    ns = 1
    for s in shape:
        ns *= s
    return (2 * q + 2 + d) * ns * es


MALL_BYTES = 256 << 20  # MI355X Infinity Cache


def run_gpu(name, steps, warmup, plan=None, profile_mode=False, variants=True):
    """Times `steps` steps of a single-lattice workload.  Kernel durations come
    from hlb_time_kernels (one HIP event pair around many back-to-back
    launches of one kernel on the library's stream).  In profile mode (a
    fixed plan) nothing else is launched: no autotuning, no standard-stencil
    run, no variants, so a profiler's trace holds only the measured plan."""
    import torch

    from paper_0902_3921_amd import hlb

    shape, storage, kw, desc = WORKLOADS[name]
    phi0 = make_inputs(name, shape)
    d = len(shape)
    q = 9 if d == 2 else 19
    es = 8 if storage == "f64" else 4
    ns = 1
    for s in shape:
        ns *= s

    def timed(params, plan=None):
        sim = hlb.Sim(shape, storage, **params)
        sim.init(phi0)
        if plan is None:
            sim.autotune()  # picks the substep plan on this lattice (state unchanged)
        else:
            sim.set_plan(*plan)
        sim.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stats = sim.reduce(raise_on_error=False)
        return sim, t1 - t0, stats

    sim, secs, stats = timed(kw, plan)
    m = sim.m
    plan = sim.plan
    names = (sim.kernel_name(0), sim.kernel_name(1))
    # kernel durations: event pairs around `reps` repetitions each; the
    # substep launches as they run in a step (after a collide-and-stream
    # launch), the first launch scaled from its back-to-back share
    reps = 20 if profile_mode else max(20, min(200, steps // 10))
    us_lb, us_first_b2b, us_ch_b2b, us_ch_step = sim.time_kernels(reps)
    us_first = us_first_b2b * us_ch_step / us_ch_b2b
    host_io = None
    if not profile_mode:
        # host transfers of the boundary (FP64 host arrays): one hlb_init_fields
        # (upload + equilibrium kernel) and one hlb_get_fields (readout kernel +
        # download), for the PCIe-inclusive rate of a run of `steps` steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.init(phi0)
        t_init = time.perf_counter() - t0
        t0 = time.perf_counter()
        sim.fields()
        t_fields = time.perf_counter() - t0
        host_io = {"init_ms": t_init * 1e3, "get_fields_ms": t_fields * 1e3,
                   "pcie_inclusive_mlups": ns * steps / (secs + t_init + t_fields) / 1e6}
    sim.close()
    mlups_sc, var_out = None, None
    if not profile_mode:
        sim_sc, secs_sc, _ = timed(dict(kw, **STANDARD_STENCIL), plan)
        sim_sc.close()
        mlups_sc = ns * steps / secs_sc / 1e6
    if not profile_mode and variants:
        # the scheme variants of the method, each with its own autotuned plan
        var_out = {}
        var_params = {"flux_advection": dict(kw, advection=1), "mu_first_force": dict(kw, force_form=0)}
        if kw.get("cd_Q", 1.0) == 1.0:
            var_params["isotropic_ch_laplacian"] = dict(kw, cd_Q=2 / 3 if d == 2 else 1 / 3)
        if d == 2:
            try:  # the D2Q5 model, where its stability bound (that of m = 1) holds
                hlb.check_params(hlb.D2Q9, **dict(kw, cd_model=1))
                var_params["d2q5_model"] = dict(kw, cd_model=1)
            except hlb.HlbError as e:
                var_out["d2q5_model"] = {"skipped": str(e)}
        for vname, vkw in var_params.items():
            vsim, vsecs, _ = timed(vkw)
            var_out[vname] = {"mlups": ns * steps / vsecs / 1e6, "m": vsim.m, "substep_plan": list(vsim.plan)}
            if vname == "d2q5_model":
                # its two kernels: f and h collide-and-stream (18 + 10 population moves and the
                # phi tile read, s bytes each), then phi = sum h (5 reads, 1 write)
                us5, usphi, _, _ = vsim.time_kernels(max(20, min(200, steps // 10)))
                b5, bphi = (18 + 10 + 1) * es, 6 * es
                var_out[vname]["kernels"] = {
                    "lb5": {"name": vsim.kernel_name(0), "us_per_launch": us5, "bytes_per_lu": b5,
                            "gbs": b5 * ns / (us5 * 1e-6) / 1e9},
                    "phi5": {"name": vsim.kernel_name(1), "us_per_launch": usphi, "bytes_per_lu": bphi,
                             "gbs": bphi * ns / (usphi * 1e-6) / 1e9}}
            vsim.close()

    lb_b, ch_b, step_b = algorithmic_bytes(d, q, es)
    seq = launch_sequence(m, plan)
    if len(seq) == 1:
        us_first = us_ch_step  # the step's only substep launch: its in-step time, unscaled
    n_first = sum(1 for k in seq if k == seq[0])
    # the dominant kernel: the instantiation with the most device time per step
    per_step = {"lb": us_lb, "ch": us_first * n_first}
    dominant = max(per_step, key=per_step.get)
    if dominant == "lb":
        dom = {"name": names[0], "bytes_per_lu": lb_b, "us": us_lb, "launches_per_step": 1}
    else:
        # a launch reads phi and u* once and writes phi once, however many substeps it fuses
        dom = {"name": names[1], "bytes_per_lu": ch_b, "us": us_first, "launches_per_step": n_first,
               "substeps_per_launch": seq[0]}
    dom["gbs"] = dom["bytes_per_lu"] * ns / (dom["us"] * 1e-6) / 1e9
    mlups = ns * steps / secs / 1e6
    return {
        "shape": shape, "storage": storage, "desc": desc, "m": m, "ns": ns, "secs": secs,
        "mlups": mlups, "mlups_standard": mlups_sc, "variants": var_out, "stats": stats,
        "plan": plan, "launches": seq, "host_io": host_io,
        "kernels": {"lb": {"name": names[0], "us_per_launch": us_lb, "bytes_per_lu": lb_b,
                           "gbs": lb_b * ns / (us_lb * 1e-6) / 1e9},
                    "ch": {"name": names[1], "us_per_launch": us_first, "launches": seq,
                           "us_all_launches_per_step": us_ch_step, "us_all_launches_back_to_back": us_ch_b2b,
                           "bytes_per_lu": ch_b,
                           "gbs_all_launches": ch_b * ns * len(seq) / (us_ch_step * 1e-6) / 1e9},
                    "kernel_us_per_step": us_lb + us_ch_step},
        "dominant": dom, "step_min_bytes_per_lu": step_b, "q": q, "d": d, "es": es,
        "mall_resident": state_bytes(shape, storage) < MALL_BYTES,
    }


def run_gpu_batch(name, steps, warmup, plan=None):
    import torch

    from paper_0902_3921_amd import hlb

    _, storage, _, desc = WORKLOADS[name]
    specs, params, phis = batch_workload()
    shapes = [s["shape"] for s in specs]
    es = 8 if storage == "f64" else 4
    batch = hlb.Batch(shapes, params, storage)
    for i, phi in enumerate(phis):
        batch.init(i, phi)
    if plan is None:
        batch.autotune()
    else:
        batch.set_plan(*plan)
    batch.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    ms = batch.m
    ns = [s[0] * s[1] for s in shapes]
    total = sum(ns)
    sub_sites = sum(n * m for n, m in zip(ns, ms))  # substep site updates per step
    nprof = max(10, min(100, steps))
    ms_lb, ms_ch = batch.step_timed(nprof)
    stats = [batch.reduce(i, raise_on_error=False) for i in range(len(shapes))]
    tile_plan = batch.plan
    plan_index = batch.plan_index
    batch.close()
    kind, fuse = tile_plan[2], tile_plan[3]
    lb_b, ch_b, step_b = algorithmic_bytes(2, 9, es)
    # a substep launch reads phi and u* and writes phi once per site of the
    # simulations it covers, however many substeps it fuses
    launch_sites = sum(n * -(-m // fuse) for n, m in zip(ns, ms))
    nlaunch = -(-max(ms) // fuse)
    t_lb = ms_lb / nprof * 1e-3                 # s per collide-and-stream launch
    t_ch_step = ms_ch / nprof * 1e-3            # s of substep launches per step
    t_ch = t_ch_step / nlaunch                  # s per substep launch (average)
    lb_gbs = lb_b * total / t_lb / 1e9
    ch_gbs = ch_b * launch_sites / t_ch_step / 1e9
    dominant = "lb" if t_lb > t_ch_step else "ch"
    tname = "float" if storage == "f32" else "double"
    lbname = f"hlb::k_lb_batch<{tname}, {tile_plan[0]}, {tile_plan[1]}>"
    chname = {0: f"hlb::k_ch_batch<{tname}, {tile_plan[4]}, {tile_plan[5]}, true>",
              1: f"hlb::k_chf_batch<{tname}, {fuse}, {tile_plan[4]}, true>",
              2: f"hlb::k_chm_batch<{tname}, {fuse}, {tile_plan[4]}>"}[kind]
    kd = ({"name": lbname, "bytes_per_lu": lb_b, "gbs": lb_gbs, "units": total, "us": t_lb * 1e6}
          if dominant == "lb" else
          {"name": chname + f" (class average over {nlaunch} launches per step)", "bytes_per_lu": ch_b,
           "gbs": ch_gbs, "units": launch_sites / nlaunch, "us": t_ch * 1e6})
    return {
        "shape": None, "storage": storage, "desc": desc, "m": f"{min(ms)}..{max(ms)} (mean {sub_sites / total:.2f})",
        "ns": total, "secs": secs, "mlups": total * steps / secs / 1e6, "mlups_standard": None,
        "stats": {"finite": all(s["finite"] for s in stats), "mass": sum(s["mass"] for s in stats),
                  "umax": max(s["umax"] for s in stats),
                  "umax_sim": max(range(len(stats)), key=lambda i: stats[i]["umax"])},
        "plan": tile_plan, "plan_index": plan_index,
        "kernels": {"lb": {"name": lbname, "us_per_launch": t_lb * 1e6, "bytes_per_lu": lb_b, "gbs": lb_gbs},
                    "ch": {"name": chname, "us_per_launch": t_ch * 1e6, "launches_per_step": nlaunch,
                           "substeps_per_launch": fuse, "substep_site_updates_per_step": sub_sites,
                           "launch_site_updates_per_step": launch_sites, "bytes_per_lu": ch_b, "gbs": ch_gbs}},
        "dominant": kd, "step_min_bytes_per_lu": step_b, "q": 9, "d": 2, "es": es,
        "nsim": len(shapes), "sites": total, "mall_resident": False,
    }


MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16


def run_surrogate(args):
    """The surrogate workload: a 100-jump rollout (50 steps a jump) of a
    held-out 256 x 256 spinodal trajectory from t = 1000, checked against the
    GPU solver every 10 jumps with fallback above 1e-2 relative L2 phi error;
    value = solver time / rollout time.  Roofline: the convolution kernels of
    one forward against the bf16 matrix-core peak."""
    import numpy as np
    import torch

    from paper_0902_3921_amd import sur, surrogate_train as st

    params = st.load()
    net = sur.Surrogate(batch=1)
    net.set_params(params)
    r = st.rollout(net, seed=100001, jumps=100, check_every=10, tol=1e-2, log=lambda *a, **k: None)
    diag = surrogate_diagnostics(net, seed=100001, t0=st.T_FIRST)
    x = torch.from_numpy(np.zeros((1, st.SIZE, st.SIZE, 3), np.float32)).cuda()
    x[..., 0] = torch.rand((st.SIZE, st.SIZE), device="cuda") * 2 - 1
    y = torch.empty_like(x)
    net.forward_timed(x, y, reps=3)
    ms_conv, ms_total, flops = net.forward_timed(x, y, reps=50)
    achieved = flops / (ms_conv * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import unet

        xs = np.random.default_rng(0).uniform(-1, 1, (1, st.SIZE, st.SIZE, 3))
        unet.forward(params, xs)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < 15.0:
            unet.forward(params, xs)
            n += 1
        secs = time.perf_counter() - t0
        cpu = {"value": n / secs, "unit": "jumps/s", "cores": torch.get_num_threads(), "kind": "oracle",
               "sample": f"{n} FP64 oracle forwards of one 256x256 state (one jump each)"}
    # the checked rollout runs the solver over every segment to check it, so
    # its wall clock is the solver's plus the surrogate's; the speedup at the
    # tolerance exists only over segments that passed it
    checked = r["solver_s"] / r["checked_rollout_s"]
    at_tol = (r["solver_accepted_s"] / r["surrogate_accepted_s"]) if r["accepted"] else None
    out = {
        "metric": "surrogate speedup at <=1e-2 phi err (rollout vs plain GPU solver)",
        "value": at_tol, "unit": "x", "n_gpus": 1, "steps": r["jumps"], "warmup": 1,
        "ms_per_step": r["surrogate_s"] / r["jumps"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "surrogate U-Net, 256x256 D2Q9 spinodal, 100 jumps of 50 steps from t=1000, "
                               "checked every 10 jumps, fallback above 1e-2 relative L2 phi error",
                   "params": int(params.size), "seed": 100001},
        "value_note": (None if r["accepted"] else
                       "no segment met the 1e-2 tolerance, so there is no speedup at it (value null)"),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / MFMA_BF16_PEAK_TFLOPS, "traffic": None,
                     "kernel": "sur::k_conv (all convolutions of one forward)", "flops_per_launch": flops},
        "rollout": {"solver_ms": r["solver_s"] * 1e3, "surrogate_ms": r["surrogate_s"] * 1e3,
                    "checked_rollout_ms": r["checked_rollout_s"] * 1e3,
                    "checked_rollout_speed_vs_solver": checked,
                    "unchecked_surrogate_speed_vs_solver": r["solver_s"] / r["surrogate_s"],
                    "accepted_segments": r["accepted"], "fallbacks": r["fallbacks"],
                    "phi_rel_l2_at_checks": r["errors"],
                    "persistence_phi_rel_l2": r["persistence_errors"],
                    "forward_ms": ms_total, "conv_ms": ms_conv},
        "error_per_jump": diag["error_per_jump"],
        "solver_fp32_vs_fp64": diag["solver_fp32_vs_fp64"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def surrogate_diagnostics(net, seed, t0, jumps=10):
    """The surrogate's relative L2 phi error after 1..jumps jumps from the
    FP32 solver's state at t0, and the FP32 solver's distance from the FP64
    solver started from the same state after the same jumps (how
    predictable the target is)."""
    import numpy as np
    import torch

    import synth
    from paper_0902_3921_amd import hlb, surrogate_train as st

    S, J = st.SIZE, st.JUMP
    ref = hlb.Sim((S, S), "f64", **st.PHYS).init(synth.spinodal((S, S), seed, 0.01))
    ref.step(t0)
    f, ph = ref.state()
    s32 = hlb.Sim((S, S), "f32", **st.PHYS)
    s32.set_state(f, ph)
    x = torch.from_numpy(st.state_of(s32.fields())[None]).cuda().contiguous()
    sur_err, fp32_err = [], []
    for _ in range(jumps):
        ref.step(J)
        s32.step(J)
        net.forward(x, x)
        r64 = ref.fields()["phi"]
        r32 = s32.fields()["phi"]
        sur_err.append(float(np.linalg.norm(x[0, ..., 0].cpu().numpy() - r32) / np.linalg.norm(r32)))
        fp32_err.append(float(np.linalg.norm(r32 - r64) / np.linalg.norm(r64)))
    ref.close()
    s32.close()
    return {"error_per_jump": sur_err, "solver_fp32_vs_fp64": fp32_err}


def profile_figures(name, kernel_name, want_valu=False):
    """From the committed rocprofv3 summary of this workload, for the kernel
    of exactly this name (the full template instantiation): HBM bytes per
    dispatch (FETCH_SIZE and WRITE_SIZE, KiB per dispatch, scaled by the copy
    calibration) and the kernel-trace average duration in us.  None for a
    figure the summary does not hold, and for both if the summary was taken
    on different library sources.  With want_valu, also the kernel's
    SQ_INSTS_VALU per dispatch (wavefront instructions), or None."""
    from paper_0902_3921_amd import build

    path = os.path.join(ROOT, "profiles", f"{name}.md")
    none = (None, None, None) if want_valu else (None, None)
    if not os.path.exists(path):
        return none
    text = open(path).read()
    if f"library source hash: {build.source_hash()}" not in text:
        return none
    traffic, avg_us, valu = None, None, None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if not cells or cells[0] != kernel_name:
            continue
        try:
            if len(cells) == 4:  # kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB
                traffic = float(cells[2]) * 1024 * FETCH_SCALE + float(cells[3]) * 1024 * WRITE_SCALE
            elif len(cells) == 6:  # kernel | calls | avg us | min us | max us | % time
                avg_us = float(cells[2])
            elif len(cells) == 3 and cells[1] == "SQ_INSTS_VALU":  # kernel | counter | value
                valu = float(cells[2])
        except ValueError:
            continue
    if want_valu:
        return traffic, avg_us, valu
    return traffic, avg_us


def copy_rate_gbs(nbytes: int, reps: int = 20) -> float:
    """Device copy rate (GB/s of bytes read + written) of a buffer moving
    `nbytes` in total, timed with HIP events: the practical streaming rate
    for a working set of this size (the Infinity Cache holds sets up to
    about 256 MB, HBM serves larger ones)."""
    import torch

    n = max(1, nbytes // 8)  # floats per buffer: nbytes / 2 read and nbytes / 2 written
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3 / reps
    return 8.0 * n / secs / 1e9


def run_cpu_baseline(name, budget_s=15.0):
    """The FP64 oracle on a bounded number of steps of the same workload."""
    from oracle import orc

    shape, storage, kw, desc = WORKLOADS[name]
    from paper_0902_3921_amd import hlb

    if shape is None:
        # simulations of the batch in order, 5 steps each, until the budget is spent
        specs, params, phis = batch_workload()
        sites, secs, nsim = 0, 0.0, 0
        for s, p, phi in zip(specs, params, phis):
            o = orc.Oracle(s["shape"], m=hlb.check_params(0, **p), **p).init(phi)
            o.step(1)
            t0 = time.perf_counter()
            o.step(5)
            secs += time.perf_counter() - t0
            sites += 5 * phi.size
            nsim += 1
            if secs > budget_s:
                break
        return {"value": sites / secs / 1e6, "unit": "MLUPS", "cores": orc.threads(), "kind": "oracle",
                "sample": f"5 steps (after 1 untimed step) of each of the first {nsim} simulations of the "
                          f"{desc} workload, one after another (FP64 oracle)"}
    m = hlb.check_params(0 if len(shape) == 2 else 1, **kw)
    phi0 = make_inputs(name, shape)
    ns = 1
    for s in shape:
        ns *= s
    o = orc.Oracle(shape, m=m, **kw).init(phi0)
    t0 = time.perf_counter()
    o.step(1)
    first = time.perf_counter() - t0
    nsteps = max(1, min(1000, int(budget_s / max(first, 1e-6))))
    t0 = time.perf_counter()
    o.step(nsteps)
    secs = time.perf_counter() - t0
    cores = orc.threads()
    # the same oracle on one thread, over a few steps
    orc.set_threads(1)
    n1 = max(1, int(3.0 / max(first * cores, 1e-6)))
    t0 = time.perf_counter()
    o.step(n1)
    secs1 = time.perf_counter() - t0
    orc.set_threads(cores)
    return {"value": ns * nsteps / secs / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{nsteps} steps of the {desc} workload (FP64 oracle, after 1 untimed step)",
            "single_thread": {"value": ns * n1 / secs1 / 1e6, "steps": n1}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="d2q9_spinodal_1024", choices=sorted(WORKLOADS) + ["surrogate_256"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plan", default=None,
                    help="plan to use instead of autotuning (e.g. for profiler runs): kind,fuse,bw,seg for one "
                         "simulation, lb,substep candidate indices for a batch")
    ap.add_argument("--no-3d", action="store_true",
                    help="leave out the 256^3 D3Q19 sub-record of the default run")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run a device copy of this many MiB (for the HBM counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU domain decomposition is design only)", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))

    if args.workload == "surrogate_256":
        run_surrogate(args)
        return
    plan = tuple(int(v) for v in args.plan.split(",")) if args.plan else None
    profile_mode = plan is not None
    batched = WORKLOADS[args.workload][0] is None
    if batched:
        r = run_gpu_batch(args.workload, args.steps, args.warmup, plan)
    else:
        r = run_gpu(args.workload, args.steps, args.warmup, plan, profile_mode=profile_mode)
    # the metric's other configuration, the 256^3 D3Q19 spinodal, as a
    # sub-record of the default run (its own autotuned plan, 200 steps)
    sub3d = None
    if args.workload == "d2q9_spinodal_1024" and not profile_mode and not args.no_3d:
        r3 = run_gpu("d3q19_spinodal_256", min(args.steps, 200), min(args.warmup, 10), variants=False)
        sub3d = summarize(r3, "d3q19_spinodal_256", min(args.steps, 200))
        sub3d.pop("host_io", None)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    cpu = None
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        cpu = run_cpu_baseline(args.workload)

    rec = summarize(r, args.workload, args.steps)
    out = {
        "metric": "MLUPS & % HBM peak (D2Q9/D3Q19 hybrid step)",
        "value": r["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if r["storage"] == "f32" else "f64",
        "data": "synthetic",
        "config": ({"workload": r["desc"], "lattice": "D2Q9", "nsim": r["nsim"], "sites": r["sites"],
                    "m": r["m"], "tile_plan": list(r["plan"]), "substep_plan": list(r["plan_index"]),
                    "stencil": "N=0.3, Q=2.5",
                    "params": "a=-0.1 b=0.1 Gamma=1, kappa and tau per simulation", "seed": 0}
                   if batched else rec["config"]),
        "roofline": rec["roofline"],
        "step_algorithmic_frac": rec["step_algorithmic_frac"],
        "mall_resident": r["mall_resident"],
        "mlups_standard_stencil": r["mlups_standard"],
        "variants": r.get("variants"),
        "host_io": r.get("host_io"),
        "kernels": r["kernels"],
        "check": {k: r["stats"][k] for k in ("finite", "mass", "umax", "umax_sim") if k in r["stats"]},
        "d3q19_spinodal_256": sub3d,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def summarize(r, workload, steps):
    """The roofline record of one run: the dominant kernel's algorithmic
    bytes per launch over its average launch duration (hlb_time_kernels),
    against the 8 TB/s HBM peak; the committed profile's measured HBM bytes
    per launch of that same kernel (exact instantiation) and its kernel-trace
    average duration, for comparison; and the step's algorithmic fraction."""
    kd = r["dominant"]
    alg_launch = kd["bytes_per_lu"] * kd.get("units", r["ns"])
    traffic, prof_us, valu = profile_figures(workload, kd["name"].split(" (")[0], want_valu=True)
    traffic_gbs = traffic / (kd["us"] * 1e-6) / 1e9 if traffic is not None else None
    # share of the chip's vector issue slots the kernel fills: a wavefront
    # FP32/FP64 VALU instruction holds one of the 4 x 256 SIMDs for 4 cycles
    valu_frac = valu * 4 / (kd["us"] * 1e-6 * CLOCK_HZ * 4 * N_CU) if valu is not None else None
    copy_gbs = copy_rate_gbs(int(alg_launch))
    rec = {
        "ms_per_step": r["secs"] / steps * 1e3,
        "mlups": r["mlups"],
        "config": None if r["shape"] is None else
        {"workload": r["desc"], "lattice": "D2Q9" if r["d"] == 2 else "D3Q19",
         "shape": list(r["shape"]), "m": r["m"], "substep_plan": list(r["plan"]),
         "launches_per_step": r.get("launches"),
         "stencil": "N=0.3, Q=2.5" if r["d"] == 2 else "N=1/6, Q=1/3",
         "params": " ".join(f"{k}={v:g}" for k, v in WORKLOADS[workload][2].items() if k in ("a", "b", "kappa",
                                                                                              "tau", "gamma")),
         "seed": 0},
        "roofline": {"bound": "hbm", "achieved": kd["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": kd["gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_gbs": traffic_gbs,
                     "traffic_frac": traffic_gbs / HBM_PEAK_GBS if traffic_gbs is not None else None,
                     "traffic_over_algorithmic": traffic / alg_launch if traffic is not None else None,
                     "kernel": kd["name"], "bytes_per_lu": kd["bytes_per_lu"],
                     "algorithmic_bytes_per_launch": alg_launch, "us_per_launch": kd["us"],
                     "launches_per_step": kd.get("launches_per_step"),
                     "profile_avg_us": prof_us, "valu_issue_frac": valu_frac,
                     "copy_gbs_same_bytes": copy_gbs, "frac_of_copy": kd["gbs"] / copy_gbs},
        "step_algorithmic_frac": r["mlups"] * 1e6 * r["step_min_bytes_per_lu"] / (HBM_PEAK_GBS * 1e9),
        "mall_resident": r["mall_resident"],
        "kernels": r["kernels"],
        "check": {k: r["stats"][k] for k in ("finite", "mass", "umax") if k in r["stats"]},
    }
    return rec


if __name__ == "__main__":
    main()
