"""Training data, training and checked rollouts of the surrogate network.

The surrogate (include/sur.h) maps the state (phi, rho u_x, rho u_y) of a
256 x 256 periodic D2Q9 spinodal decomposition to the state 50 timesteps
later.  Its data come from the library's own batched solver (hlb.Batch):
trajectories from phi ~ U(-0.01, 0.01) (seed = trajectory index), n = 1,
u = 0, at a = -0.1, b = 0.1, kappa = 0.1, tau = 1, Gamma = 1 and the paper's
stencil N = 0.3, Q = 2.5, sampled every 50 steps over t in [1000, 6000].

    python -m paper_0902_3921_amd.surrogate_train --out weights.npz

writes the trained FP32 parameters with the recipe that produced them.
A rollout advances a state by jumps of the surrogate and compares phi with
the solver every `check_every` jumps; where the relative L2 error exceeds
the tolerance, the solver's state replaces the surrogate's (a fallback).
The solver runs every segment to check it, so a checked rollout costs the
solver's time plus the surrogate's; its times are reported separately.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

PHYS = dict(a=-0.1, b=0.1, kappa=0.1, tau=1.0, gamma=1.0, N=0.3, Q=2.5)
JUMP = 50           # lattice Boltzmann steps per surrogate jump
SIZE = 256
T_FIRST, T_LAST = 1000, 6000
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "surrogate_weights.npz")


def state_of(fields) -> np.ndarray:
    """(phi, n u_x, n u_y) as an [H, W, 3] float32 array from hlb fields."""
    n, u, phi = fields["n"], fields["u"], fields["phi"]
    return np.stack([phi, n * u[0], n * u[1]], axis=-1).astype(np.float32)


def generate(n_traj: int, pairs_per_traj: int = 8, group: int = 250, seed0: int = 0, log=print):
    """Snapshots [n_traj, pairs_per_traj + 1, H, W, 3] (a float32 device
    tensor) of trajectories seed0 .. seed0 + n_traj - 1, JUMP steps apart.
    Trajectory i starts recording at a time spread over [T_FIRST, T_LAST -
    JUMP * pairs_per_traj] by its group."""
    import torch

    import synth
    from . import hlb

    snaps = torch.empty((n_traj, pairs_per_traj + 1, SIZE, SIZE, 3), dtype=torch.float32, device="cuda")
    ngroups = -(-n_traj // group)
    span = T_LAST - JUMP * pairs_per_traj - T_FIRST
    for g in range(ngroups):
        ids = list(range(g * group, min(n_traj, (g + 1) * group)))
        t_start = T_FIRST + (span * g) // max(1, ngroups - 1)
        t0 = time.perf_counter()
        batch = hlb.Batch([(SIZE, SIZE)] * len(ids), PHYS, "f32")
        for k, i in enumerate(ids):
            batch.init(k, synth.spinodal((SIZE, SIZE), seed0 + i, 0.01))
        batch.autotune()
        batch.step(t_start)
        for j in range(pairs_per_traj + 1):
            if j:
                batch.step(JUMP)
            for k, i in enumerate(ids):
                snaps[i, j] = torch.from_numpy(state_of(batch.fields(k)))
        batch.close()
        log(f"data group {g + 1}/{ngroups}: {len(ids)} trajectories from t = {t_start}, "
            f"{time.perf_counter() - t0:.1f} s", flush=True)
    return snaps


def train(net, snaps, iters: int, batch: int, lr: float, seed: int = 0, log=print, log_every: int = 200,
          pushforward: float = 0.0, noise: float = 0.0):
    """Adam on random (state, state + JUMP) pairs, cosine learning-rate decay
    from lr to lr / 100.  With probability `pushforward` (after the first
    third of the iterations) an iteration instead takes the network's own
    prediction of a state one jump ahead as input and the state two jumps
    ahead as target, without a gradient through the first jump (the
    "pushforward" training of Brandstetter, Worrall and Welling), so that the
    network learns to correct the errors it makes.  With `noise` > 0 every
    input also receives Gaussian noise of that fraction of each channel's
    standard deviation over the data, and the target stays clean (noise
    injection, Sanchez-Gonzalez et al.), for the same purpose.  Returns the
    list of (iteration, loss)."""
    import torch

    n_traj, n_snap = snaps.shape[0], snaps.shape[1]
    gen = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    t0 = time.perf_counter()
    x = torch.empty((batch, SIZE, SIZE, 3), dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    sigma = None
    if noise > 0:
        std = torch.stack([snaps[..., c].std() for c in range(3)])
        sigma = (noise * std).view(1, 1, 1, 3)
        ngen = torch.Generator(device="cuda").manual_seed(seed + 1)
    for it in range(iters):
        push = it >= iters // 3 and float(torch.rand((), generator=gen)) < pushforward
        ti = torch.randint(0, n_traj, (batch,), generator=gen)
        si = torch.randint(0, n_snap - (2 if push else 1), (batch,), generator=gen)
        x.copy_(snaps[ti.cuda(), si.cuda()])
        if sigma is not None:
            x.add_(torch.randn(x.shape, generator=ngen, device="cuda") * sigma)
        if push:
            net.forward(x, x)
            y.copy_(snaps[ti.cuda(), (si + 2).cuda()])
        else:
            y.copy_(snaps[ti.cuda(), (si + 1).cuda()])
        rate = lr * (0.01 + 0.99 * 0.5 * (1 + np.cos(np.pi * it / iters)))
        if it % log_every == 0 or it == iters - 1:
            loss = net.loss_grad(x, y)
            hist.append((it, loss))
            log(f"iter {it} loss {loss:.4e} lr {rate:.2e} {time.perf_counter() - t0:.0f} s", flush=True)
        else:
            net.loss_grad_async(x, y)
        net.adam_step(rate)
    return hist


def save(path, params, meta):
    np.savez(path, params=np.asarray(params, np.float32), **{k: np.asarray(v) for k, v in meta.items()})


def load(path=WEIGHTS):
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: train with `python -m paper_0902_3921_amd.surrogate_train`")
    with np.load(path, allow_pickle=False) as d:
        return d["params"].astype(np.float32)


def rollout(net, seed: int, jumps: int = 100, check_every: int = 10, tol: float = 1e-2, t0: int = T_FIRST,
            log=print):
    """Surrogate rollout from the solver's state at t0 of trajectory `seed`,
    checked against the solver every check_every jumps; where phi's relative
    L2 error exceeds `tol` the solver's state replaces the surrogate's (a
    fallback).  The solver runs every segment to check it.  Returns a dict
    with the times of the solver's segments (all, and those whose surrogate
    segment passed), of the surrogate's forwards (all, and those that
    passed), the wall clock of the checked rollout (surrogate plus checking solver),
    the errors at every check and the number of fallbacks."""
    import torch

    import synth
    from . import hlb

    sim = hlb.Sim((SIZE, SIZE), "f32", **PHYS)
    sim.init(synth.spinodal((SIZE, SIZE), seed, 0.01))
    sim.autotune()
    sim.step(t0)
    x = torch.from_numpy(state_of(sim.fields())[None]).cuda().contiguous()
    seg_steps = JUMP * check_every
    solver_s, sur_s, errors, fallbacks = 0.0, 0.0, [], 0
    solver_ok_s, sur_ok_s = 0.0, 0.0
    persistence = []  # error of the segment's starting state (no change at all)
    y = torch.empty_like(x)
    net.forward(x, y)  # warm-up
    torch.cuda.synchronize()
    for seg in range(jumps // check_every):
        torch.cuda.synchronize()
        a = time.perf_counter()
        sim.step(seg_steps)
        torch.cuda.synchronize()
        seg_solver = time.perf_counter() - a
        solver_s += seg_solver
        ref = state_of(sim.fields())
        start = x[0].cpu().numpy()
        persistence.append(float(np.linalg.norm(start[..., 0] - ref[..., 0]) / np.linalg.norm(ref[..., 0])))
        a = time.perf_counter()
        for _ in range(check_every):
            net.forward(x, x)
        torch.cuda.synchronize()
        seg_sur = time.perf_counter() - a
        sur_s += seg_sur
        got = x[0].cpu().numpy()
        err = float(np.linalg.norm(got[..., 0] - ref[..., 0]) / np.linalg.norm(ref[..., 0]))
        errors.append(err)
        if err > tol:
            fallbacks += 1
            x.copy_(torch.from_numpy(ref[None]))
        else:
            solver_ok_s += seg_solver
            sur_ok_s += seg_sur
        log(f"segment {seg + 1}: t = {t0 + (seg + 1) * seg_steps}, phi rel L2 error {err:.3e}"
            f"{' -> solver state' if err > tol else ''}", flush=True)
    sim.close()
    nseg = jumps // check_every
    return {"solver_s": solver_s, "surrogate_s": sur_s, "checked_rollout_s": solver_s + sur_s,
            "accepted": nseg - fallbacks, "solver_accepted_s": solver_ok_s, "surrogate_accepted_s": sur_ok_s,
            "errors": errors, "persistence_errors": persistence, "fallbacks": fallbacks,
            "jumps": jumps, "check_every": check_every, "tol": tol, "t0": t0}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--trajectories", type=int, default=2000)
    ap.add_argument("--pairs", type=int, default=8)
    ap.add_argument("--iters", type=int, default=24000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--rollout-seed", type=int, default=100000)
    ap.add_argument("--pushforward", type=float, default=0.5)
    ap.add_argument("--noise", type=float, default=0.0)
    args = ap.parse_args(argv)

    import torch

    from . import sur

    if not torch.cuda.is_available():
        print("surrogate training needs a GPU", file=sys.stderr)
        return 1
    t0 = time.perf_counter()
    snaps = generate(args.trajectories, args.pairs)
    print(f"data: {tuple(snaps.shape)} in {time.perf_counter() - t0:.0f} s", flush=True)
    net = sur.Surrogate(batch=args.batch)
    net.set_params(sur.he_init(args.seed))
    hist = train(net, snaps, args.iters, args.batch, args.lr, args.seed, pushforward=args.pushforward,
                 noise=args.noise)
    params = net.params()
    del snaps
    test = sur.Surrogate(batch=1)
    test.set_params(params)
    r = rollout(test, args.rollout_seed)
    free = rollout(test, args.rollout_seed, tol=float("inf"))
    meta = dict(trajectories=args.trajectories, pairs=args.pairs, iters=args.iters, batch=args.batch, lr=args.lr,
                pushforward=args.pushforward, noise=args.noise,
                seed=args.seed, final_loss=hist[-1][1], rollout_errors=np.array(r["errors"]),
                free_rollout_errors=np.array(free["errors"]), loss_history=np.array(hist),
                recipe="spinodal 256x256 D2Q9 FP32, a=-0.1 b=0.1 kappa=0.1 tau=1 Gamma=1 N=0.3 Q=2.5, "
                       f"snapshots every {JUMP} steps over t in [{T_FIRST}, {T_LAST}]")
    save(args.out, params, meta)
    print(f"saved {args.out}; checked rollout errors {np.round(r['errors'], 4).tolist()}, fallbacks "
          f"{r['fallbacks']}; unchecked rollout errors {np.round(free['errors'], 4).tolist()}; "
          f"total {time.perf_counter() - t0:.0f} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
