"""Learned coarse solver for the Euler equations (the data-driven Euler
discretisation section 6.2 names as future work, built like the planar
shallow-water one): training data from fine classic Euler runs, coarsened by
exact block averages; curriculum training of the 4 -> 96 coefficient network
with the unrolled loss of eq 2.28; evaluation of the density against the
fine reference, next to the plain MINMOD scheme at several resolutions.

Every numerical step runs in libfv's HIP kernels (classic Euler solver,
network, learned Euler stage, adjoint, Adam, coarsening); this module only
orchestrates.

    python -m paper_2602_08670_amd.learned_euler_solver --out results.json
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import fv, inputs
from .learned_solver import graph_replay, rel_l2

GAMMA = 1.4


def fine_dt(n_fine: int, c_max: float = 4.3, safety: float = 1.25) -> float:
    """Fixed fine step: CFL 0.4 in the two-axis sum form with a margin over
    the largest |u| + c of the smooth Euler data (|u| <= 0.71, c <= 3.55)."""
    return 0.4 / (safety * 2.0 * c_max * n_fine)


def trajectory(seed: int, n_fine: int, factor: int, n_coarse_steps: int):
    """Coarse snapshots [n_coarse_steps + 1, 4, n, n] (torch CUDA float32) of
    a fine periodic classic Euler run (HLLE, MINMOD, Heun, fixed step),
    block-averaged by `factor` every `factor` fine steps."""
    import torch

    q0 = inputs.random_smooth_euler(n_fine, seed=seed)
    s = fv.Solver(q0, prec=fv.FV_F32, dt_fixed=fine_dt(n_fine))
    out = [fv.coarsen(s.q, factor)]
    for _ in range(n_coarse_steps):
        s.run(factor)
        out.append(fv.coarsen(s.q, factor))
    traj = torch.stack(out)
    torch.cuda.synchronize()
    s.close()
    return traj


def init_params(seed: int) -> np.ndarray:
    """He-scaled random weights, zero biases, zero last layer (the network
    starts at the base coefficients)."""
    rng = np.random.default_rng(seed)
    layers = [(4, 32), (32, 32), (32, 32), (32, 32), (32, 96)]
    ws, bs = [], []
    for i, (ci, co) in enumerate(layers):
        w = rng.standard_normal((co, ci, 3, 3)) * math.sqrt(2.0 / (9 * ci))
        ws.append(w * 0.0 if i == len(layers) - 1 else w)
        bs.append(np.zeros(co))
    return fv.params_to_vector(ws, bs)


def normalisation(data):
    d = data.double()
    mean = [float(d[:, :, v].mean()) if v in (0, 3) else 0.0 for v in range(4)]
    std = [max(float(d[:, :, v].std()), 1e-3) for v in range(4)]
    return mean, [1.0 / s for s in std], std


def rollout_score(net, q0s, refs, steps):
    """(blow-ups, median rel L2 of rho) of learned rollouts of the states
    q0s (one batch, the net's B) against refs."""
    import torch

    q = torch.stack([torch.as_tensor(x) for x in q0s]).to("cuda").contiguous()
    net.update()
    net.step(q, steps)
    out = q.cpu().double().numpy()
    errs = np.array([rel_l2(out[b, 0], refs[b][0]) if np.all(np.isfinite(out[b])) else np.inf
                     for b in range(len(q0s))])
    return int(np.sum(~(errs <= 1.0))), float(np.median(errs))


def main():
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--n-fine", type=int, default=512)
    ap.add_argument("--factor", type=int, default=8)
    ap.add_argument("--train-seeds", type=int, default=48)
    ap.add_argument("--steps", type=int, default=200, help="coarse steps of trajectories and evaluation")
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--T", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=2e-5)
    ap.add_argument("--val-seeds", type=int, default=8)
    ap.add_argument("--val-every", type=int, default=100)
    ap.add_argument("--eval-seeds", type=int, default=16)
    ap.add_argument("--plain-sizes", default="64,128,256")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    n = a.n_fine // a.factor
    dt_c = fine_dt(a.n_fine) * a.factor
    t0 = time.perf_counter()
    data = torch.stack([trajectory(s, a.n_fine, a.factor, a.steps) for s in range(2000, 2000 + a.train_seeds)])
    print(f"[data] {tuple(data.shape)} in {time.perf_counter() - t0:.1f} s", flush=True)
    vq, vr = [], []
    for s in range(4000, 4000 + a.val_seeds):
        tr = trajectory(s, a.n_fine, a.factor, a.steps)
        vq.append(tr[0].cpu().numpy())
        vr.append(tr[-1].double().cpu().numpy())
    mean, inv_std, std = normalisation(data)
    params = torch.tensor(init_params(0), device="cuda")
    net = fv.EulerLearned(params.cpu().numpy(), a.batch, n, n, dt_c, mean=mean, inv_std=inv_std)
    vnet = fv.EulerLearned(params.cpu().numpy(), a.val_seeds, n, n, dt_c, mean=mean, inv_std=inv_std)
    trn = fv.EulerTrainer(net, fv.make_euler_train_config(a.batch, n, n, a.T, dt_c, scale=tuple(std), lr=a.lr))

    def score():
        vnet.params.copy_(net.params)
        return rollout_score(vnet, vq, vr, a.steps)

    rng = np.random.default_rng(1)
    n_traj, S1 = data.shape[0], data.shape[1]
    best = (score(), 0, net.params.clone())
    hist = []
    t1 = time.perf_counter()
    for it in range(a.iters):
        T = min(a.T, 1 + (it * a.T) // max(1, a.iters // 2))
        ti = torch.as_tensor(rng.integers(0, n_traj, a.batch), device="cuda")
        ki = torch.as_tensor(rng.integers(0, S1 - T, a.batch), device="cuda")
        q0 = data[ti, ki]
        tg = data[ti[None, :], ki[None, :] + torch.arange(1, T + 1, device="cuda")[:, None]]
        loss, stats = trn.step(q0, tg)
        trn.set_lr(a.lr_final + 0.5 * (a.lr - a.lr_final) * (1.0 + math.cos(math.pi * it / max(1, a.iters - 1))))
        trn.adam()
        hist.append(loss)
        if it % 100 == 0:
            print(f"[train] it {it} T {T} loss {loss:.4e} fallback {stats[0]} redone {stats[1]}", flush=True)
        if (it + 1) % a.val_every == 0 or it + 1 == a.iters:
            sc = score()
            if sc < best[0]:
                best = (sc, it + 1, net.params.clone())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    trn.close()
    print(f"[train] {a.iters} iterations in {wall:.1f} s; selected iteration {best[1]} (val {best[0]})", flush=True)

    # evaluation on held-out seeds, one batch
    seeds = list(range(5000, 5000 + a.eval_seeds))
    refs, q0c, q0f = [], [], []
    for s in seeds:
        tr = trajectory(s, a.n_fine, a.factor, a.steps)
        refs.append(tr[-1].double().cpu().numpy())
        q0c.append(tr[0].cpu().numpy())
        q0f.append(inputs.random_smooth_euler(a.n_fine, seed=s))
    res = {"n_fine": a.n_fine, "n_coarse": n, "factor": a.factor, "steps": a.steps, "dt": dt_c,
           "train": {"iters": a.iters, "batch": a.batch, "T": a.T, "wall_s": wall, "selected_iteration": best[1],
                     "val_score": best[0], "loss_first": hist[0], "loss_last": hist[-1]}, "cases": {}}
    for name, pv in (("untrained", torch.tensor(init_params(0), device="cuda")), ("learned", best[2])):
        en = fv.EulerLearned(pv.cpu().numpy(), len(seeds), n, n, dt_c, mean=mean, inv_std=inv_std)
        q = torch.tensor(np.stack(q0c), device="cuda").contiguous()
        en.step(q, a.steps)
        fb, rd, fr, rc = en.stats()
        out = q.cpu().double().numpy()
        errs = [rel_l2(out[b, 0], refs[b][0]) if np.all(np.isfinite(out[b])) else float("inf") for b in range(len(seeds))]
        en.close()
        # time to solution of one solve, graph-replayed
        e1 = fv.EulerLearned(pv.cpu().numpy(), 1, n, n, dt_c, mean=mean, inv_std=inv_std, stream=torch.cuda.Stream())
        q1 = torch.tensor(q0c[0][None], device="cuda").contiguous()
        tts = graph_replay(lambda k: e1.step(q1, k), a.steps, 50 if a.steps % 50 == 0 else a.steps, e1.stream)
        e1.close()
        ea = np.asarray(errs)
        res["cases"][name] = {"rel_l2_rho": float(np.mean(ea)), "median": float(np.median(ea)),
                              "blowups": int(np.sum(~(ea <= 1.0))), "per_seed": errs, "time_to_solution_s": tts,
                              "fallback_faces": int(fb.sum()), "redone_steps": int(rd.sum())}
        print(f"[eval] {name}: rel L2(rho) mean {np.mean(ea):.3e} median {np.median(ea):.3e} max {np.max(ea):.3e}, "
              f"{tts * 1e3:.1f} ms, fallbacks {int(fb.sum())}, redone {int(rd.sum())}", flush=True)
    for m in (int(v) for v in a.plain_sizes.split(",") if v):
        sub = m // n
        errs, times = [], []
        for b, s in enumerate(seeds):
            q0m = fv.coarsen(torch.tensor(q0f[b], dtype=torch.float32, device="cuda"), a.n_fine // m).cpu().numpy()
            stp = torch.cuda.Stream()
            sp = fv.Solver(q0m, prec=fv.FV_F32, dt_fixed=dt_c / sub, stream=stp)
            if b == 0:
                times.append(graph_replay(lambda k: fv.fv_run(sp.h, k * sub), a.steps,
                                          50 if a.steps % 50 == 0 else a.steps, stp))
            else:
                sp.run(a.steps * sub)
            outm = sp.state()
            sp.close()
            if sub > 1:
                outm = outm.reshape(4, n, sub, n, sub).mean(axis=(2, 4))
            errs.append(rel_l2(outm[0], refs[b][0]))
        res["cases"][f"plain{m}"] = {"rel_l2_rho": float(np.mean(errs)), "median": float(np.median(errs)),
                                     "per_seed": errs, "time_to_solution_s": times[0]}
        print(f"[eval] plain{m}: rel L2(rho) mean {np.mean(errs):.3e} median {np.median(errs):.3e} "
              f"max {np.max(errs):.3e}, {times[0] * 1e3:.1f} ms", flush=True)
    net.close()
    vnet.close()
    print(json.dumps(res), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
