"""Learned coarse solver workflow (thesis section 5.4 approach on the planar
shallow-water equations): training data from fine classic runs, coarsened by
exact block averages; curriculum training of the coefficient network with
the unrolled loss of eq 2.28; evaluation against the fine reference.

Every numerical step runs in libfv's HIP kernels (classic solver, network,
learned step, adjoint, Adam, coarsening); this module only orchestrates.

Run the full experiment:  python -m paper_2602_08670_amd.learned_solver --out results.json
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import fv, inputs

G = 9.81


def fine_dt(n_fine: int, c_max: float = math.sqrt(G * 1.6), safety: float = 1.25) -> float:
    """Fixed fine step: CFL 0.4 in the two-axis sum form with a margin over
    the largest gravity-wave speed of the data (depth <= 1.6)."""
    return 0.4 / (safety * 2.0 * c_max * n_fine)


def trajectory(seed: int, n_fine: int, factor: int, n_coarse_steps: int, device="cuda"):
    """Coarse snapshots [n_coarse_steps + 1, 3, n, n] (torch CUDA float32) of
    a fine periodic classic run (HLLE, MINMOD, Heun, fixed step), every
    `factor` fine steps, block-averaged by `factor`."""
    import torch

    dtf = fine_dt(n_fine)
    q0 = inputs.random_smooth_swe(n_fine, seed=seed)
    s = fv.Solver(q0, prec=fv.FV_F32, dt_fixed=dtf, device=device)
    out = [fv.coarsen(s.q, factor)]
    for _ in range(n_coarse_steps):
        s.run(factor)
        out.append(fv.coarsen(s.q, factor))
    traj = torch.stack(out)
    torch.cuda.synchronize()
    s.close()
    return traj


def dataset(seeds, n_fine, factor, n_coarse_steps, device="cuda"):
    import torch

    return torch.stack([trajectory(s, n_fine, factor, n_coarse_steps, device) for s in seeds])


def normalisation(data):
    """Input normalisation and loss scales from the training data."""
    d = data.double()
    mean = [1.0, 0.0, 0.0]
    std = [float(d[:, :, 0].std()), float(d[:, :, 1].std()), float(d[:, :, 2].std())]
    std = [max(s, 1e-3) for s in std]
    return mean, [1.0 / s for s in std], std


def init_params(seed: int) -> np.ndarray:
    """He-scaled random weights, zero biases, zero last layer (the network
    starts at the base coefficients)."""
    rng = np.random.default_rng(seed)
    layers = [(3, 32), (32, 32), (32, 32), (32, 32), (32, 72)]
    ws, bs = [], []
    for i, (ci, co) in enumerate(layers):
        w = rng.standard_normal((co, ci, 3, 3)) * math.sqrt(2.0 / (9 * ci))
        if i == len(layers) - 1:
            w = w * 0.0
        ws.append(w)
        bs.append(np.zeros(co))
    return fv.params_to_vector(ws, bs)


def validation_set(seeds, n_fine, factor, n_coarse_steps):
    """Held-out rollouts for checkpoint selection: the coarse initial states
    and the coarsened fine states n_coarse_steps coarse steps later."""
    q0, ref = [], []
    for sd in seeds:
        tr = trajectory(sd, n_fine, factor, n_coarse_steps)
        q0.append(tr[0].cpu().numpy())
        ref.append(tr[-1].double().cpu().numpy())
    return {"q0": q0, "ref": ref, "steps": n_coarse_steps}


def rollout_error(model, val, dt_c, direct: bool = False, blend: bool = False):
    """Score of the learned rollouts of a validation set (the model's packed
    weights re-packed from its master parameters): (number of rollouts that
    blew up -- non-finite, or a relative L2 depth error above 1 --, median
    relative L2 depth error).  Lower is better, compared as a tuple: a
    single hard validation state does not decide between two stable
    iterates, a blow-up always does."""
    model.update()
    errs = []
    for q0, ref in zip(val["q0"], val["ref"]):
        s = fv.Solver(q0, prec=fv.FV_F32, dt_fixed=dt_c, learned=1, h_ref=1.0)
        (s.direct_step if direct else s.blend_step if blend else s.learned_step)(model, val["steps"], want_stats=False)
        out = s.state()
        s.close()
        errs.append(rel_l2(out[0], ref[0]) if np.all(np.isfinite(out)) else float("inf"))
    errs = np.asarray(errs)
    return int(np.sum(~(errs <= 1.0))), float(np.median(errs))


def train(data, iters: int, B: int = 16, T_max: int = 8, lr: float = 1e-3, seed: int = 0, log_every: int = 0,
          model=None, dt_c: float | None = None, n_fine: int | None = None, factor: int | None = None,
          lr_final: float | None = None, direct: bool = False, val=None, val_every: int = 25, blend: bool = False):
    """Curriculum training on windows of the coarse trajectories data
    [n_traj, S+1, 3, n, n].  T grows 1 -> T_max over the first half; with
    lr_final the learning rate follows a cosine from lr to lr_final.  blend:
    the scheme with the flux-limiter blend of its face fluxes is trained.

    val (validation_set): every val_every iterations, and for the initial
    parameters, the learned rollout of the validation states is scored
    (rollout_error); training returns the parameters with the best score.
    The unrolled loss only sees windows of T_max steps, so parameters that
    fit those windows can still drift over a long rollout; selecting on the
    long rollout keeps such iterates out."""
    import torch

    n_traj, S1, _, n, _ = data.shape
    if dt_c is None:
        dt_c = fine_dt(n_fine) * factor
    mean, inv_std, std = normalisation(data)
    if model is None:
        model = fv.Model(init_params(seed), fv.make_model_desc(mean=mean, inv_std=inv_std))
    cfg = fv.make_train_config(B, n, n, T_max, dt_c, h_ref=1.0, scale=tuple(std), lr=lr, direct=direct, blend=blend)
    tr = fv.Trainer(model, cfg)
    rng = np.random.default_rng(seed + 1)
    hist = []
    best = None
    if val is not None:
        best = (rollout_error(model, val, dt_c, direct, blend), 0, model.params.clone())
    t0 = time.perf_counter()
    for it in range(iters):
        T = min(T_max, 1 + (it * T_max) // max(1, iters // 2))
        ti = torch.as_tensor(rng.integers(0, n_traj, B), device=data.device)
        ki = torch.as_tensor(rng.integers(0, S1 - T, B), device=data.device)
        q0 = data[ti, ki]
        tg = data[ti[None, :], ki[None, :] + torch.arange(1, T + 1, device=data.device)[:, None]]  # [T, B, 3, n, n]
        loss, stats = tr.step(q0, tg)
        if lr_final is not None:
            tr.set_lr(lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * it / max(1, iters - 1))))
        tr.adam()
        hist.append((it, T, loss))
        if log_every and it % log_every == 0:
            print(f"[train] it {it} T {T} loss {loss:.4e} fallback {stats[0]} redone {stats[1]}", flush=True)
        if val is not None and ((it + 1) % val_every == 0 or it + 1 == iters):
            e = rollout_error(model, val, dt_c, direct, blend)
            if e < best[0]:
                best = (e, it + 1, model.params.clone())
    if best is not None:
        model.params.copy_(best[2])
        model.update()
        model.selected = {"iteration": best[1], "val_blowups": best[0][0], "val_median_rel_l2_h": best[0][1]}
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tr.close()
    return model, hist, wall


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def mean_rel_h(h, href):
    """Mean relative depth error |h_ref - h| / h_ref over the cells (the
    thesis's error metric of section 3, taken in absolute value)."""
    return float(np.mean(np.abs(href - h) / href))


def graph_replay(launch, total: int, chunk: int, stream):
    """Capture launch(chunk) (work enqueued on `stream`) in one graph and
    replay it total/chunk times; returns the wall time of the replays."""
    import torch

    assert total % chunk == 0
    with torch.cuda.stream(stream):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            launch(chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(total // chunk):
        g.replay()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def evaluate(model, seeds, n_fine, factor, n_coarse_steps, plain_sizes=(64, 128, 256, 512), chunk=50,
             direct: bool = False, blend: bool = False, refs: dict | None = None, verbose: bool = False):
    """Errors at the final time of the learned coarse solver and of the plain
    scheme at plain_sizes against the fine reference (block-averaged), and
    graph-replayed time-to-solution of each.  refs: a dict that caches the
    fine references per seed across calls."""
    import torch

    n = n_fine // factor
    dt_c = fine_dt(n_fine) * factor
    res = {"seeds": list(seeds), "n_coarse": n, "n_fine": n_fine, "steps": n_coarse_steps, "dt": dt_c,
           "t_end": dt_c * n_coarse_steps, "cases": {}}
    keys = ["learned"] + [f"plain{m}" for m in plain_sizes]
    errs, hs, times, fb = ({k: [] for k in keys} for _ in range(4))
    refs = {} if refs is None else refs
    for seed in seeds:
        if seed not in refs:
            refs[seed] = trajectory(seed, n_fine, factor, n_coarse_steps)[-1].double().cpu().numpy()
        ref = refs[seed]
        q0f = torch.tensor(inputs.random_smooth_swe(n_fine, seed=seed), dtype=torch.float32, device="cuda")
        q0c = fv.coarsen(q0f, factor).cpu().numpy()
        st = torch.cuda.Stream()
        sl = fv.Solver(q0c, prec=fv.FV_F32, dt_fixed=dt_c, learned=1, h_ref=1.0, stream=st)
        lstep = fv.fv_direct_step if direct else fv.fv_blend_step if blend else fv.fv_learned_step
        times["learned"].append(graph_replay(lambda k: lstep(sl.h, model.h, k, want_stats=False),
                                             n_coarse_steps, chunk, st))
        out = sl.state()
        fb["learned"].append(lstep(sl.h, model.h, 0, want_stats=True))
        errs["learned"].append(rel_l2(out[0], ref[0]))
        hs["learned"].append(mean_rel_h(out[0], ref[0]))
        sl.close()
        for m in plain_sizes:
            sub = m // n
            q0m = fv.coarsen(q0f, n_fine // m).cpu().numpy()
            stp = torch.cuda.Stream()
            sp = fv.Solver(q0m, prec=fv.FV_F32, dt_fixed=dt_c / sub, stream=stp)
            times[f"plain{m}"].append(graph_replay(lambda k: fv.fv_run(sp.h, k * sub), n_coarse_steps, chunk, stp))
            outm = sp.state()
            if sub > 1:
                outm = outm.reshape(3, n, sub, n, sub).mean(axis=(2, 4))
            errs[f"plain{m}"].append(rel_l2(outm[0], ref[0]))
            hs[f"plain{m}"].append(mean_rel_h(outm[0], ref[0]))
            sp.close()
        if verbose:
            print(f"[eval] seed {seed}: " + ", ".join(f"{k} {errs[k][-1]:.3e}" for k in keys), flush=True)
    for k in keys:
        res["cases"][k] = {"rel_l2_h": float(np.mean(errs[k])), "mean_rel_h": float(np.mean(hs[k])),
                           "time_to_solution_s": float(np.median(times[k])), "per_seed_rel_l2_h": errs[k]}
    res["cases"]["learned"]["fallback_faces_redone_steps"] = fb["learned"]
    return res


def main():
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--n-fine", type=int, default=2048)
    ap.add_argument("--factor", type=int, default=32)
    ap.add_argument("--train-seeds", type=int, default=40)
    ap.add_argument("--traj-steps", type=int, default=1000,
                    help="coarse steps of each training trajectory (the evaluation horizon: a network trained on "
                         "shorter trajectories meets states it never saw and can blow up)")
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--T", type=int, default=32, help="unrolled steps of the loss (eq 2.28 uses 32)")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=2e-5, help="end of the cosine schedule (<= 0: constant)")
    ap.add_argument("--eval-seeds", type=int, default=32)
    ap.add_argument("--val-seeds", type=int, default=8, help="held-out rollouts for checkpoint selection")
    ap.add_argument("--val-steps", type=int, default=1000, help="coarse steps of each validation rollout")
    ap.add_argument("--val-every", type=int, default=100)
    ap.add_argument("--eval-steps", type=int, default=1000)
    ap.add_argument("--plain-sizes", default="64,128,256,512",
                    help="grid sides of the plain-scheme comparison runs (multiples of the coarse side)")
    ap.add_argument("--schemes", default="stencil",
                    help="comma-separated schemes trained and evaluated on the same data: stencil (the learned "
                         "stencil coefficients), direct (the direct face states of section 5.3), blend (the "
                         "stencil coefficients with the flux-limiter blend of section 2.5.3, second approach)")
    ap.add_argument("--eval-blend", action="store_true",
                    help="also evaluate the stencil network trained without the blend with the blend")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    plain_sizes = tuple(int(v) for v in a.plain_sizes.split(",") if v)
    schemes = [x for x in a.schemes.split(",") if x]
    assert all(x in ("stencil", "direct", "blend") for x in schemes), schemes
    t0 = time.perf_counter()
    data = dataset(range(1000, 1000 + a.train_seeds), a.n_fine, a.factor, a.traj_steps)
    tdata = time.perf_counter() - t0
    print(f"[data] {tuple(data.shape)} in {tdata:.1f} s", flush=True)
    val = validation_set(range(3000, 3000 + a.val_seeds), a.n_fine, a.factor, a.val_steps) if a.val_seeds else None
    refs = {}
    out = {}
    eval_seeds = range(5000, 5000 + a.eval_seeds)
    for k, scheme in enumerate(schemes):
        direct, blend = scheme == "direct", scheme == "blend"
        model, hist, wall = train(data, a.iters, a.batch, a.T, a.lr, log_every=100, n_fine=a.n_fine,
                                  factor=a.factor, lr_final=a.lr_final if a.lr_final > 0 else None, direct=direct,
                                  val=val, val_every=a.val_every, blend=blend)
        print(f"[train {scheme}] {a.iters} iterations in {wall:.1f} s, loss {hist[0][2]:.3e} -> {hist[-1][2]:.3e}; "
              f"selected {getattr(model, 'selected', None)}", flush=True)
        res = evaluate(model, eval_seeds, a.n_fine, a.factor, a.eval_steps, plain_sizes=plain_sizes if k == 0 else (),
                       direct=direct, blend=blend, refs=refs, verbose=True)
        print(f"[eval {scheme}] " + ", ".join(f"{c}: rel L2(h) {v['rel_l2_h']:.3e} in "
                                             f"{v['time_to_solution_s'] * 1e3:.1f} ms" for c, v in res["cases"].items()),
              flush=True)
        untrained = fv.Model(init_params(0), model.desc)
        res["untrained"] = evaluate(untrained, eval_seeds, a.n_fine, a.factor, a.eval_steps, plain_sizes=(),
                                    direct=direct, blend=blend, refs=refs)["cases"]["learned"]
        print(f"[eval {scheme}] untrained: rel L2(h) {res['untrained']['rel_l2_h']:.3e}", flush=True)
        if a.eval_blend and scheme == "stencil":
            res["blend"] = evaluate(model, eval_seeds, a.n_fine, a.factor, a.eval_steps, plain_sizes=(), blend=True,
                                    refs=refs)["cases"]["learned"]
            print(f"[eval {scheme}] with the blend: rel L2(h) {res['blend']['rel_l2_h']:.3e} in "
                  f"{res['blend']['time_to_solution_s'] * 1e3:.1f} ms", flush=True)
        res["scheme"] = {"stencil": "stencil coefficients", "direct": "direct face states",
                         "blend": "stencil coefficients with the flux-limiter blend"}[scheme]
        res["train"] = {"iters": a.iters, "batch": a.batch, "T": a.T, "wall_s": wall, "data_s": tdata,
                        "selected": getattr(model, "selected", None), "val_seeds": a.val_seeds,
                        "val_steps": a.val_steps, "traj_steps": a.traj_steps, "loss_first": hist[0][2],
                        "loss_last": hist[-1][2], "snapshots": int(data.shape[0] * data.shape[1])}
        out[scheme] = res
        model.close()
    print(json.dumps(out), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
