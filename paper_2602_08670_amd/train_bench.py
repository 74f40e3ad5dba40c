"""Training-step timing: the unrolled loss of eq 2.28 with its full backward
(learned FV adjoint, network input and weight gradients) and the Adam update,
on batches of coarse windows from a small seeded classic-scheme dataset.

    python -m paper_2602_08670_amd.train_bench --batch 16 --T 16 --iters 60

Every kernel is libfv's; the windows are gathered with torch indexing (data
plumbing).  Reports the median wall time per phase over the timed iterations
(each phase synchronised, so the times are GPU-bound step times)."""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import fv
from . import learned_solver as ls


def main():
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--T", type=int, default=16)
    ap.add_argument("--n-fine", type=int, default=512)
    ap.add_argument("--factor", type=int, default=8)
    ap.add_argument("--seeds", type=int, default=4)
    ap.add_argument("--traj-steps", type=int, default=64)
    ap.add_argument("--iters", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    B, T = a.batch, a.T
    data = ls.dataset(range(1000, 1000 + a.seeds), a.n_fine, a.factor, a.traj_steps)
    n = a.n_fine // a.factor
    print(f"[data] {tuple(data.shape)}", flush=True)
    mean, inv_std, std = ls.normalisation(data)
    model = fv.Model(ls.init_params(0), fv.make_model_desc(mean=mean, inv_std=inv_std))
    cfg = fv.make_train_config(B, n, n, T, ls.fine_dt(a.n_fine) * a.factor, h_ref=1.0, scale=tuple(std), lr=1e-3)
    tr = fv.Trainer(model, cfg)
    rng = np.random.default_rng(1)
    n_traj, S1 = data.shape[0], data.shape[1]
    tw = torch.arange(1, T + 1, device=data.device)
    ph = {"gather": [], "step": [], "adam": []}
    for it in range(a.warmup + a.iters):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ti = torch.as_tensor(rng.integers(0, n_traj, B), device=data.device)
        ki = torch.as_tensor(rng.integers(0, S1 - T, B), device=data.device)
        q0 = data[ti, ki].contiguous()
        tg = data[ti[None, :], ki[None, :] + tw[:, None]].contiguous()  # [T, B, 3, n, n]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tr.step(q0, tg)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tr.adam()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if it >= a.warmup:
            ph["gather"].append(t1 - t0)
            ph["step"].append(t2 - t1)
            ph["adam"].append(t3 - t2)
    tr.close()
    model.close()
    res = {"batch": B, "T": T, "grid": n, "iters": a.iters,
           **{f"{k}_ms": 1e3 * float(np.median(v)) for k, v in ph.items()}}
    # learned stages (forward and backward) x cells per second
    res["stage_cells_per_s"] = B * T * 2 * n * n / (res["step_ms"] * 1e-3)
    print(json.dumps(res), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
