"""Grid-size sweep of the FP32 classic step.

Workload per size N: shallow water over the seeded bed (8 Gaussians under a
free surface of 16 Gaussian bumps, at rest), N x N, reflective walls, HLLE,
MINMOD, Heun, CFL 0.4 with the wave-speed reduction every step; or (--eqn
euler) the seeded four-quadrant Euler data.  For each size and seed: `runs`
timed runs of `steps` steps (HIP events on the solver's stream, after a
warm-up), median and spread reported as cell-updates/s, the algorithmic HBM
fraction (28 B per cell-update for shallow water over a bed, 32 B for Euler,
against 8 TB/s) and the ALU fraction (543 / 715 FP32 operations per
cell-update, an FMA counted as two, against the 78.6 TFLOP/s non-packed FP32
vector peak).  One JSON line per (size, seed) is printed as it completes.

    python -m paper_2602_08670_amd.stage_sweep --sizes 1024 2048 4096 8192 --seeds 0 1 2 --runs 5 --out FILE
"""
from __future__ import annotations

import argparse
import json
import statistics
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
ALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
BYTES = {"swe": 28, "euler": 32}
FLOP = {"swe": 543, "euler": 715}


def steps_for(n: int) -> int:
    return int(min(400, max(20, (1 << 28) // (n * n))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[1024, 2048, 4096, 8192])
    ap.add_argument("--seeds", type=int, nargs="+", default=[0, 1, 2])
    ap.add_argument("--runs", type=int, default=5)
    ap.add_argument("--steps", type=int, default=0, help="steps per timed run (0: by size)")
    ap.add_argument("--eqn", choices=["swe", "euler"], default="swe")
    ap.add_argument("--out", default="")
    a = ap.parse_args()

    import torch

    from paper_2602_08670_amd import fv, inputs

    rows = []
    for n in a.sizes:
        for seed in a.seeds:
            t0 = time.perf_counter()
            if a.eqn == "swe":
                q0, b = inputs.swe_bathy(n, seed=seed)
            else:
                q0, b = inputs.euler_quadrants(n, seed=seed), None
            s = fv.Solver(q0.astype(np.float32), None if b is None else b.astype(np.float32), prec=fv.FV_F32,
                          bc_x=fv.FV_BC_WALL, bc_y=fv.FV_BC_WALL)
            del q0, b
            steps = a.steps or steps_for(n)
            s.run(max(5, steps // 10))
            torch.cuda.synchronize()
            times = []
            for _ in range(a.runs):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(s.stream)
                s.run(steps)
                e1.record(s.stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1) / 1e3 / steps)
            _, done = s.time()
            s.close()
            med = statistics.median(times)
            rate = n * n / med
            row = {"eqn": a.eqn, "n": n, "seed": seed, "steps_per_run": steps, "runs": a.runs,
                   "us_per_step_median": round(med * 1e6, 3),
                   "us_per_step_min": round(min(times) * 1e6, 3), "us_per_step_max": round(max(times) * 1e6, 3),
                   "gcups": round(rate / 1e9, 2),
                   "hbm_frac": round(BYTES[a.eqn] * rate / 1e9 / HBM_PEAK_GBS, 4),
                   "alu_frac": round(FLOP[a.eqn] * rate / 1e12 / ALU_PEAK_TFLOPS, 4),
                   "setup_s": round(time.perf_counter() - t0 - sum(times) * steps, 1), "steps_done": done}
            rows.append(row)
            print(json.dumps(row), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f, indent=1)
            f.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
