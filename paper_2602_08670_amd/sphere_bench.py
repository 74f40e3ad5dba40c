"""Throughput of the spherical shallow-water step (sections 2.4 and 3.3):
cell-updates per second of fv_sphere_run on a 2n x n grid, timed with HIP
events on the solver's stream over K steps after W warm-up steps, inputs
resident on the device.

    python -m paper_2602_08670_amd.sphere_bench --n 512 --steps 200

Workload: a solid-body flow of speed 0.3 balanced by the Coriolis term
(omega 0.5, g 1) with four Gaussian depth bumps (inputs.sphere_state), HLLE,
MINMOD, Heun, CFL 0.4 with the device reduction every step.  Prints one
JSON line per precision."""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import fv, inputs


def run(n: int, steps: int, warmup: int, prec: int, flux: int, seed: int = 0) -> dict:
    import torch

    kw = dict(prec=prec, flux=flux, g=1.0, omega=0.5)
    probe = fv.SphereSolver(np.stack([np.ones((n, 2 * n))] + [np.zeros((n, 2 * n))] * 3), **kw)
    cen = probe.centres()
    probe.close()
    q0 = inputs.sphere_state(cen, seed=seed, u0=0.3, omega=0.5)
    s = fv.SphereSolver(q0, **kw)
    s.run(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.run(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    t, k = s.time()
    tot = s.totals()
    s.close()
    cells = 2 * n * n
    return {"metric": "sphere_cell_updates_per_s", "n": n, "cells": cells, "prec": "f64" if prec == fv.FV_F64 else "f32",
            "steps": steps, "ms_per_step": ms / steps, "value": cells * steps / (ms * 1e-3), "unit": "cell-updates/s",
            "sim_time": t, "mass": float(tot[0]), "energy": float(tot[1])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[512])
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prec", choices=["f32", "f64", "both"], default="both")
    a = ap.parse_args()
    precs = {"f32": [fv.FV_F32], "f64": [fv.FV_F64], "both": [fv.FV_F32, fv.FV_F64]}[a.prec]
    for n in a.n:
        for p in precs:
            print(json.dumps(run(n, a.steps, a.warmup, p, fv.FV_FLUX_HLLE)), flush=True)


if __name__ == "__main__":
    main()
