"""Network pass (BF16 MFMA) latency and throughput.

The stencil-coefficient network of the thesis's section 2.5.3 (fourth
approach: five 3x3 convolutions 3 -> 32 -> 32 -> 32 -> 32 -> 72, ReLU) over
batches of 64^2 coarse shallow-water states, timed with HIP events on the
model's stream for two kernels of libfv:

- the one-launch tiled pass (8 x 8 output tiles, all five layers per
  workgroup, the form the learned step and the server run);
- the layer-by-layer pass (one launch per layer, activations through HBM,
  the form training runs).

The rate is algorithmic: 98 496 FLOP per pixel per evaluation (an FMA counted
as two), whatever a kernel recomputes on tile halos, against the dense BF16
MFMA peak of the MI355X (2.5 PFLOP/s).

    python -m paper_2602_08670_amd.network_bench --batches 1,256 --reps 50
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import fv, inputs

FLOP_PER_PIXEL = (27 * 32 + 3 * 288 * 32 + 288 * 72) * 2
BF16_PEAK_TFLOPS = 2500.0
N = 64


def _time(fn, reps, stream, torch):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps  # microseconds per pass


def run(batches, reps):
    import torch

    assert FLOP_PER_PIXEL == 98496
    rng = np.random.default_rng(0)
    vec = (rng.standard_normal(fv.fv_model_param_count()) * 0.02).astype(np.float32)
    m = fv.Model(vec, fv.make_model_desc(mean=(1.0, 0.0, 0.0), inv_std=(10.0, 10.0, 10.0)))
    st = m.stream
    out = {"flop_per_pixel": FLOP_PER_PIXEL, "peak_tflops": BF16_PEAK_TFLOPS, "grid": N, "reps": reps, "runs": []}
    for B in batches:
        q = np.stack([inputs.random_smooth_swe(N, seed=s) for s in range(B)]).astype(np.float32)
        qd = torch.as_tensor(q, device=m.device).contiguous()
        z = torch.empty((B, N, N, 72), dtype=torch.float32, device=m.device)
        nb = fv.fv_model_forward_scratch_bytes(B, N, N)
        sc = torch.empty(nb, dtype=torch.uint8, device=m.device)
        flop = FLOP_PER_PIXEL * B * N * N
        for name, fn in (("tiled", lambda: fv.fv_model_forward_tiled(m.h, qd.data_ptr(), B, N, N, z.data_ptr())),
                         ("layer_by_layer", lambda: fv.fv_model_forward(m.h, qd.data_ptr(), B, N, N, z.data_ptr(),
                                                                         sc.data_ptr(), nb))):
            us = _time(fn, reps, st, torch)
            tf = flop / (us * 1e-6) / 1e12
            rec = {"kernel": name, "batch": B, "pixels": B * N * N, "us_per_pass": round(us, 2),
                   "tflops": round(tf, 2), "frac_of_peak": round(tf / BF16_PEAK_TFLOPS, 4)}
            out["runs"].append(rec)
            print(f"[network] {name:15s} batch {B:4d}: {us:9.2f} us per pass, {tf:8.2f} TFLOP/s "
                  f"({tf / BF16_PEAK_TFLOPS:.2%} of the BF16 peak)", flush=True)
    m.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--batches", default="1,256")
    ap.add_argument("--reps", type=int, default=50)
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    res = run([int(b) for b in a.batches.split(",")], a.reps)
    print(json.dumps(res), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
