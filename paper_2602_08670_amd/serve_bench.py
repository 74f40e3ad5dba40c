"""Serving benchmark: a seeded stream of shallow-water (over a bed) and Euler
solves of mixed sizes and step counts, run through the continuous-batching
server and through one-solve-at-a-time launches on the same GPU.

Reports whole-stream cell-updates/s and p50/p99 latency (arrival to
completion).  Arrivals: all at t = 0 (saturated), or a Poisson process at a
given rate.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import fv, inputs

SIZES = (64, 128, 256, 512, 1024)


def request_stream(n_req: int, seed: int, sizes=SIZES, steps_lo=100, steps_hi=2000):
    """(kind, n, steps, ic_seed) per request: kind 50/50, n uniform over sizes,
    steps uniform in [steps_lo, steps_hi]; draws in that order per request."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_req):
        kind = "swe" if rng.uniform() < 0.5 else "euler"
        n = int(rng.choice(sizes))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        out.append((kind, n, steps, int(rng.integers(0, 4))))
    return out


class ICCache:
    def __init__(self):
        self.c = {}

    def get(self, kind, n, s):
        key = (kind, n, s)
        if key not in self.c:
            if kind == "swe":
                q, b = inputs.swe_bathy(n, seed=s)
                self.c[key] = (q.astype(np.float32), b.astype(np.float32))
            else:
                self.c[key] = (inputs.euler_quadrants(n, seed=s).astype(np.float32), None)
        return self.c[key]


def arrivals(n_req: int, rate: float, seed: int):
    if rate <= 0:
        return np.zeros(n_req)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return np.cumsum(rng.exponential(1.0 / rate, n_req))


def run_server(stream, ics, arr, pool_bytes=24 << 30, steps_per_round=32, max_solves=1024):
    """Drive the server with the given arrival times (seconds after start)."""
    import torch

    t_create = time.perf_counter()
    srv = fv.Server(pool_bytes, max_solves=max_solves, steps_per_round=steps_per_round, max_items=1 << 18)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    clock_offset = t0 - t_create  # server timestamps count from its creation
    ids = [None] * len(stream)
    nxt = 0
    while True:
        now = time.perf_counter() - t0
        while nxt < len(stream) and arr[nxt] <= now:
            kind, n, steps, s = stream[nxt]
            q, b = ics.get(kind, n, s)
            ids[nxt] = srv.submit(q, steps, bed=b)
            nxt += 1
        a, qd = srv.round()
        if a == 0 and qd == 0:
            if nxt >= len(stream):
                break
            time.sleep(max(0.0, arr[nxt] - (time.perf_counter() - t0)))
    wall = time.perf_counter() - t0
    done, cells = [], 0
    for i, rid in enumerate(ids):
        inf = srv.info(rid)
        assert inf.state == 2, (i, inf.state)
        kind, n, steps, _ = stream[i]
        cells += n * n * steps
        done.append(inf.t_done - clock_offset)
    srv.close()
    return wall, cells, np.array(done), ids


def run_server_latency(stream, ics, arr, **kw):
    wall, cells, t_done, _ = run_server(stream, ics, arr, **kw)
    lat = t_done - arr
    return {"wall_s": wall, "cell_updates": cells, "mcups": cells / wall / 1e6,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(np.mean(lat))}


def run_fifo(stream, ics):
    """One solve at a time: init, run, read back, in arrival order."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cells = 0
    lat = []
    for kind, n, steps, s in stream:
        q, b = ics.get(kind, n, s)
        sv = fv.Solver(q, b, prec=fv.FV_F32, bc_x=fv.FV_BC_WALL, bc_y=fv.FV_BC_WALL)
        sv.run(steps)
        sv.state()
        sv.close()
        cells += n * n * steps
        lat.append(time.perf_counter() - t0)
    wall = time.perf_counter() - t0
    lat = np.array(lat)
    return {"wall_s": wall, "cell_updates": cells, "mcups": cells / wall / 1e6,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--load", type=float, default=0.8, help="Poisson rate as a fraction of the saturated rate")
    ap.add_argument("--no-fifo", action="store_true")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    stream = request_stream(a.requests, a.seed)
    ics = ICCache()
    for kind, n, steps, s in stream:
        ics.get(kind, n, s)
    res = {"requests": a.requests, "seed": a.seed}
    sat = run_server_latency(stream, ics, np.zeros(a.requests))
    res["batched_saturated"] = sat
    rate = a.load * a.requests / sat["wall_s"]
    res["poisson_rate_per_s"] = rate
    res["batched_poisson"] = run_server_latency(stream, ics, arrivals(a.requests, rate, a.seed))
    if not a.no_fifo:
        res["fifo_one_at_a_time"] = run_fifo(stream, ics)
    print(json.dumps(res, indent=1), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
