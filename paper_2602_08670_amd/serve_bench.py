"""Serving benchmark: a seeded stream of solves of mixed sizes and step
counts, run through the continuous-batching server and through
one-solve-at-a-time launches on the same GPU.

Default stream: shallow water over a bed and Euler, 50/50, sides
{64..1024}, 100..2000 steps.  --mixed: learned and plain shallow-water
solves, 50/50; learned sides {32, 64, 128, 256} on a periodic domain of side
n/64 (the training resolution dx = 1/64) at the training step, with a
network trained in-process on a short dataset; plain sides {64..2048} over a
bed with walls.

Reports whole-stream cell-updates/s and p50/p99 latency (arrival to
completion).  Arrivals: all at t = 0 (saturated), or a Poisson process at a
given rate.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import fv, inputs

SIZES = (64, 128, 256, 512, 1024)
LEARNED_SIZES = (32, 64, 128, 256)
PLAIN_SIZES_MIXED = (64, 128, 256, 512, 1024, 2048)


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


def mixed_stream(n_req: int, seed: int, steps_lo=100, steps_hi=2000):
    """(kind, n, steps, ic_seed): kind learned/swe 50/50, n uniform over the
    kind's sizes, steps uniform in [steps_lo, steps_hi]; draws in that order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_req):
        learned = rng.uniform() < 0.5
        n = int(rng.choice(LEARNED_SIZES if learned else PLAIN_SIZES_MIXED))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        out.append(("learned" if learned else "swe", n, steps, int(rng.integers(0, 4))))
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
            elif kind == "learned":
                self.c[key] = (inputs.random_smooth_swe(n, seed=s).astype(np.float32), None)
            else:
                self.c[key] = (inputs.euler_quadrants(n, seed=s).astype(np.float32), None)
        return self.c[key]


def submit_kw(kind, n, learned_dt):
    if kind == "learned":
        return {"learned": True, "dt_fixed": learned_dt, "lx": n / 64.0}
    return {}


def arrivals(n_req: int, rate: float, seed: int):
    if rate <= 0:
        return np.zeros(n_req)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return np.cumsum(rng.exponential(1.0 / rate, n_req))


def run_server(stream, ics, arr, pool_bytes=24 << 30, steps_per_round=32, max_solves=1024, model=None,
               learned_dt=0.0, direct=False):
    """Drive the server with the given arrival times (seconds after start).
    direct: launch every kernel directly instead of replaying captured graphs."""
    import torch

    t_create = time.perf_counter()
    srv = fv.Server(pool_bytes, max_solves=max_solves, steps_per_round=steps_per_round, max_items=1 << 22,
                    model=model, direct=direct)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    clock_offset = t0 - t_create  # server timestamps count from its creation
    ids = [None] * len(stream)
    nxt = 0
    rounds = 0
    while True:
        now = time.perf_counter() - t0
        while nxt < len(stream) and arr[nxt] <= now:
            kind, n, steps, s = stream[nxt]
            q, b = ics.get(kind, n, s)
            ids[nxt] = srv.submit(q, steps, bed=b, **submit_kw(kind, n, learned_dt))
            nxt += 1
        a, qd = srv.round()
        rounds += 1
        if rounds % 200 == 0:
            print(f"[serve] {nxt}/{len(stream)} submitted, {a} running, {qd} queued", file=sys.stderr, flush=True)
        if a == 0 and qd == 0:
            if nxt >= len(stream):
                break
            time.sleep(max(0.0, arr[nxt] - (time.perf_counter() - t0)))
    wall = time.perf_counter() - t0
    done, cells, queued = [], 0, []
    fallback = redone = 0
    for i, rid in enumerate(ids):
        inf = srv.info(rid)
        assert inf.state == 2, (i, inf.state)
        kind, n, steps, _ = stream[i]
        cells += n * n * steps
        done.append(inf.t_done - clock_offset)
        queued.append(inf.rounds_queued)
        fallback += inf.fallback_faces
        redone += inf.redone_steps
    st = srv.stats()
    run_server.last_stats = {"rounds_queued_max": int(max(queued)), "rounds_queued_p99": float(np.percentile(queued, 99)),
                             "rounds": st.rounds, "graph_replays": st.graph_replays,
                             "graphs_captured": st.graphs_captured, "grid_updates": st.grid_updates,
                             "layered_rounds": st.layered_rounds,
                             "host_launch_s": st.host_launch_s, "host_wait_s": st.host_wait_s,
                             "host_capture_s": st.host_capture_s, "host_admit_s": st.host_admit_s,
                             "host_retire_s": st.host_retire_s}
    srv.close()
    return wall, cells, np.array(done), ids, (fallback, redone)


def run_server_latency(stream, ics, arr, **kw):
    wall, cells, t_done, _, (fb, red) = run_server(stream, ics, arr, **kw)
    lat = t_done - arr
    res = {"wall_s": wall, "cell_updates": cells, "mcups": cells / wall / 1e6,
           "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
           "mean_s": float(np.mean(lat))}
    kinds = sorted({k for k, *_ in stream})
    if len(kinds) > 1:
        for kd in kinds:
            sel = np.array([k == kd for k, *_ in stream])
            res[f"p50_s_{kd}"] = float(np.percentile(lat[sel], 50))
            res[f"p99_s_{kd}"] = float(np.percentile(lat[sel], 99))
    if "learned" in kinds:
        res["learned_fallback_faces"] = int(fb)
        res["learned_redone_steps"] = int(red)
    res["server"] = dict(run_server.last_stats)
    return res


def run_fifo(stream, ics, model=None, learned_dt=0.0):
    """One solve at a time: init, run, read back, in arrival order."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cells = 0
    lat = []
    for i, (kind, n, steps, s) in enumerate(stream):
        q, b = ics.get(kind, n, s)
        if kind == "learned":
            sv = fv.Solver(q, prec=fv.FV_F32, dt_fixed=learned_dt, learned=1, lx=n / 64.0, ly=n / 64.0)
            fv.fv_learned_step(sv.h, model.h, steps, want_stats=False)
        else:
            sv = fv.Solver(q, b, prec=fv.FV_F32, bc_x=fv.FV_BC_WALL, bc_y=fv.FV_BC_WALL)
            sv.run(steps)
        sv.state()
        sv.close()
        cells += n * n * steps
        lat.append(time.perf_counter() - t0)
        if (i + 1) % 200 == 0:
            print(f"[fifo] {i + 1}/{len(stream)} done", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    lat = np.array(lat)
    return {"wall_s": wall, "cell_updates": cells, "mcups": cells / wall / 1e6,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99))}


def quick_model(train_seeds=8, traj_steps=256, iters=800):
    """A network trained in-process for the mixed stream (the serving
    figures do not depend on how well it is trained; its cost does not
    depend on its weights)."""
    from . import learned_solver as LS

    data = LS.dataset(range(1000, 1000 + train_seeds), 2048, 32, traj_steps)
    model, hist, wall = LS.train(data, iters, 16, 8, 1e-3, n_fine=2048, factor=32, lr_final=2e-5)
    print(f"[model] trained {iters} iterations in {wall:.1f} s, loss {hist[-1][2]:.3e}", flush=True)
    return model, LS.fine_dt(2048) * 32


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--load", type=float, default=0.8, help="Poisson rate as a fraction of the saturated rate")
    ap.add_argument("--mixed", action="store_true", help="learned + plain shallow-water stream")
    ap.add_argument("--pool-gb", type=float, default=24.0)
    ap.add_argument("--no-fifo", action="store_true")
    ap.add_argument("--compare-direct", action="store_true",
                    help="also run the saturated stream with direct launches instead of graph replay")
    ap.add_argument("--direct-last", action="store_true", help="with --compare-direct: run the direct pass "
                    "after the graph pass")
    ap.add_argument("--direct", action="store_true", help="launch every kernel directly instead of replaying "
                    "captured graphs")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    model, ldt = (quick_model() if a.mixed else (None, 0.0))
    stream = mixed_stream(a.requests, a.seed) if a.mixed else request_stream(a.requests, a.seed)
    ics = ICCache()
    for kind, n, steps, s in stream:
        ics.get(kind, n, s)
    kw = {"pool_bytes": int(a.pool_gb * (1 << 30)), "model": model, "learned_dt": ldt}
    if a.direct:
        kw["direct"] = True
    res = {"requests": a.requests, "seed": a.seed, "mixed": a.mixed, "pool_gb": a.pool_gb}
    # warm-up, not part of any figure: the first pass through a process loads
    # the kernels' code and first-touches the host buffers of the request
    # copies and results (about 1 s for the plain stream); the plain stream is
    # replayed whole, the mixed one (a minute per pass) by its first requests
    nw = min(64, a.requests) if a.mixed else a.requests
    run_server(stream[:nw], ics, np.zeros(nw), **kw)
    res["warmup_requests"] = nw
    def direct_pass():
        dsat = run_server_latency(stream, ics, np.zeros(a.requests), **{**kw, "direct": True})
        res["batched_saturated_direct"] = dsat
        print(f"[saturated, direct launches] {dsat['mcups']:.0f} Mcell-updates/s in {dsat['wall_s']:.1f} s",
              flush=True)

    if a.compare_direct and not a.direct_last:
        direct_pass()
    sat = run_server_latency(stream, ics, np.zeros(a.requests), **kw)
    res["batched_saturated"] = sat
    print(f"[saturated] {sat['mcups']:.0f} Mcell-updates/s in {sat['wall_s']:.1f} s", flush=True)
    if a.compare_direct and a.direct_last:
        direct_pass()
    rate = a.load * a.requests / sat["wall_s"]
    res["poisson_rate_per_s"] = rate
    res["batched_poisson"] = run_server_latency(stream, ics, arrivals(a.requests, rate, a.seed), **kw)
    print(f"[poisson] p50 {res['batched_poisson']['p50_s']:.3f} s p99 {res['batched_poisson']['p99_s']:.3f} s",
          flush=True)
    if not a.no_fifo:
        res["fifo_one_at_a_time"] = run_fifo(stream, ics, model, ldt)
    print(json.dumps(res, indent=1), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
