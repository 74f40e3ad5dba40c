"""Serving: continuous batching of mixed shallow-water / Euler solves.

Each request's result is bit-identical to the same solve run alone through
fv_run (the batched launch executes the single-solve kernel's per-cell code
and each solve keeps its own CFL reduction), requests are admitted as memory
frees up, and late arrivals overlap with running solves."""
import numpy as np
import pytest
import torch

from paper_2602_08670_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fv():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2602_08670_amd import fv as F

    return F


def make_req(kind, n, seed):
    if kind == "swe":
        q, b = I.swe_bathy(n, seed=seed)
        return q.astype(np.float32), b.astype(np.float32)
    return I.euler_quadrants(n, seed=seed).astype(np.float32), None


def alone(fv, q, b, steps):
    s = fv.Solver(q, b, prec=fv.FV_F32, bc_x=fv.FV_BC_WALL, bc_y=fv.FV_BC_WALL)
    s.run(steps)
    out = s.state().astype(np.float32)
    t, _ = s.time()
    s.close()
    return out, t


def test_mix_bitwise_equals_alone(fv):
    specs = [("swe", 64, 1, 37), ("euler", 128, 2, 50), ("swe", 200, 3, 24), ("euler", 64, 4, 61),
             ("swe", 128, 5, 5), ("euler", 96, 6, 48)]
    srv = fv.Server(64 << 20, max_solves=16, steps_per_round=12, max_items=1 << 14)
    ids = []
    for kind, n, seed, steps in specs:
        q, b = make_req(kind, n, seed)
        ids.append(srv.submit(q, steps, bed=b))
    rounds = 0
    while True:
        a, qd = srv.round()
        rounds += 1
        if a == 0 and qd == 0:
            break
        assert rounds < 100
    for rid, (kind, n, seed, steps) in zip(ids, specs):
        q, b = make_req(kind, n, seed)
        got = srv.result(rid, q.shape)
        ref, t = alone(fv, q, b, steps)
        inf = srv.info(rid)
        print(f"[serve] {kind} {n}^2 {steps} steps: t={inf.sim_time:.6f} alone t={t:.6f}", flush=True)
        assert inf.state == 2 and inf.steps_done == steps
        assert np.array_equal(got, ref), (kind, n, steps)
        assert inf.sim_time == t
    srv.close()


def test_admission_by_memory_and_late_arrivals(fv):
    """A pool that holds only two 256^2 solves: the third waits until one
    finishes; a request submitted while others run joins at the next round."""
    q, b = make_req("swe", 256, 9)
    req_bytes = fv.Server.request_bytes(fv.make_request(q, 10, bed=b)[0])
    import ctypes

    cfg_ov = fv.lib.fv_server_pool_overhead(fv.fv_server_config(ctypes.sizeof(fv.fv_server_config), 8, 10, 0,
                                                               1 << 14))
    assert cfg_ov > 0
    pool = cfg_ov + 2 * req_bytes + 300 * 1024  # room for two 256^2 solves and a small one
    srv = fv.Server(pool, max_solves=8, steps_per_round=10, max_items=1 << 14)
    r1 = srv.submit(q, 30, bed=b)
    r2 = srv.submit(q, 10, bed=b)
    r3 = srv.submit(q, 10, bed=b)
    a, qd = srv.round()
    assert (a, qd) == (1, 1)  # r2 finished in the first server round, r3 still queued (memory)
    assert srv.info(r1).state == 1
    assert srv.info(r3).state == 0 and srv.info(r2).state == 2
    r4 = srv.submit(*make_req("euler", 64, 3)[:1], 20)  # late arrival, small
    a, qd = srv.round()
    assert srv.info(r3).state == 2 and srv.info(r4).state in (1, 2)
    while srv.round() != (0, 0):
        pass
    for rid in (r1, r2, r3, r4):
        assert srv.info(rid).state == 2
    assert srv.info(r4).t_admit > srv.info(r1).t_admit
    ref, _ = alone(fv, q, b, 30)
    assert np.array_equal(srv.result(r1, q.shape), ref)
    srv.close()


@pytest.mark.parametrize("max_bypass", [3, -1])
def test_admission_ageing_bounds_the_wait_of_a_large_request(fv, max_bypass):
    """A pool of about four 64^2 solves; four small solves finishing at
    staggered rounds, then a 128^2 solve (about three small ones), then a
    stream of small ones.  With plain first fit every freed hole goes to the
    next small request and the large one waits until the stream runs dry;
    with ageing (max_bypass 3) nothing is admitted behind it once it has not
    fitted for 3 rounds, so it runs after at most 3 rounds plus the
    remaining rounds of the solves already running."""
    import ctypes

    qs, bs = make_req("swe", 64, 11)
    ql, bl = make_req("swe", 128, 12)
    small = fv.Server.request_bytes(fv.make_request(qs, 8, bed=bs)[0])
    large = fv.Server.request_bytes(fv.make_request(ql, 8, bed=bl)[0])
    K = 8
    ov = fv.lib.fv_server_pool_overhead(fv.fv_server_config(ctypes.sizeof(fv.fv_server_config), 64, K, 0, 1 << 14))
    assert 2 * small < large < 4 * small
    srv = fv.Server(ov + 4 * small + 65536, max_solves=64, steps_per_round=K, max_items=1 << 14,
                    max_bypass=max_bypass)
    first = [srv.submit(qs, K * (k + 1), bed=bs) for k in range(4)]
    big = srv.submit(ql, K, bed=bl)
    stream = [srv.submit(qs, 4 * K, bed=bs) for _ in range(24)]
    rounds = 0
    while srv.round() != (0, 0):
        rounds += 1
        assert rounds < 400
    inf = srv.info(big)
    waits = [srv.info(r).rounds_queued for r in stream]
    print(f"[serve ageing] max_bypass {max_bypass}: large request queued {inf.rounds_queued} rounds, "
          f"small ones up to {max(waits)}; {rounds} rounds", flush=True)
    assert inf.state == 2 and inf.steps_done == K
    assert all(srv.info(r).state == 2 for r in first + stream)
    if max_bypass > 0:
        assert inf.rounds_queued <= max_bypass + 4 + 1
    else:
        assert inf.rounds_queued >= 15
    srv.close()


def test_request_larger_than_pool_rejected(fv):
    q, b = make_req("swe", 512, 1)
    srv = fv.Server(4 << 20, max_solves=4, steps_per_round=4, max_items=1 << 12)
    with pytest.raises(fv.FvError) as e:
        srv.submit(q, 10, bed=b)
    assert e.value.code == fv.FV_E_NOMEM
    srv.close()


def small_model(fv, seed, scale=0.02, bias_last=0.0):
    """A network with small seeded weights (and an optional constant bias on
    the raw coefficients of the last layer)."""
    rng = np.random.default_rng(seed)
    vec = (rng.standard_normal(49448) * scale).astype(np.float32)
    vec[-72:] += bias_last
    return fv.Model(vec, fv.make_model_desc(mean=(1.0, 0.0, 0.0), inv_std=(10.0, 10.0, 10.0)))


def test_learned_mix_bitwise_equals_alone(fv):
    """Learned requests of several sizes served together with plain ones: each
    learned result (state, time, fallback and redo counts) is bit-identical to
    fv_learned_step on the same solve alone -- the server's work-list kernels
    and the single solve's own launches do the same arithmetic per stage."""
    from paper_2602_08670_amd import learned_solver as LS

    m = small_model(fv, 11, scale=0.03, bias_last=0.5)
    dt = LS.fine_dt(2048) * 32
    learned_specs = [(32, 1, 37), (64, 2, 25), (48, 3, 31), (128, 4, 12)]
    plain_specs = [("swe", 64, 5, 20), ("euler", 96, 6, 30)]
    srv = fv.Server(256 << 20, max_solves=16, steps_per_round=10, max_items=1 << 14, model=m)
    lids, pids = [], []
    for n, seed, steps in learned_specs:
        q = I.random_smooth_swe(n, seed=seed).astype(np.float32)
        lids.append(srv.submit(q, steps, learned=True, dt_fixed=dt))
    for kind, n, seed, steps in plain_specs:
        q, b = make_req(kind, n, seed)
        pids.append(srv.submit(q, steps, bed=b))
    rounds = 0
    while True:
        a, qd = srv.round()
        rounds += 1
        if a == 0 and qd == 0:
            break
        assert rounds < 100
    for rid, (n, seed, steps) in zip(lids, learned_specs):
        q = I.random_smooth_swe(n, seed=seed).astype(np.float32)
        got = srv.result(rid, q.shape)
        inf = srv.info(rid)
        s = fv.Solver(q, prec=fv.FV_F32, dt_fixed=dt, learned=1)
        fb, red = s.learned_step(m, steps)
        ref = s.state().astype(np.float32)
        t, k = s.time()
        s.close()
        print(f"[serve learned] {n}^2 {steps} steps: t={inf.sim_time:.6f} alone t={t:.6f}, fallback "
              f"{inf.fallback_faces}/{fb}, redone {inf.redone_steps}/{red}", flush=True)
        assert inf.state == 2 and inf.steps_done == steps
        assert np.array_equal(got, ref), (n, steps)
        assert inf.sim_time == t
        assert (inf.fallback_faces, inf.redone_steps) == (fb, red)
    for rid, (kind, n, seed, steps) in zip(pids, plain_specs):
        q, b = make_req(kind, n, seed)
        ref, t = alone(fv, q, b, steps)
        assert np.array_equal(srv.result(rid, q.shape), ref), (kind, n)
    srv.close()
    m.close()


def test_learned_request_needs_model(fv):
    srv = fv.Server(64 << 20, max_solves=4, steps_per_round=4, max_items=1 << 12)
    q = I.random_smooth_swe(32, seed=0).astype(np.float32)
    with pytest.raises(fv.FvError):
        srv.submit(q, 5, learned=True, dt_fixed=1e-3)
    srv.close()


def test_graph_replay_equals_direct_launches(fv):
    """Rounds replayed from captured graphs give the same bits as direct
    launches.  Requests arrive over several rounds, so the work-lists, the
    launch grids and the kinds of work present change between replays (and
    eager admission work runs between them); steps whose lists are empty run
    launches that read a tile count of zero."""
    from paper_2602_08670_amd import learned_solver as LS

    m = small_model(fv, 5, scale=0.03, bias_last=0.5)
    waves = [
        [("swe", 1024, 1, 7), ("swe", 256, 2, 9), ("euler", 128, 3, 30)],
        [("learned", 1024, 4, 5), ("learned", 128, 5, 9), ("learned", 128, 6, 14)],
        [("swe", 192, 7, 12), ("euler", 64, 8, 3)],
        [],
        [("learned", 64, 9, 6), ("euler", 1024, 10, 5)],
    ]

    def request(kind, n, seed):
        if kind == "learned":
            q = I.random_smooth_swe(n, seed=seed).astype(np.float32)
            return q, None, dict(learned=True, dt_fixed=LS.fine_dt(2048) * 2048 / n)
        q, b = make_req(kind, n, seed)
        return q, b, {}

    runs = []
    for direct in (False, True):
        srv = fv.Server(3 << 30, max_solves=16, steps_per_round=4, max_items=1 << 20, model=m, direct=direct)
        ids = []
        for wave in waves:
            for kind, n, seed, steps in wave:
                q, b, kw = request(kind, n, seed)
                ids.append((srv.submit(q, steps, bed=b, **kw), q.shape))
            srv.round()
        rounds = 0
        while srv.round() != (0, 0):
            rounds += 1
            assert rounds < 100
        out = []
        for rid, shape in ids:
            inf = srv.info(rid)
            out.append((srv.result(rid, shape), inf.state, inf.steps_done, inf.sim_time, inf.fallback_faces,
                        inf.redone_steps))
        st = srv.stats()
        srv.close()
        runs.append(out)
        print(f"[serve graph] direct={direct}: {len(out)} requests, {st.rounds} rounds, {st.graph_replays} "
              f"replays of {st.graphs_captured} graphs, {st.grid_updates} grid updates", flush=True)
        if direct:
            assert st.graph_replays == 0 and st.graphs_captured == 0
        else:
            assert st.graph_replays == st.rounds and 0 < st.graphs_captured < st.graph_replays
            assert st.grid_updates > 0
    specs = [s for wave in waves for s in wave]
    for spec, g, d in zip(specs, runs[0], runs[1]):
        assert g[1] == 2 and g[2] == spec[3], spec
        assert np.array_equal(g[0], d[0]), spec
        assert g[1:] == d[1:], spec
    m.close()


def test_learned_split_and_fused_rounds_agree(fv):
    """The three launch forms of a learned step -- the network pass and the
    learned stage fused per stage with the coefficients in LDS, separate
    launches with alpha through HBM, and separate launches with the network
    pass layer by layer on 16 x 16 tiles -- give the same bits (state, time,
    fallback and redo counts), so a server may pick any per round."""
    from paper_2602_08670_amd import learned_solver as LS

    # zero last-layer weights and large per-channel biases: constant
    # coefficients far from the constraint set, so many face sides fall back
    rng = np.random.default_rng(7)
    vec = (rng.standard_normal(49448) * 0.02).astype(np.float32)
    vec[-72 - 72 * 288:-72] = 0.0
    vec[-72:] = rng.uniform(-400, 400, 72).astype(np.float32)
    m = fv.Model(vec, fv.make_model_desc(mean=(1.0, 0.0, 0.0), inv_std=(10.0, 10.0, 10.0)))
    dt = LS.fine_dt(2048) * 32
    specs = [(32, 1, 13), (64, 2, 9), (128, 3, 7), (256, 4, 5)]
    runs = []
    for split, layered in ((1, -1), (1 << 30, 0), (1, 1)):
        srv = fv.Server(1 << 30, max_solves=8, steps_per_round=4, max_items=1 << 16, model=m, learned_split=split,
                        learned_layered=layered)
        ids = []
        for n, seed, steps in specs:
            q = I.random_smooth_swe(n, seed=seed).astype(np.float32)
            ids.append((srv.submit(q, steps, learned=True, dt_fixed=dt), q.shape))
        rounds = 0
        while srv.round() != (0, 0):
            rounds += 1
            assert rounds < 100
        out = []
        for rid, shape in ids:
            inf = srv.info(rid)
            out.append((srv.result(rid, shape), inf.state, inf.sim_time, inf.fallback_faces, inf.redone_steps))
        st = srv.stats()
        print(f"[serve split] split {split} layered {layered}: {st.rounds} rounds, {st.layered_rounds} layer by layer",
              flush=True)
        assert (st.layered_rounds > 0) == (layered == 1)
        srv.close()
        runs.append(out)
    fb = [o[3] for o in runs[0]]
    print(f"[serve split] fallback faces per request {fb}", flush=True)
    assert sum(fb) > 0  # the comparison covers fallback faces
    for spec, a, b, c in zip(specs, runs[0], runs[1], runs[2]):
        assert a[1] in (2, 3), spec
        assert np.array_equal(a[0], b[0], equal_nan=True), spec
        assert a[1:] == b[1:], spec
        assert np.array_equal(a[0], c[0], equal_nan=True), spec
        assert a[1:] == c[1:], spec
    # the single-solve step picks its form by the same rule (256^2 and up:
    # separate launches) and matches both
    done = 0
    for (n, seed, steps), a in zip(specs, runs[0]):
        if a[1] != 2:
            continue  # a failed solve reports an error alone; its served state was compared above
        done += 1
        q = I.random_smooth_swe(n, seed=seed).astype(np.float32)
        s = fv.Solver(q, prec=fv.FV_F32, dt_fixed=dt, learned=1)
        fbs, red = s.learned_step(m, steps)
        ref = s.state().astype(np.float32)
        t, _ = s.time()
        s.close()
        assert np.array_equal(a[0], ref, equal_nan=True), n
        assert (a[2], a[3], a[4]) == (t, fbs, red), n
    print(f"[serve split] states {[o[1] for o in runs[0]]}, {done} compared with the solve alone", flush=True)
    assert runs[0][-1][1] == 2  # the 256^2 solve (separate launches alone) is among them
    m.close()
