"""GPU admissibility redo of the learned schemes (section 5.2: a negative depth
makes the learned solve produce NaN): a shallow state (depth about 0.1) and a
large random head make a learned stage leave cells with non-positive depth,
so the solve's whole step is redone with the plain MINMOD scheme.  The
oracle pins that case to its plain step exactly (tests/test_oracle_learned.py);
here the GPU must take the same redo decisions and reach the oracle's state
(the redone step is the plain FP32 step: relative L2 <= 1e-5 after one step).
Over three steps the redo counts must agree and the states stay within the
learned step's tolerance."""
import numpy as np
import pytest
import torch

from parity import rel_errors, state_rel
from paper_2602_08670_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fv():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2602_08670_amd import fv as F

    return F


@pytest.fixture(scope="module")
def L():
    from oracle import learned

    return learned


def shallow_state(n=32):
    q0 = I.random_smooth_swe(n, seed=2)
    q0[0] *= 0.1
    return q0


def run(fv, L, scheme, p, q0, dt, nsteps, flux="hlle"):
    fl = fv.FV_FLUX_HLLE if flux == "hlle" else fv.FV_FLUX_RUSANOV
    ny, n = q0.shape[-2:]
    vec = fv.params_to_vector([w.numpy() for w in p["w"]], [b.numpy() for b in p["b"]])
    m = fv.Model(vec, fv.make_model_desc(mean=tuple(p["mean"].tolist()), inv_std=tuple(p["inv_std"].tolist())))
    s = fv.Solver(q0.astype(np.float32), prec=fv.FV_F32, dt_fixed=dt, learned=1, flux=fl)
    print(f"[gpu] redo {scheme} {flux} {ny}x{n} x{nsteps}", flush=True)
    step = {"learned": s.learned_step, "direct": s.direct_step, "blend": s.blend_step}[scheme]
    stats = step(m, nsteps)
    out = s.state()
    s.close()
    m.close()
    qo = torch.tensor(q0.astype(np.float32).astype(np.float64))[None]
    red = 0
    with torch.no_grad():
        for _ in range(nsteps):
            if scheme == "direct":
                qo, st = L.direct_step(p, qo, dt, 1.0 / n, 1.0 / ny, flux=flux)
            else:
                qo, st = L.learned_step(p, qo, dt, 1.0 / n, 1.0 / ny, flux=flux, blend=scheme == "blend")
            red += int(st["redone"].sum())
    return out, qo[0].numpy(), stats, red


@pytest.mark.parametrize("scheme", ["learned", "direct", "blend"])
@pytest.mark.parametrize("flux", ["hlle", "rusanov"])
def test_forced_redo_matches_oracle(fv, L, scheme, flux):
    p = L.init_params(2, scale_last=10.0)
    q0 = shallow_state()
    out, ref, stats, ored = run(fv, L, scheme, p, q0, 1e-3, 1, flux)
    print(f"[redo {scheme} {flux} 1 step] gpu {stats} oracle redo {ored} {rel_errors(out, ref)}", flush=True)
    assert ored == 1
    assert stats[1] == 1
    assert state_rel(out, ref) <= 1e-5
    qp = L.plain_step(torch.tensor(q0.astype(np.float32).astype(np.float64))[None], 1e-3, 1 / 32, 1 / 32)
    assert state_rel(out, qp[0].numpy()) <= 1e-5
    out, ref, stats, ored = run(fv, L, scheme, p, q0, 1e-3, 3, flux)
    print(f"[redo {scheme} {flux} 3 steps] gpu {stats} oracle redo {ored} {rel_errors(out, ref)}", flush=True)
    assert ored >= 1 and stats[1] == ored
    assert state_rel(out, ref) <= 1e-4


@pytest.mark.parametrize("n", [32, 128])
@pytest.mark.parametrize("scheme", ["learned", "blend", "direct"])
def test_redo_inside_a_call_bitwise(fv, L, scheme, n):
    """A single solve's learned steps run two launches per step: a flagged
    step is redone inside the next step's first launch (each workgroup redoes
    it on the region it reads), the call's last step by the commit-or-redo and
    redo launches.  States, time and counts are bit-identical to one-step
    calls (every step ended by those launches) and, for the learned scheme,
    to the server (separate launches at the end of every step), for an even
    and an odd step count.  32^2 runs the single solve's 4 x 4 network tiles,
    128^2 its 8 x 8 tiles (the server's)."""
    p = L.init_params(2, scale_last=10.0)
    q0 = shallow_state(n).astype(np.float32)
    vec = fv.params_to_vector([w.numpy() for w in p["w"]], [b.numpy() for b in p["b"]])
    m = fv.Model(vec, fv.make_model_desc(mean=tuple(p["mean"].tolist()), inv_std=tuple(p["inv_std"].tolist())))
    dt = 1e-3 * 32 / n
    for steps in (4, 5):
        s = fv.Solver(q0, prec=fv.FV_F32, dt_fixed=dt, learned=1)
        step = {"learned": s.learned_step, "direct": s.direct_step, "blend": s.blend_step}[scheme]
        fb, red = step(m, steps)
        got, (t, k) = s.state(), s.time()
        s.close()
        s = fv.Solver(q0, prec=fv.FV_F32, dt_fixed=dt, learned=1)
        step = {"learned": s.learned_step, "direct": s.direct_step, "blend": s.blend_step}[scheme]
        for _ in range(steps):
            fb1, red1 = step(m, 1)
        one, (t1, k1) = s.state(), s.time()
        s.close()
        print(f"[redo in call] {scheme} {n}^2 {steps} steps: redone {red} / one-step calls {red1}, fallback "
              f"{fb}/{fb1}", flush=True)
        assert red >= 2 and (fb, red) == (fb1, red1)
        assert np.array_equal(got, one) and (t, k) == (t1, k1) and k == steps
        if scheme != "learned":
            continue
        srv = fv.Server(64 << 20, max_solves=4, steps_per_round=10, max_items=1 << 12, model=m)
        rid = srv.submit(q0, steps, learned=True, dt_fixed=dt)
        rounds = 0
        while True:
            a, qd = srv.round()
            rounds += 1
            if a == 0 and qd == 0:
                break
            assert rounds < 10
        served = srv.result(rid, q0.shape)
        inf = srv.info(rid)
        srv.close()
        print(f"[redo in call] served: redone {inf.redone_steps}, fallback {inf.fallback_faces}", flush=True)
        assert np.array_equal(served, got.astype(np.float32))
        assert (inf.fallback_faces, inf.redone_steps) == (fb, red) and inf.sim_time == t
    m.close()


@pytest.mark.parametrize("scheme", ["learned", "direct"])
def test_graph_replay_with_redos_bitwise(fv, L, scheme):
    """Learned steps captured in a HIP graph (an even number per graph, so
    that the replays keep alternating the flag slots) and replayed three
    times give the bits, time and redo count of the same steps called
    directly, with every step redone."""
    import torch

    p = L.init_params(2, scale_last=10.0)
    q0 = shallow_state().astype(np.float32)
    vec = fv.params_to_vector([w.numpy() for w in p["w"]], [b.numpy() for b in p["b"]])
    m = fv.Model(vec, fv.make_model_desc(mean=tuple(p["mean"].tolist()), inv_std=tuple(p["inv_std"].tolist())))
    dt, chunk, reps = 1e-3, 4, 3
    st = torch.cuda.Stream()
    s = fv.Solver(q0, prec=fv.FV_F32, dt_fixed=dt, learned=1, stream=st)
    step = s.direct_step if scheme == "direct" else s.learned_step
    with torch.cuda.stream(st):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            step(m, chunk, want_stats=False)
    torch.cuda.synchronize()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    got, (t, k) = s.state(), s.time()
    fb, red = step(m, 0)
    s.close()
    s = fv.Solver(q0, prec=fv.FV_F32, dt_fixed=dt, learned=1)
    step = s.direct_step if scheme == "direct" else s.learned_step
    fb1, red1 = step(m, chunk * reps)
    ref, (t1, k1) = s.state(), s.time()
    s.close()
    m.close()
    print(f"[graph redo] {scheme}: replayed redone {red} fallback {fb}; direct redone {red1} fallback {fb1}",
          flush=True)
    assert red1 == chunk * reps and (fb, red) == (fb1, red1)
    assert np.array_equal(got, ref) and (t, k) == (t1, k1)
