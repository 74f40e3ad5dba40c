"""GPU direct face-state scheme (thesis section 5.3): the network's four face
states per cell, each face's flux from its two cells' states, against the
oracle's direct_step through the C ABI (fv_direct_step).

Tolerances as the learned step's: the network runs in BF16 with FP32
accumulation on the GPU and in double precision (BF16 rounding passed
through) in the oracle, so face states agree to the BF16 rounding of the
hidden activations: state relative L2 <= 1e-4 after one step and <= 1e-3
after 50 steps; fallback counts within 1 % (a BF16 rounding decision can
flip a face depth's sign near zero)."""
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


def params(L, seed, scale_last, head_bias=None):
    p = L.init_params(seed, scale_last=scale_last)
    g = torch.Generator().manual_seed(seed + 200)
    for l in range(4):
        p["b"][l] = (torch.rand(p["b"][l].shape, generator=g, dtype=torch.float64) * 0.2 - 0.05).float().double()
    if head_bias is not None:
        b = p["b"][4].clone()
        b[:len(head_bias)] = torch.as_tensor(head_bias, dtype=torch.float64)
        p["b"][4] = b.float().double()
    return p


def run_direct(fv, L, p, q0, dt, nsteps, flux="hlle"):
    fl = fv.FV_FLUX_HLLE if flux == "hlle" else fv.FV_FLUX_RUSANOV
    ny, n = q0.shape[-2:]
    vec = fv.params_to_vector([w.numpy() for w in p["w"]], [b.numpy() for b in p["b"]])
    m = fv.Model(vec, fv.make_model_desc(mean=tuple(p["mean"].tolist()), inv_std=tuple(p["inv_std"].tolist())))
    s = fv.Solver(q0.astype(np.float32), prec=fv.FV_F32, dt_fixed=dt, learned=1, flux=fl)
    print(f"[gpu] direct step {flux} {ny}x{n} x{nsteps}", flush=True)
    stats = s.direct_step(m, nsteps)
    t, k = s.time()
    out = s.state()
    s.close()
    m.close()
    qo = torch.tensor(q0.astype(np.float32).astype(np.float64))[None]
    fb, red = 0, 0
    with torch.no_grad():
        for _ in range(nsteps):
            qo, st = L.direct_step(p, qo, dt, 1.0 / n, 1.0 / ny, flux=flux)
            fb += st["fallback_faces"]
            red += int(st["redone"].sum())
    return out, qo[0].numpy(), stats, (fb, red), (t, k)


@pytest.mark.parametrize("flux", ["hlle", "rusanov"])
def test_direct_step_parity(fv, L, flux):
    p = params(L, 3, scale_last=0.05)
    q0 = I.random_smooth_swe(64, seed=21)
    dt = 7.4e-4
    out, ref, stats, ostats, (t, k) = run_direct(fv, L, p, q0, dt, 1, flux)
    print(f"[direct 1 step] {rel_errors(out, ref)}", flush=True)
    assert state_rel(out, ref) <= 1e-4
    assert k == 1 and abs(t - dt) < 1e-9
    out, ref, stats, ostats, _ = run_direct(fv, L, p, q0, dt, 50, flux)
    print(f"[direct 50 steps] {rel_errors(out, ref)} stats gpu {stats} oracle {ostats}", flush=True)
    assert state_rel(out, ref) <= 1e-3
    assert stats == (0, 0) and ostats == (0, 0)


def test_direct_step_parity_layer_by_layer_pass(fv, L):
    """64 x 20 (rows not a multiple of 8): the step's network pass runs
    layer by layer instead of as one tiled launch; parity as above."""
    p = params(L, 7, scale_last=0.05)
    q0 = I.random_smooth_swe(64, seed=25)[:, :20].copy()
    out, ref, stats, ostats, _ = run_direct(fv, L, p, q0, 4e-4, 1)
    print(f"[direct 64x20 1 step] {rel_errors(out, ref)}", flush=True)
    assert state_rel(out, ref) <= 1e-4
    out, ref, stats, ostats, _ = run_direct(fv, L, p, q0, 4e-4, 20)
    print(f"[direct 64x20 20 steps] {rel_errors(out, ref)} stats gpu {stats} oracle {ostats}", flush=True)
    assert state_rel(out, ref) <= 1e-3
    assert stats == ostats


def test_direct_zero_head_is_first_order(fv, L):
    """A zero head: every face state is its cell average (the first-order
    scheme); parity with the oracle, which pins that case to the classic
    first-order oracle."""
    p = params(L, 4, scale_last=0.0)
    q0 = I.random_smooth_swe(32, seed=22)
    out, ref, stats, ostats, _ = run_direct(fv, L, p, q0, 1.5e-3, 10)
    print(f"[direct zero head] {rel_errors(out, ref)}", flush=True)
    assert state_rel(out, ref) <= 1e-5
    assert stats == (0, 0)


def test_direct_negative_depth_head_keeps_depths_positive(fv, L):
    """Height-head bias -200 on every side (-20 de-normalised): the Softplus
    keeps every face depth positive (about 4e-9 of its cell's), so no side
    falls back, on the GPU as in the oracle, and the states agree."""
    hb = [0.0] * 12
    for f in range(4):
        hb[3 * f] = -200.0
    p = params(L, 5, scale_last=0.0, head_bias=hb)
    q0 = I.random_smooth_swe(64, seed=23, humps=4)
    out, ref, stats, ostats, _ = run_direct(fv, L, p, q0, 2e-4, 2)
    print(f"[direct positive] gpu {stats} oracle {ostats} err {state_rel(out, ref):.2e}", flush=True)
    assert stats == (0, 0) and ostats == (0, 0)
    assert state_rel(out, ref) <= 1e-5


def test_direct_fallback_counts_and_state(fv, L):
    """Height-head bias -1e4 (-1e3 de-normalised): the Softplus underflows to
    zero depth in FP32 and in FP64 alike, so every face side of both stages takes its MINMOD state
    (2 axes x 2 sides per cell and stage, counted on both sides) and the step
    is the plain MINMOD step."""
    hb = [0.0] * 12
    for f in range(4):
        hb[3 * f] = -1.0e4
    p = params(L, 5, scale_last=0.3, head_bias=hb)
    q0 = I.random_smooth_swe(64, seed=23, humps=4)
    out, ref, stats, ostats, _ = run_direct(fv, L, p, q0, 2e-4, 1)
    print(f"[direct fallback] gpu {stats} oracle {ostats} err {state_rel(out, ref):.2e}", flush=True)
    assert ostats == (2 * 4 * 64 * 64, 0)
    assert stats == ostats
    assert state_rel(out, ref) <= 1e-5


def test_direct_step_conserves_mass(fv, L):
    """Periodic, any head: the GPU step conserves mass to FP32 rounding."""
    p = params(L, 6, scale_last=0.3)
    q0 = I.random_smooth_swe(64, seed=24)
    vec = fv.params_to_vector([w.numpy() for w in p["w"]], [b.numpy() for b in p["b"]])
    m = fv.Model(vec, fv.make_model_desc(mean=tuple(p["mean"].tolist()), inv_std=tuple(p["inv_std"].tolist())))
    s = fv.Solver(q0.astype(np.float32), prec=fv.FV_F32, dt_fixed=5e-4, learned=1)
    m0 = s.totals()[0]
    stats = s.direct_step(m, 20)
    m1 = s.totals()[0]
    s.close()
    m.close()
    print(f"[direct mass] {m0:.9e} -> {m1:.9e} stats {stats}", flush=True)
    assert stats[1] == 0
    assert abs(m1 - m0) <= 1e-6 * abs(m0)
