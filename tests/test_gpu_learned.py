"""GPU <-> oracle parity of the learned-coefficient path, through the C ABI.

The oracle (oracle/learned.py) evaluates the network in double precision with
bfloat16 rounding at the points where the GPU rounds (normalised input,
post-ReLU activations, weights); the GPU accumulates in FP32 on MFMA.  A
rounding decision differs when an FP32 sum lands on the other side of a
bfloat16 midpoint than the double sum; each such activation moves by one
bfloat16 ulp (2^-8 relative).  The oracle's float32-accumulation shadow
(same rounding points, float32 sums) measures how far FP32 accumulation alone
moves z from the double result.  With few pixels a handful of flips
dominates, so the GPU's z must stay within max(2 x shadow distance, 5e-4)
relative L2, and at most 1 % of the entries may differ by more than
1e-3 max|z| (a wrong tap, channel or lane mapping corrupts most of them).  The state
tolerances after 1 and 100 learned steps (1e-4 and 1e-3 relative L2 of the
state vector) add FP32 state storage and the FP32 flux arithmetic."""
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


def oracle_params(L, seed, scale_last, bias_last=None):
    p = L.init_params(seed, scale_last=scale_last)
    g = torch.Generator().manual_seed(seed + 100)
    for l in range(4):
        p["b"][l] = (torch.rand(p["b"][l].shape, generator=g, dtype=torch.float64) * 0.2 - 0.05).float().double()
    if bias_last is not None:
        p["b"][4] = torch.as_tensor(bias_last, dtype=torch.float64).float().double()
    return p


def gpu_model(fv, p):
    vec = fv.params_to_vector([w.numpy() for w in p["w"]], [b.numpy() for b in p["b"]])
    desc = fv.make_model_desc(mean=tuple(p["mean"].tolist()), inv_std=tuple(p["inv_std"].tolist()))
    return fv.Model(vec, desc)


def test_network_forward_matches_oracle(fv, L):
    p = oracle_params(L, 1, scale_last=0.3)
    q = np.stack([I.random_smooth_swe(64, seed=s) for s in range(3)])
    q[:, 1] = 0.05 * np.sin(np.arange(64) / 7.0)[None, None, :]
    q32 = q.astype(np.float32)
    print("[gpu] network forward B=3 64x64", flush=True)
    m = gpu_model(fv, p)
    z = m.forward(torch.tensor(q32, device="cuda")).cpu().double().numpy()  # [B, ny, nx, 72]
    check_z(L, p, q32, z, "64x64 B=3")
    m.close()


def check_z(L, p, q32, z, tag):
    qd = torch.tensor(q32.astype(np.float64))
    zo = L.cnn(p, qd).permute(0, 2, 3, 1).numpy()
    zs = L.cnn(p, qd, shadow_f32=True).permute(0, 2, 3, 1).numpy()
    rel = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    floor = np.linalg.norm(zs - zo) / np.linalg.norm(zo)
    print(f"[net {tag}] rel L2 {rel:.2e} (float32-accumulation shadow {floor:.2e}), max abs "
          f"{np.abs(z - zo).max():.2e}, max |z| {np.abs(zo).max():.2e}", flush=True)
    frac = float(np.mean(np.abs(z - zo) > 1e-3 * np.abs(zo).max()))
    assert rel <= max(2.0 * floor, 5e-4)
    assert frac <= 0.01, frac


def test_network_ragged_batch_and_sizes(fv, L):
    """32x32 and 16x64 grids, batch of 5 (grid not a multiple of the 64-pixel workgroup per solve)."""
    p = oracle_params(L, 2, scale_last=0.3)
    m = gpu_model(fv, p)
    for ny, nx, B in ((32, 32, 5), (16, 64, 2), (64, 16, 1)):
        q = (1.0 + 0.1 * np.random.default_rng(ny * nx + B).standard_normal((B, 3, ny, nx))).astype(np.float32)
        z = m.forward(torch.tensor(q, device="cuda")).cpu().double().numpy()
        check_z(L, p, q, z, f"{ny}x{nx} B={B}")
    m.close()


def test_tiled_forward_bitwise_equals_layer_by_layer(fv, L):
    """The one-launch tiled pass recomputes each tile's halo in LDS but keeps
    every output's MFMA order, bias, ReLU and BF16 rounding: z must be
    bit-identical to the layer-by-layer pass (several tiles, periodic wrap
    across tile and grid edges, batches)."""
    p = oracle_params(L, 3, scale_last=0.3)
    m = gpu_model(fv, p)
    # the last three select 16-, 8- and 16-row workgroup tiles in the layer-by-layer pass
    for ny, nx, B in ((64, 64, 3), (32, 32, 5), (8, 16, 1), (24, 48, 2), (64, 64, 128), (64, 64, 64), (24, 64, 256)):
        q = (1.0 + 0.1 * np.random.default_rng(7 * ny + nx + B).standard_normal((B, 3, ny, nx))).astype(np.float32)
        qt = torch.tensor(q, device="cuda")
        z1 = m.forward(qt).cpu().numpy()
        z2 = m.forward_tiled(qt).cpu().numpy()
        ndiff = int(np.sum(z1 != z2))
        print(f"[tiled] {ny}x{nx} B={B}: {ndiff} differing of {z1.size}", flush=True)
        assert ndiff == 0
    m.close()


def test_layer_by_layer_forward_independent_of_batch(fv, L):
    """The layer-by-layer pass picks its workgroup tile height from the grid
    size (16, 8 or 4 rows); a solve's z is the same bits in a large batch
    (16- or 8-row tiles, the last tile cut by ny) as alone (4-row tiles)."""
    p = oracle_params(L, 4, scale_last=0.3)
    m = gpu_model(fv, p)
    for ny, nx, B in ((36, 64, 128), (24, 64, 256)):
        q = (1.0 + 0.1 * np.random.default_rng(ny + B).standard_normal((B, 3, ny, nx))).astype(np.float32)
        qt = torch.tensor(q, device="cuda")
        zb = m.forward(qt).cpu().numpy()
        for b in (0, B // 2, B - 1):
            z1 = m.forward(qt[b:b + 1].contiguous()).cpu().numpy()
            ndiff = int(np.sum(z1[0] != zb[b]))
            print(f"[batch] {ny}x{nx} B={B} solve {b}: {ndiff} differing", flush=True)
            assert ndiff == 0
    m.close()


def run_learned(fv, L, p, q0, dt, nsteps, flux="hlle"):
    fl = fv.FV_FLUX_HLLE if flux == "hlle" else fv.FV_FLUX_RUSANOV
    n = q0.shape[-1]
    m = gpu_model(fv, p)
    s = fv.Solver(q0.astype(np.float32), prec=fv.FV_F32, dt_fixed=dt, learned=1, flux=fl)
    stats = s.learned_step(m, nsteps)
    t, k = s.time()
    out = s.state()
    s.close()
    m.close()
    qo = torch.tensor(q0.astype(np.float32).astype(np.float64))[None]
    fb, red = 0, 0
    with torch.no_grad():
        for _ in range(nsteps):
            qo, st = L.learned_step(p, qo, dt, 1.0 / n, 1.0 / n, flux=flux)
            fb += st["fallback_faces"]
            red += int(st["redone"].sum())
    return out, qo[0].numpy(), stats, (fb, red), (t, k)


@pytest.mark.parametrize("flux", ["hlle", "rusanov"])
def test_learned_step_parity(fv, L, flux):
    p = oracle_params(L, 3, scale_last=0.05)
    q0 = I.random_smooth_swe(64, seed=11)
    dt = 7.4e-4
    out, ref, stats, ostats, (t, k) = run_learned(fv, L, p, q0, dt, 1, flux)
    print(f"[learned 1 step] {rel_errors(out, ref)}", flush=True)
    assert state_rel(out, ref) <= 1e-4
    assert k == 1 and abs(t - dt) < 1e-9
    out, ref, stats, ostats, _ = run_learned(fv, L, p, q0, dt, 100, flux)
    print(f"[learned 100 steps] {rel_errors(out, ref)} stats gpu {stats} oracle {ostats}", flush=True)
    assert state_rel(out, ref) <= 1e-3
    assert stats == (0, 0) and ostats == (0, 0)


@pytest.mark.parametrize("ny,nx", [(48, 80), (24, 48), (96, 64)])
def test_learned_step_parity_rectangular(fv, L, ny, nx):
    """Rectangular periodic grids (rows cut from a square state: both sides
    wrap the same data): 48 x 80 and 24 x 48 run the single solve's 4 x 4
    network tiles, 96 x 64 its 8 x 8 tiles (more 4 x 4 tiles than resident
    workgroups).  Three learned steps against the oracle with dx = 1/nx and
    dy = 1/ny, within the learned step's tolerance."""
    p = oracle_params(L, 3, scale_last=0.05)
    q0 = I.random_smooth_swe(max(nx, ny), seed=21)[:, :ny, :nx].astype(np.float32)
    dt, nsteps = 4e-4, 3
    m = gpu_model(fv, p)
    s = fv.Solver(q0, prec=fv.FV_F32, dt_fixed=dt, learned=1)
    print(f"[gpu] learned step {ny}x{nx} x{nsteps}", flush=True)
    stats = s.learned_step(m, nsteps)
    out = s.state()
    s.close()
    m.close()
    qo = torch.tensor(q0.astype(np.float64))[None]
    fb = 0
    with torch.no_grad():
        for _ in range(nsteps):
            qo, st = L.learned_step(p, qo, dt, 1.0 / nx, 1.0 / ny)
            fb += st["fallback_faces"]
    print(f"[learned {ny}x{nx}] {rel_errors(out, qo[0].numpy())} stats gpu {stats} oracle fallback {fb}", flush=True)
    assert state_rel(out, qo[0].numpy()) <= 3e-4
    assert stats[1] == 0 and abs(stats[0] - fb) <= 0.01 * fb + 2


def test_zero_network_is_fromm(fv, L, orc):
    """A zero last layer gives alpha_base (Fromm); parity with the oracle."""
    p = oracle_params(L, 4, scale_last=0.0)
    q0 = I.random_smooth_swe(64, seed=12)
    out, ref, *_ = run_learned(fv, L, p, q0, 7.4e-4, 20)
    assert state_rel(out, ref) <= 1e-4


def test_fallback_counts_and_state(fv, L):
    """A large last-layer bias sends many face sides to the MINMOD state:
    counts and states agree with the oracle."""
    rng = np.random.default_rng(5)
    p = oracle_params(L, 5, scale_last=0.0, bias_last=rng.uniform(-400, 400, 72))
    q0 = I.random_smooth_swe(64, seed=13, humps=4)
    out, ref, stats, ostats, _ = run_learned(fv, L, p, q0, 2e-4, 1)
    print(f"[fallback] gpu {stats} oracle {ostats} err {state_rel(out, ref):.2e}", flush=True)
    assert ostats[0] > 100
    assert abs(stats[0] - ostats[0]) <= 0.01 * ostats[0] + 2
    assert ostats[1] >= 1
    assert stats[1] == ostats[1]
    assert state_rel(out, ref) <= 1e-4


def test_learned_step_rejects_unsupported(fv):
    q0 = I.random_smooth_swe(64, seed=1)
    p = np.zeros(fv.fv_model_param_count(), dtype=np.float32)
    m = fv.Model(p)
    s = fv.Solver(q0, prec=fv.FV_F32, dt_fixed=1e-4, learned=0)
    with pytest.raises(fv.FvError) as e:
        s.learned_step(m, 1)
    assert e.value.code == fv.FV_E_UNSUPPORTED
    s.close()
    m.close()
