"""GPU <-> oracle parity of the learned Euler step (oracle/learned_euler.py)
through the C ABI (fv_euler_learned_*).

Tolerances as the planar learned path's: the network's raw coefficients
within max(2 x the oracle's float32-accumulation shadow distance, 5e-4)
relative L2 with at most 1 % of the entries off by more than 1e-3 max|z|;
the state within 1e-4 relative L2 after one learned step and 1e-3 after 50;
fallback counts within 1 % and redo decisions equal; the FP64 totals of
mass, momentum and energy conserved to 1e-6 (FP32 state)."""
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
def E():
    from oracle import learned_euler

    return learned_euler


def oracle_params(E, seed, scale_last, bias_last=None):
    p = E.init_params(seed, scale_last=scale_last)
    g = torch.Generator().manual_seed(seed + 100)
    for l in range(4):
        p["b"][l] = (torch.rand(p["b"][l].shape, generator=g, dtype=torch.float64) * 0.2 - 0.05).float().double()
    if bias_last is not None:
        p["b"][4] = torch.as_tensor(bias_last, dtype=torch.float64).float().double()
    return p


def gpu_net(fv, p, B, n, dt, flux="hlle"):
    vec = fv.params_to_vector([w.numpy() for w in p["w"]], [b.numpy() for b in p["b"]])
    return fv.EulerLearned(vec, B, n, n, dt, flux=fv.FV_FLUX_HLLE if flux == "hlle" else fv.FV_FLUX_RUSANOV,
                           mean=tuple(p["mean"].tolist()), inv_std=tuple(p["inv_std"].tolist()))


def states(seeds, n):
    return np.stack([I.random_smooth_euler(n, seed=s) for s in seeds]).astype(np.float32)


def test_network_forward_matches_oracle(fv, E):
    p = oracle_params(E, 1, scale_last=0.3)
    q32 = states([0, 1, 2], 48)
    print("[gpu] Euler network forward B=3 48x48", flush=True)
    net = gpu_net(fv, p, 3, 48, 1e-3)
    z = net.forward(torch.tensor(q32, device="cuda")).cpu().double().numpy()  # [B, ny, nx, 96]
    net.close()
    qd = torch.tensor(q32.astype(np.float64))
    zo = E.L.cnn(p, qd).permute(0, 2, 3, 1).numpy()
    zs = E.L.cnn(p, qd, shadow_f32=True).permute(0, 2, 3, 1).numpy()
    rel = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    floor = np.linalg.norm(zs - zo) / np.linalg.norm(zo)
    frac = float(np.mean(np.abs(z - zo) > 1e-3 * np.abs(zo).max()))
    print(f"[euler net] rel L2 {rel:.2e} (shadow {floor:.2e}), off entries {frac:.4f}", flush=True)
    assert rel <= max(2.0 * floor, 5e-4)
    assert frac <= 0.01


def run(fv, E, p, q0, dt, nsteps, flux="hlle"):
    B, _, n, _ = q0.shape
    net = gpu_net(fv, p, B, n, dt, flux)
    q = torch.tensor(q0, device="cuda").contiguous()
    net.step(q, nsteps)
    fb, rd, fr, rc = net.stats()
    out = q.cpu().double().numpy()
    net.close()
    qo = torch.tensor(q0.astype(np.float64))
    ofb, ord_ = 0, np.zeros(B, dtype=np.int64)
    with torch.no_grad():
        for _ in range(nsteps):
            qo, st = E.learned_step(p, qo, dt, 1.0 / n, 1.0 / n, flux=flux)
            ofb += st["fallback_faces"]
            ord_ += st["redone"].numpy().astype(np.int64)
    return out, qo.numpy(), (int(fb.sum()), rd), (ofb, ord_), rc


@pytest.mark.parametrize("flux", ["hlle", "rusanov"])
def test_learned_step_parity(fv, E, flux):
    p = oracle_params(E, 3, scale_last=0.05)
    q0 = states([11, 12], 64)
    dt = 5e-4
    print(f"[gpu] learned Euler {flux} 2 x 64^2, 1 and 50 steps", flush=True)
    out, ref, st, ost, rc = run(fv, E, p, q0, dt, 1, flux)
    for b in range(2):
        print(f"[euler 1 step] solve {b} {rel_errors(out[b], ref[b])}", flush=True)
        assert state_rel(out[b], ref[b]) <= 1e-4
    out, ref, st, ost, rc = run(fv, E, p, q0, dt, 50, flux)
    for b in range(2):
        print(f"[euler 50 steps] solve {b} {rel_errors(out[b], ref[b])} stats gpu {st} oracle {ost}", flush=True)
        assert state_rel(out[b], ref[b]) <= 1e-3
    assert rc == fv.FV_OK
    assert abs(st[0] - ost[0]) <= 0.01 * ost[0] + 2
    assert st[1].tolist() == ost[1].tolist()


def test_learned_step_parity_rectangular(fv, E):
    """A rectangular 48 x 80 solve (rows cut from an 80 x 80 state), whose
    4 x 4 network tiles all get a workgroup: three learned steps against the
    oracle with dx = 1/80 and dy = 1/48."""
    p = oracle_params(E, 3, scale_last=0.05)
    ny, nx, dt, nsteps = 48, 80, 3e-4, 3
    q0 = np.stack([I.random_smooth_euler(nx, seed=13)[:, :ny, :]]).astype(np.float32)
    net = fv.EulerLearned(fv.params_to_vector([w.numpy() for w in p["w"]], [b.numpy() for b in p["b"]]), 1, nx, ny,
                          dt, mean=tuple(p["mean"].tolist()), inv_std=tuple(p["inv_std"].tolist()))
    print(f"[gpu] learned Euler {ny}x{nx} x{nsteps}", flush=True)
    q = torch.tensor(q0, device="cuda").contiguous()
    net.step(q, nsteps)
    fb, rd, fr, rc = net.stats()
    out = q.cpu().double().numpy()
    net.close()
    qo = torch.tensor(q0.astype(np.float64))
    with torch.no_grad():
        for _ in range(nsteps):
            qo, _ = E.learned_step(p, qo, dt, 1.0 / nx, 1.0 / ny)
    print(f"[euler {ny}x{nx}] {rel_errors(out[0], qo[0].numpy())}", flush=True)
    assert rc == fv.FV_OK and int(rd.sum()) == 0
    assert state_rel(out[0], qo[0].numpy()) <= 3e-4


def test_zero_head_is_fromm_and_conserves(fv, E):
    """A zero last layer (Fromm's stencils): parity over 20 steps on a
    ragged 48 x 20 grid, and FP64 sums of every conserved variable kept."""
    p = oracle_params(E, 4, scale_last=0.0)
    n = 48
    q0 = np.stack([I.random_smooth_euler(n, seed=5)[:, :20, :]]).astype(np.float32)
    # a periodic 48 x 20 grid: rows cut from a 48 x 48 state are not periodic
    # in y, which is fine for parity (both sides wrap the same data)
    net = fv.EulerLearned(fv.params_to_vector([w.numpy() for w in p["w"]], [b.numpy() for b in p["b"]]), 1, n, 20,
                          4e-4, mean=tuple(p["mean"].tolist()), inv_std=tuple(p["inv_std"].tolist()))
    q = torch.tensor(q0, device="cuda").contiguous()
    net.step(q, 20)
    out = q.cpu().double().numpy()
    net.close()
    qo = torch.tensor(q0.astype(np.float64))
    with torch.no_grad():
        for _ in range(20):
            qo, _ = E.learned_step(p, qo, 4e-4, 1.0 / n, 1.0 / 20)
    print(f"[euler fromm 48x20] {rel_errors(out[0], qo[0].numpy())}", flush=True)
    assert state_rel(out[0], qo[0].numpy()) <= 1e-4
    s0 = q0.astype(np.float64).sum(axis=(2, 3))
    s1 = out.sum(axis=(2, 3))
    scale = np.abs(q0.astype(np.float64)).sum(axis=(2, 3))
    assert np.all(np.abs(s1 - s0) <= 1e-6 * scale), (s0, s1)


def test_fallback_and_redo(fv, E):
    """A large head and a step near the CFL limit on a low-pressure and a
    mild state: many face sides fall back and a solve redoes its step with
    the plain scheme (here the mild one: its learned stage leaves a cell
    with p <= 0); the GPU agrees with the oracle on the counts, on which
    solve is redone and on both states."""
    n = 32
    qa = I.random_smooth_euler(n, seed=2)
    kin = 0.5 * (qa[1] ** 2 + qa[2] ** 2) / qa[0]
    qa[3] = kin + 0.1 * (qa[3] - kin)
    qb = I.random_smooth_euler(n, seed=3)
    q0 = np.stack([qa, qb]).astype(np.float32)
    p = oracle_params(E, 2, scale_last=10.0)
    print("[gpu] learned Euler fallback/redo 2 x 32^2", flush=True)
    out, ref, st, ost, rc = run(fv, E, p, q0, 5e-3, 1)
    print(f"[euler fallback] gpu {st} oracle {ost} errs {[state_rel(out[b], ref[b]) for b in range(2)]}", flush=True)
    assert ost[0] > 100 and ost[1].sum() >= 1
    assert abs(st[0] - ost[0]) <= 0.01 * ost[0] + 2
    assert st[1].tolist() == ost[1].tolist()
    for b in range(2):
        assert state_rel(out[b], ref[b]) <= 1e-4


def test_batch_equals_single(fv, E):
    """Each solve of a batch of three gives the same bits as alone."""
    p = oracle_params(E, 6, scale_last=0.1)
    q0 = states([21, 22, 23], 32)
    outs = []
    for B, qq in ((3, q0), (1, q0[1:2])):
        net = gpu_net(fv, p, B, 32, 5e-4)
        q = torch.tensor(qq, device="cuda").contiguous()
        net.step(q, 5)
        outs.append(q.cpu().numpy())
        net.close()
    assert np.array_equal(outs[0][1], outs[1][0])


def test_fused_stage_equals_separate_launches(fv, E):
    """A batch whose tiles outnumber the resident workgroups runs the network
    pass and the learned stage as separate launches; one solve runs them
    fused in one launch per stage.  The same bits per solve, over steps with
    fallbacks."""
    p = oracle_params(E, 7, scale_last=10.0)
    B, n = 20, 64  # 20 x 64 tiles of 8 x 8 exceed one workgroup per CU
    q0 = states(list(range(40, 40 + B)), n)
    kin = 0.5 * (q0[:, 1] ** 2 + q0[:, 2] ** 2) / q0[:, 0]
    q0[:, 3] = kin + 0.1 * (q0[:, 3] - kin)  # low pressure: some learned sides fall back
    net = gpu_net(fv, p, B, n, 5e-4)
    q = torch.tensor(q0, device="cuda").contiguous()
    net.step(q, 6)
    fb, _, _, _ = net.stats()
    batched = q.cpu().numpy()
    net.close()
    print(f"[euler fused] batch of {B}: fallback sides {int(fb.sum())}", flush=True)
    assert fb.sum() > 0
    for b in (0, 7, B - 1):
        one = gpu_net(fv, p, 1, n, 5e-4)
        q1 = torch.tensor(q0[b:b + 1], device="cuda").contiguous()
        one.step(q1, 6)
        fb1, _, _, _ = one.stats()
        one.close()
        print(f"[euler fused] solve {b}: fallback sides {fb[b]} / alone {fb1[0]}", flush=True)
        assert np.array_equal(q1.cpu().numpy()[0], batched[b])
        assert fb1[0] == fb[b]


@pytest.mark.parametrize("n", [32, 64])
def test_redo_inside_a_call_bitwise(fv, E, n):
    """Two launches per step on whole 8 x 8 tiles: a solve whose step is
    flagged is redone inside the next step's first launch (each workgroup
    redoes it on the region it reads), the call's last step by the
    commit-or-redo and redo launches.  Over steps with redos of both solves,
    states and counts equal one-step calls (every step ended by those
    launches) bit for bit, for an even and an odd step count.  Two 32^2
    solves run on 4 x 4 network tiles, two 64^2 solves on 8 x 8 tiles."""
    qa = I.random_smooth_euler(n, seed=2)
    kin = 0.5 * (qa[1] ** 2 + qa[2] ** 2) / qa[0]
    qa[3] = kin + 0.1 * (qa[3] - kin)
    q0 = np.stack([qa, I.random_smooth_euler(n, seed=3)]).astype(np.float32)
    p = E.init_params(2, scale_last=10.0)
    for steps in (4, 5):
        res = []
        for calls in (1, steps):
            net = gpu_net(fv, p, 2, n, 5e-3 * 32 / n)
            q = torch.tensor(q0, device="cuda").contiguous()
            for _ in range(calls):
                net.step(q, steps // calls)
            fb, rd, fr, rc = net.stats()
            res.append((q.cpu().numpy(), fb.tolist(), rd.tolist(), fr.tolist(), rc))
            net.close()
        print(f"[euler redo in call] {steps} steps: one call {res[0][1:]} / one-step calls {res[1][1:]}", flush=True)
        assert res[0][4] == fv.FV_OK and max(res[0][3]) == 0
        assert sum(res[0][2]) >= (steps if n == 32 else 2)
        assert np.array_equal(res[0][0], res[1][0]) and res[0][1:] == res[1][1:]


@pytest.mark.parametrize("n", [32, 64])
def test_frozen_solve_leaves_the_batch_unchanged(fv, E, n):
    """A solve whose state is inadmissible from the start (negative pressure
    in a band) fails its plain redo and is frozen; the other solve of the
    batch runs on, bit-identical to the same solve alone, in the two-launch
    form whose workgroups skip a frozen solve's tiles (4 x 4 network tiles at
    32^2, 8 x 8 at 64^2)."""
    p = E.init_params(2, scale_last=0.05)
    bad = I.random_smooth_euler(n, seed=6)
    kin = 0.5 * (bad[1] ** 2 + bad[2] ** 2) / bad[0]
    bad[3, n // 4:n // 2, :] = kin[n // 4:n // 2, :] - 0.05  # p < 0 in a band of rows
    good = I.random_smooth_euler(n, seed=7)
    q0 = np.stack([bad, good]).astype(np.float32)
    dt, steps = 5e-4 * 32 / n, 4
    net = gpu_net(fv, p, 2, n, dt)
    q = torch.tensor(q0, device="cuda").contiguous()
    net.step(q, steps)
    fb, rd, fr, rc = net.stats()
    both = q.cpu().numpy()
    net.close()
    one = gpu_net(fv, p, 1, n, dt)
    q1 = torch.tensor(q0[1:2], device="cuda").contiguous()
    one.step(q1, steps)
    fb1, rd1, fr1, rc1 = one.stats()
    alone = q1.cpu().numpy()
    one.close()
    print(f"[euler frozen {n}^2] frozen {fr.tolist()} rc {rc}, redone {rd.tolist()}, fallback {fb.tolist()}; "
          f"alone frozen {fr1.tolist()} rc {rc1}", flush=True)
    assert fr.tolist() == [1, 0] and rc == fv.FV_E_INADMISSIBLE
    assert fr1.tolist() == [0] and rc1 == fv.FV_OK
    assert np.array_equal(both[1], alone[0]) and (fb[1], rd[1]) == (fb1[0], rd1[0])


def test_invalid_configurations_rejected(fv):
    vec = np.zeros(fv.lib.fv_euler_net_param_count(), dtype=np.float32)
    for kw in (dict(nx=40), dict(flux=fv.FV_FLUX_ROE), dict(dt=0.0)):
        args = dict(B=1, nx=32, ny=32, dt=1e-3)
        args.update(kw)
        with pytest.raises(fv.FvError):
            fv.EulerLearned(vec, **args)


# ---- training (eq 2.28 on the Euler state) ---------------------------------
# Tolerances as the planar trainer's: the GPU backward runs the network in
# BF16 with FP32 accumulation, the oracle in double precision with bfloat16
# rounding passed straight through; cosine >= 0.999 and relative L2 <= 1e-2
# for the parameter and input gradients, every layer's cosine >= 0.995, the
# loss within 1e-3.

def _grad_vec(ws, bs):
    parts = []
    for w, b in zip(ws, bs):
        parts += [w.reshape(-1), b.reshape(-1)]
    return torch.cat(parts).numpy()


def _cos(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.mark.parametrize("flux,ny,nx", [("hlle", 32, 32), ("rusanov", 32, 32), ("hlle", 24, 48)])
def test_gradients_match_oracle(fv, E, flux, ny, nx):
    B, T, dt = 2, 2, 4e-4 * 32 / nx
    p = oracle_params(E, 21, scale_last=0.1)
    q0 = np.stack([I.random_smooth_euler(nx, seed=40 + b)[:, :ny, :] for b in range(B)]).astype(np.float32)
    with torch.no_grad():
        tg, qq = [], torch.tensor(q0.astype(np.float64)) * 1.002
        for _ in range(T):
            qq = E.plain_step(qq, dt, 1 / nx, 1 / ny, flux=flux)
            tg.append(qq.float().double())
        tg = torch.stack(tg, 1)  # [B, T, 4, ny, nx]
    scale = (0.1, 0.1, 0.1, 0.2)
    print(f"[gpu] Euler train grad parity {flux} B={B} T={T} {ny}x{nx}", flush=True)
    vec = fv.params_to_vector([w.numpy() for w in p["w"]], [b.numpy() for b in p["b"]])
    fl = fv.FV_FLUX_HLLE if flux == "hlle" else fv.FV_FLUX_RUSANOV
    net = fv.EulerLearned(vec, B, nx, ny, dt, flux=fl, mean=tuple(p["mean"].tolist()),
                          inv_std=tuple(p["inv_std"].tolist()))
    tr = fv.EulerTrainer(net, fv.make_euler_train_config(B, nx, ny, T, dt, flux=fl, scale=scale))
    tgt = torch.tensor(tg.permute(1, 0, 2, 3, 4).numpy().astype(np.float32), device="cuda")
    loss, stats = tr.step(torch.tensor(q0, device="cuda"), tgt)
    g_gpu = tr.grads.cpu().double().numpy()
    gq_gpu = tr.input_grad().cpu().double().numpy()
    tr.close()
    net.close()
    for t in p["w"] + p["b"]:
        t.requires_grad_(True)
    qv = torch.tensor(q0.astype(np.float64), requires_grad=True)
    lo = E.rollout_loss(p, qv, tg, dt, 1 / nx, 1 / ny, scale, flux=flux)
    gw = torch.autograd.grad(lo, p["w"] + p["b"] + [qv])
    g_or = _grad_vec(gw[:5], gw[5:10])
    gq_or = gw[10].numpy()
    c, rel = _cos(g_gpu, g_or), np.linalg.norm(g_gpu - g_or) / np.linalg.norm(g_or)
    cq, relq = _cos(gq_gpu.ravel(), gq_or.ravel()), np.linalg.norm(gq_gpu - gq_or) / np.linalg.norm(gq_or)
    print(f"[euler grad] loss gpu {loss:.6e} oracle {lo.item():.6e}; theta cos {c:.6f} rel {rel:.2e}; "
          f"q0 cos {cq:.6f} rel {relq:.2e}; stats {stats}", flush=True)
    assert abs(loss - lo.item()) <= 1e-3 * lo.item()
    assert c >= 0.999 and rel <= 1e-2
    assert cq >= 0.999 and relq <= 1e-2
    off = 0
    for l, (w, b) in enumerate(zip(gw[:5], gw[5:10])):
        k = w.numel() + b.numel()
        assert _cos(g_gpu[off:off + k], g_or[off:off + k]) >= 0.995, l
        off += k


def test_adam_reduces_loss(fv, E):
    """Fitting a rollout of the plain scheme from the same states: Adam on the
    GPU gradients lowers the unrolled loss within 60 iterations, and the
    parameters stay finite."""
    B, n, T, dt = 4, 32, 4, 4e-4
    p = oracle_params(E, 7, scale_last=0.0)
    q0 = states([50, 51, 52, 53], n)
    with torch.no_grad():
        tg, qq = [], torch.tensor(q0.astype(np.float64))
        for _ in range(T):
            qq = E.plain_step(qq, dt, 1 / n, 1 / n)
            tg.append(qq.float())
    tgt = torch.stack(tg).to("cuda")  # [T, B, 4, n, n]
    net = gpu_net(fv, p, B, n, dt)
    tr = fv.EulerTrainer(net, fv.make_euler_train_config(B, n, n, T, dt, lr=3e-4))
    qd = torch.tensor(q0, device="cuda")
    losses = []
    for _ in range(60):
        loss, _ = tr.step(qd, tgt)
        losses.append(loss)
        tr.adam()
    print(f"[euler adam] loss {losses[0]:.4e} -> {losses[-1]:.4e}", flush=True)
    assert losses[-1] < 0.5 * losses[0]
    assert bool(torch.isfinite(net.params).all())
    tr.close()
    net.close()


@pytest.mark.parametrize("B,ny,nx", [(1, 64, 64), (3, 48, 32), (2, 24, 80)])
def test_tiled_forward_bitwise_equals_layer_by_layer(fv, E, B, ny, nx):
    """The one-launch network pass (8 x 8 tiles, halo recomputed in LDS) gives
    the same bits as the layer-by-layer pass: per output the MFMA order,
    bias, ReLU and BF16 rounding are the same."""
    p = oracle_params(E, 8, scale_last=0.3)
    q = np.stack([I.random_smooth_euler(max(nx, ny), seed=30 + b)[:, :ny, :nx] for b in range(B)]).astype(np.float32)
    vec = fv.params_to_vector([w.numpy() for w in p["w"]], [b.numpy() for b in p["b"]])
    net = fv.EulerLearned(vec, B, nx, ny, 1e-3, mean=tuple(p["mean"].tolist()), inv_std=tuple(p["inv_std"].tolist()))
    qd = torch.tensor(q, device="cuda")
    z0 = net.forward(qd).cpu().numpy()
    z1 = net.forward_tiled(qd).cpu().numpy()
    net.close()
    print(f"[euler tiled {B}x{ny}x{nx}] max |diff| {np.abs(z0 - z1).max():.3e}", flush=True)
    assert np.array_equal(z0, z1)
