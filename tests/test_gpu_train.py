"""GPU training path: gradients of the unrolled loss (eq 2.28) against the
oracle's automatic differentiation, determinism, optimisation progress and
the block-average coarsening.

Gradient tolerance: the GPU backward runs the network in BF16 with FP32
accumulation (activations, weights and the back-propagated signals are
BF16), the oracle in double precision with bfloat16 rounding passed
straight through, so the gradients agree to a few bfloat16 ulps per
operation: cosine similarity >= 0.999 and relative L2 <= 1e-2.

The flux-limiter blend is trained with the limiter frozen in the gradient
(its derivative, of order one over the local difference, overflows on a flat
background): the blend cases use the same data as the others, flat
background included, and the same bounds."""
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


@pytest.fixture(scope="module")
def L():
    from oracle import learned

    return learned


def params(L, seed, scale_last=0.05):
    p = L.init_params(seed, scale_last=scale_last)
    g = torch.Generator().manual_seed(seed + 7)
    for l in range(5):
        p["b"][l] = (torch.rand(p["b"][l].shape, generator=g, dtype=torch.float64) * 0.1 - 0.02).float().double()
    return p


def vec(fv, p):
    return fv.params_to_vector([w.numpy() for w in p["w"]], [b.numpy() for b in p["b"]])


def grad_vec(p_grads_w, p_grads_b):
    parts = []
    for w, b in zip(p_grads_w, p_grads_b):
        parts += [w.reshape(-1), b.reshape(-1)]
    return torch.cat(parts).numpy()


def cos(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def batch(n, B, seed0, ny=None):
    """B smooth states on an n x n grid; with ny < n the first ny rows (the
    periodic seam then carries a jump)."""
    q = np.stack([I.random_smooth_swe(n, seed=seed0 + b) for b in range(B)])
    q[:, 1] = 0.02 * np.sin(2 * np.pi * np.arange(n) / n)[None, None, :]
    if ny is not None:
        q = q[:, :, :ny].copy()
    return q.astype(np.float32)


@pytest.mark.parametrize("flux,ny,nx,direct,blend", [("hlle", 32, 32, False, False), ("rusanov", 32, 32, False, False),
                                                     ("hlle", 24, 48, False, False), ("hlle", 32, 32, True, False),
                                                     ("rusanov", 32, 32, True, False), ("hlle", 32, 32, False, True),
                                                     ("rusanov", 32, 32, False, True), ("hlle", 24, 48, False, True)])
def test_gradients_match_oracle(fv, L, flux, ny, nx, direct, blend):
    """Square grids, and 24 x 48: rows past the last full 16-row tile of the
    input-gradient convolutions; the learned scheme, the direct face-state
    scheme (section 5.3: the adjoint passes each side's gradient to its own
    cell and to its own cell's channels of the network output) and the
    learned scheme with the flux-limiter blend (section 2.5.3, second
    approach: through the low-resolution flux, the limiter frozen)."""
    B, T, dt = 2, 2, 1.2e-3 * 32 / nx
    p = params(L, 21)
    q0 = batch(nx, B, 40, ny)
    # targets: the plain scheme from slightly perturbed states (non-zero loss)
    with torch.no_grad():
        tg, qq = [], torch.tensor(q0.astype(np.float64)) * 1.002
        for _ in range(T):
            qq = L.plain_step(qq, dt, 1 / nx, 1 / ny, flux=flux)
            tg.append(qq.float().double())
        tg = torch.stack(tg, 1)  # [B, T, 3, ny, nx]
    scale = (0.05, 0.02, 0.02)
    print(f"[gpu] train grad parity {flux} B={B} T={T} {ny}x{nx} direct={direct} blend={blend}", flush=True)
    m = fv.Model(vec(fv, p), fv.make_model_desc(mean=(1.0, 0.0, 0.0), inv_std=(10.0, 10.0, 10.0)))
    cfg = fv.make_train_config(B, nx, ny, T, dt, flux=fv.FV_FLUX_HLLE if flux == "hlle" else fv.FV_FLUX_RUSANOV,
                               scale=scale, h_ref=1.0, direct=direct, blend=blend)
    tr = fv.Trainer(m, cfg)
    tgt = torch.tensor(tg.permute(1, 0, 2, 3, 4).numpy().astype(np.float32), device="cuda")
    loss, stats = tr.step(torch.tensor(q0, device="cuda"), tgt)
    g_gpu = tr.grads.cpu().double().numpy()
    gq_gpu = tr.input_grad().cpu().double().numpy()
    tr.close()
    m.close()
    # oracle: autograd of the same rollout
    for t in p["w"] + p["b"]:
        t.requires_grad_(True)
    qv = torch.tensor(q0.astype(np.float64), requires_grad=True)
    lo = L.rollout_loss(p, qv, tg, dt, 1 / nx, 1 / ny, scale, flux=flux, direct=direct, blend=blend)
    gw = torch.autograd.grad(lo, p["w"] + p["b"] + [qv])
    g_or = grad_vec(gw[:5], gw[5:10])
    gq_or = gw[10].numpy()
    c, rel = cos(g_gpu, g_or), np.linalg.norm(g_gpu - g_or) / np.linalg.norm(g_or)
    cq, relq = cos(gq_gpu.ravel(), gq_or.ravel()), np.linalg.norm(gq_gpu - gq_or) / np.linalg.norm(gq_or)
    print(f"[grad] loss gpu {loss:.6e} oracle {lo.item():.6e}; theta cos {c:.6f} rel {rel:.2e}; "
          f"q0 cos {cq:.6f} rel {relq:.2e}; stats {stats}", flush=True)
    assert abs(loss - lo.item()) <= 1e-3 * lo.item()
    assert c >= 0.999 and rel <= 1e-2
    assert np.all(np.isfinite(g_gpu)) and np.all(np.isfinite(gq_gpu))
    assert cq >= 0.999 and relq <= 1e-2
    # per layer: the weight gradient of every layer is right (not only the large ones)
    off = 0
    for l, (w, b) in enumerate(zip(gw[:5], gw[5:10])):
        k = w.numel() + b.numel()
        a, o = g_gpu[off:off + k], g_or[off:off + k]
        assert cos(a, o) >= 0.995, (l, cos(a, o))
        off += k


def test_gradients_bitwise_repeatable(fv, L):
    n, B, T, dt = 32, 3, 2, 1.0e-3
    p = params(L, 22)
    q0 = torch.tensor(batch(n, B, 50), device="cuda")
    tgt = torch.stack([q0 * 1.001, q0 * 0.999])
    m = fv.Model(vec(fv, p))
    tr = fv.Trainer(m, fv.make_train_config(B, n, n, T, dt))
    l1, _ = tr.step(q0, tgt)
    g1 = tr.grads.clone()
    l2, _ = tr.step(q0, tgt)
    assert l1 == l2 and torch.equal(g1, tr.grads)
    tr.close()
    m.close()


def test_gradients_batch_equals_mean_of_solves(fv, L):
    """The loss of eq 2.28 averages over the batch, so the gradient of a
    batch of sixteen 64^2 solves is the mean of the sixteen single-solve
    gradients: per pixel the two runs compute the same values (the batch
    takes 16, 8 or 4-row tiles where a solve alone takes others), only the
    order of the FP32 sums over pixels and workgroups differs."""
    n, B, T, dt = 64, 16, 2, 6.0e-4
    p = params(L, 24)
    q0 = torch.tensor(batch(n, B, 70), device="cuda")
    tgt = torch.stack([q0 * 1.001, q0 * 0.999])
    print(f"[gpu] train batch vs solves B={B} {n}x{n}", flush=True)
    m = fv.Model(vec(fv, p), fv.make_model_desc(mean=(1.0, 0.0, 0.0), inv_std=(10.0, 10.0, 10.0)))
    tr = fv.Trainer(m, fv.make_train_config(B, n, n, T, dt))
    lb, _ = tr.step(q0, tgt)
    gb = tr.grads.double().cpu().numpy()
    tr.close()
    tr1 = fv.Trainer(m, fv.make_train_config(1, n, n, T, dt))
    gs, ls = np.zeros_like(gb), 0.0
    for b in range(B):
        l1, _ = tr1.step(q0[b:b + 1].contiguous(), tgt[:, b:b + 1].contiguous())
        gs += tr1.grads.double().cpu().numpy() / B
        ls += l1 / B
    tr1.close()
    m.close()
    rel = np.linalg.norm(gb - gs) / np.linalg.norm(gs)
    print(f"[grad] batch loss {lb:.6e} mean {ls:.6e}; rel {rel:.2e}", flush=True)
    assert abs(lb - ls) <= 1e-6 * ls
    assert rel <= 1e-4
    off = 0
    for l in range(5):
        k = p["w"][l].numel() + p["b"][l].numel()
        a, o = gb[off:off + k], gs[off:off + k]
        assert np.linalg.norm(a - o) <= 1e-4 * np.linalg.norm(o), l
        off += k


@pytest.mark.parametrize("direct,blend", [(False, False), (True, False), (False, True)])
def test_adam_reduces_loss(fv, L, direct, blend):
    """A few Adam steps on one batch lower the unrolled loss (learned and
    direct face-state schemes)."""
    n, B, T, dt = 32, 4, 3, 1.0e-3
    p = params(L, 23, scale_last=0.02)
    q0 = torch.tensor(batch(n, B, 60), device="cuda")
    tg = []
    with torch.no_grad():
        qq = torch.tensor(q0.cpu().numpy().astype(np.float64))
        for _ in range(T):
            qq = L.plain_step(qq, dt, 1 / n, 1 / n)
            tg.append(qq.float())
    tgt = torch.stack(tg).cuda()
    m = fv.Model(vec(fv, p))
    tr = fv.Trainer(m, fv.make_train_config(B, n, n, T, dt, lr=3e-4, direct=direct, blend=blend))
    losses = []
    for _ in range(30):
        loss, _ = tr.step(q0, tgt)
        losses.append(loss)
        tr.adam()
    print(f"[adam] direct={direct} blend={blend} loss {losses[0]:.4e} -> {losses[-1]:.4e}", flush=True)
    assert losses[-1] < 0.5 * losses[0]
    tr.close()
    m.close()


def test_coarsen_block_average(fv, L):
    """fv_coarsen against the oracle's block average (pinned by brute force):
    FP32 in, FP64 accumulation, so within FP32 rounding of the result."""
    x = torch.rand(3, 256, 128, device="cuda")
    c = fv.coarsen(x, 32).cpu().double().numpy()
    ref = L.block_average(x.cpu().double(), 32).numpy()
    assert np.abs(c - ref).max() <= 1e-7
