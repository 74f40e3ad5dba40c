"""Pins of the learned-path oracle (oracle/learned.py): projection invariants,
exactness on linear data, special cases that reduce to the (separately
pinned) classic oracle, brute-force convolution, bfloat16 rounding, the
fallback wiring, and autograd gradients against central finite differences."""
import itertools
import math

import numpy as np
import pytest
import torch

from paper_2602_08670_amd import inputs as I

F64 = torch.float64


@pytest.fixture(scope="module")
def L():
    from oracle import learned

    return learned


def test_projection_invariants(L):
    A = L.moment_matrix(1)
    P = L.projector(1)
    assert torch.allclose(P @ P, P, atol=1e-15)
    assert torch.allclose(P, P.T, atol=1e-15)
    assert int(torch.linalg.matrix_rank(P)) == 4
    assert torch.abs(A @ P).max() < 1e-15
    e0 = torch.tensor([1.0, 0.0], dtype=F64)
    for side in range(2):
        assert torch.abs(A @ L.ALPHA_BASE[side] - e0).max() < 1e-15
    g = torch.Generator().manual_seed(0)
    z = torch.randn(4, 72, 5, 6, generator=g, dtype=F64) * 3
    a = L.coefficients(z, P)
    res = torch.einsum("pk,baswkhx->baswphx", A, a) - e0[None, None, None, None, :, None, None]
    assert res.abs().max() < 1e-14
    a0 = L.coefficients(torch.zeros(1, 72, 2, 2, dtype=F64), P)
    assert torch.equal(a0[0, 1, 0, 2, :, 1, 1], L.ALPHA_BASE[0])


def test_moment_matrix_matches_cell_average_integrals(L):
    """Row 1 is the cell centre (cell average of x); row 2 adds 1/12."""
    A = L.moment_matrix(2)
    assert torch.allclose(A[0], torch.ones(6, dtype=F64))
    assert torch.allclose(A[1], L.OFFSETS)
    assert torch.allclose(A[2], L.OFFSETS ** 2 + 1.0 / 12.0)


def test_constrained_faces_exact_on_linear_data(L):
    """Any alpha = alpha_base + P z reproduces the face value of a linear field
    from its cell averages (interior faces, away from the periodic seam)."""
    n = 24
    x = torch.arange(n, dtype=F64)  # cell centres in cell units
    q = torch.zeros(1, 3, n, n, dtype=F64)
    q[0, 0] = 2.0 + 0.03 * x[None, :] - 0.01 * x[:, None]
    q[0, 1] = 0.5 - 0.02 * x[None, :]
    q[0, 2] = 0.1 + 0.04 * x[:, None]
    g = torch.Generator().manual_seed(1)
    a = L.coefficients(torch.randn(1, 72, n, n, generator=g, dtype=F64), L.projector(1))
    QL, QR = L.learned_faces(q, a, axis=0)
    face = lambda f: f  # noqa: E731
    for v, (c0, cx, cy) in enumerate([(2.0, 0.03, -0.01), (0.5, -0.02, 0.0), (0.1, 0.0, 0.04)]):
        exact = c0 + cx * (x[None, :] + 0.5) + cy * x[:, None]  # value at face i+1/2
        sl = (slice(None), slice(3, n - 3))
        assert torch.abs(QL[0, v][sl] - exact[sl]).max() < 1e-12
        assert torch.abs(QR[0, v][sl] - exact[sl]).max() < 1e-12
    QL, QR = L.learned_faces(q, a, axis=1)
    exact = 2.0 + 0.03 * x[None, :] - 0.01 * (x[:, None] + 0.5)
    assert torch.abs(QL[0, 0][3:n - 3] - exact[3:n - 3]).max() < 1e-12


@pytest.mark.parametrize("flux,cflux", [("hlle", 0), ("rusanov", 1)])
def test_one_hot_alpha_equals_first_order_classic(L, orc, flux, cflux):
    """alpha_L = e(cell i), alpha_R = e(cell i+1) is the first-order scheme:
    the learned operator equals the classic oracle with recon=FIRST."""
    q0, _ = I.swe_bathy(32, seed=3)
    q0[1] = 0.05 * np.sin(2 * np.pi * np.arange(32) / 32)[None, :]
    q0[2] = -0.04 * np.cos(2 * np.pi * np.arange(32) / 32)[:, None]
    q = torch.tensor(q0)[None]
    a = torch.zeros(1, 2, 2, 3, 6, 32, 32, dtype=F64)
    a[:, :, 0, :, 2] = 1.0
    a[:, :, 1, :, 3] = 1.0
    Lq, nfb = L.rhs(q, a, 1 / 32, 1 / 32, flux=flux)
    ref = orc.rhs(orc.Config(nx=32, ny=32, recon=orc.FIRST, flux=cflux), q0)
    assert nfb == 0
    assert np.abs(Lq[0].numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("flux,cflux", [("hlle", 0), ("rusanov", 1)])
def test_plain_minmod_equals_classic(L, orc, flux, cflux):
    q0, _ = I.swe_bathy(32, seed=4)
    q0[1] = 0.05 * np.sin(2 * np.pi * np.arange(32) / 32)[None, :]
    q = torch.tensor(q0)[None]
    Lq, _ = L.rhs(q, None, 1 / 32, 1 / 32, flux=flux)
    ref = orc.rhs(orc.Config(nx=32, ny=32, flux=cflux), q0)
    assert np.abs(Lq[0].numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    qs = L.plain_step(q, 1e-3, 1 / 32, 1 / 32, flux=flux)
    ref, *_ = orc.run(orc.Config(nx=32, ny=32, flux=cflux, dt_fixed=1e-3), q0, None, 1)
    assert np.abs(qs[0].numpy() - ref).max() <= 1e-13


def test_all_faces_fall_back_gives_plain_scheme(L):
    """Coefficients that make every learned depth negative send every face
    side to the MINMOD state: the operator equals the plain one exactly."""
    q0 = I.random_smooth_swe(16, seed=2)
    q = torch.tensor(q0)[None]
    a = torch.zeros(1, 2, 2, 3, 6, 16, 16, dtype=F64)
    a[:, :, :, :, 2] = -1.0
    Lq, nfb = L.rhs(q, a, 1 / 16, 1 / 16)
    ref, _ = L.rhs(q, None, 1 / 16, 1 / 16)
    assert nfb == 2 * 2 * 16 * 16
    assert torch.equal(Lq, ref)


def test_conv_bruteforce_and_library(L):
    g = torch.Generator().manual_seed(5)
    x = torch.randn(2, 2, 5, 4, generator=g, dtype=F64)
    w = torch.randn(3, 2, 3, 3, generator=g, dtype=F64)
    b = torch.randn(3, generator=g, dtype=F64)
    out = L.conv3x3_periodic(x, w, b)
    ref = torch.zeros(2, 3, 5, 4, dtype=F64)
    for n, o, y, xx, c, ky, kx in itertools.product(range(2), range(3), range(5), range(4), range(2), range(3),
                                                     range(3)):
        ref[n, o, y, xx] += w[o, c, ky, kx] * x[n, c, (y + ky - 1) % 5, (xx + kx - 1) % 4]
    ref += b[None, :, None, None]
    assert torch.allclose(out, ref, atol=1e-13)
    lib = torch.nn.functional.conv2d(torch.nn.functional.pad(x, (1, 1, 1, 1), mode="circular"), w, b)
    assert torch.allclose(out, lib, atol=1e-13)


def test_bf16_round_to_nearest_even(L):
    v = torch.tensor([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20, -3.0 - 2.0 ** -7],
                     dtype=F64)
    r = L.bf16(v, ste=False)
    assert r.tolist() == [1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -3.0]


def test_zero_last_layer_gives_fromm(L):
    """With z = 0 every face uses Fromm's stencils."""
    p = L.init_params(0, hidden=8, layers=[(3, 8), (8, 8), (8, 72)])
    q = torch.tensor(I.random_smooth_swe(12, seed=1))[None]
    z = L.cnn(p, q)
    assert torch.equal(z, torch.zeros_like(z))


def test_rollout_loss_zero_on_own_rollout(L):
    p = L.init_params(3, hidden=8, scale_last=0.05, layers=[(3, 8), (8, 8), (8, 72)])
    q = torch.tensor(I.random_smooth_swe(16, seed=6))[None]
    dt = 5e-4
    tg = []
    qq = q
    for _ in range(3):
        qq, _ = L.learned_step(p, qq, dt, 1 / 16, 1 / 16)
        tg.append(qq)
    tg = torch.stack(tg, 1).detach()
    assert float(L.rollout_loss(p, q, tg, dt, 1 / 16, 1 / 16, [0.1, 0.1, 0.1])) < 1e-28


@pytest.mark.slow
@pytest.mark.parametrize("direct,blend", [(False, False), (True, False), (False, True)])
def test_autograd_matches_central_differences(L, direct, blend):
    """d loss / d theta and d loss / d q0 from automatic differentiation agree
    with central finite differences (h = 1e-6) on a small network and grid
    (bfloat16 rounding off so the loss is smooth), for the learned, the
    direct face-state and the flux-limiter-blended rollouts.  The blend is
    trained with the limiter frozen: its gradient is that of the loss with
    every phi held at the value of the unperturbed rollout, so the finite
    differences replay the recorded phis."""
    p = L.init_params(4, hidden=4, scale_last=0.2, layers=[(3, 4), (4, 4), (4, 72)])
    p["b"][0] = torch.full((4,), 0.3, dtype=F64)
    q0 = torch.tensor(I.random_smooth_swe(8, seed=7, humps=2))[None]
    q0[:, 1] = 0.02
    dt = 2e-3
    with torch.no_grad():
        tg = []
        qq = q0 + 0.001
        for _ in range(2):
            qq = L.plain_step(qq, dt, 1 / 8, 1 / 8)
            tg.append(qq)
        tg = torch.stack(tg, 1)
    leaves = p["w"] + p["b"]
    for t in leaves:
        t.requires_grad_(True)
    qv = q0.clone().requires_grad_(True)
    tape = {"frozen": True, "tape": []} if blend else None
    loss = L.rollout_loss(p, qv, tg, dt, 1 / 8, 1 / 8, [0.1, 0.05, 0.05], round_bf16=False, direct=direct, blend=blend,
                          limiter=tape)
    grads = torch.autograd.grad(loss, leaves + [qv])
    g = torch.Generator().manual_seed(11)

    def central(t, flat, k, h):
        def ev():
            rep = {"replay": True, "tape": tape["tape"], "pos": 0} if blend else None
            return L.rollout_loss(p, qv.detach() if t is not qv else qv, tg, dt, 1 / 8, 1 / 8, [0.1, 0.05, 0.05],
                                  round_bf16=False, direct=direct, blend=blend, limiter=rep)

        with torch.no_grad():
            old = flat[k].item()
            flat[k] = old + h
            lp = ev()
            flat[k] = old - h
            lm = ev()
            flat[k] = old
        return (lp - lm).item() / (2 * h)

    h = 1e-6
    checked = 0
    for t, gr in zip(leaves + [qv], grads):
        flat = t.detach().view(-1)
        for _ in range(3):
            k = int(torch.randint(0, flat.numel(), (1,), generator=g))
            fd = central(t, flat, k, h)
            an = gr.view(-1)[k].item()
            assert abs(fd - an) <= 1e-6 * abs(fd) + 1e-10, (fd, an)
            checked += 1
    assert checked == 3 * len(leaves + [qv])
    if blend:
        # the frozen-limiter gradient differs from the full derivative
        # (through phi) of the same loss: the limiter's share is dropped
        leaves2 = [x.detach().clone().requires_grad_(True) for x in leaves]
        p2 = dict(p, w=leaves2[:len(p["w"])], b=leaves2[len(p["w"]):])
        full = torch.autograd.grad(L.rollout_loss(p2, qv, tg, dt, 1 / 8, 1 / 8, [0.1, 0.05, 0.05], round_bf16=False,
                                                  blend=True, limiter={}), [qv])[0]
        assert float((full - grads[-1]).abs().max()) > 1e-3 * float(grads[-1].abs().max())


# ---- direct face states (section 5.3) --------------------------------------

def _params_head(L, seed, head_bias=None, scale_last=0.0):
    p = L.init_params(seed, scale_last=scale_last)
    if head_bias is not None:
        p["b"][-1] = p["b"][-1].clone()
        p["b"][-1][:len(head_bias)] = torch.tensor(head_bias, dtype=F64)
    return p


@pytest.mark.parametrize("flux,cflux", [("hlle", 0), ("rusanov", 1)])
def test_direct_zero_head_is_first_order_classic(L, orc, flux, cflux):
    """A zero head leaves every face state at its cell average: the direct
    scheme is then the first-order scheme of the classic oracle (recon=FIRST),
    operator and Heun step."""
    q0, _ = I.swe_bathy(32, seed=5)
    q0[1] = 0.05 * np.sin(2 * np.pi * np.arange(32) / 32)[None, :]
    q0[2] = -0.04 * np.cos(2 * np.pi * np.arange(32) / 32)[:, None]
    q = torch.tensor(q0)[None]
    p = _params_head(L, 1)
    Lq, nfb = L.direct_rhs(p, q, 1 / 32, 1 / 32, flux=flux)
    ref = orc.rhs(orc.Config(nx=32, ny=32, recon=orc.FIRST, flux=cflux), q0)
    assert int(nfb.sum()) == 0
    assert np.abs(Lq[0].numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    qs, st = L.direct_step(p, q, 1e-3, 1 / 32, 1 / 32, flux=flux)
    ref, *_ = orc.run(orc.Config(nx=32, ny=32, recon=orc.FIRST, flux=cflux, dt_fixed=1e-3), q0, None, 1)
    assert np.abs(qs[0].numpy() - ref).max() <= 1e-13
    assert not bool(st["redone"].any())


def test_direct_face_pairing_reproduces_minmod(L, monkeypatch):
    """With a head that outputs the MINMOD face states (depth: the ratio
    (q_h +- s_h/2) / q_h through the inverse of the shifted Softplus;
    momenta: +-s/2 in normalised units; + on the right and top sides, - on
    the left and bottom), cell i's right state and cell i+1's left state are
    MINMOD's two states of face i+1/2 on both axes: the direct operator
    equals the plain MINMOD one.  Pins which cell's side meets which, the
    depth's scaling by its own cell, and the de-normalisation of the momenta."""
    q0 = I.random_smooth_swe(24, seed=6)
    q0[1] = 0.03 * np.sin(2 * np.pi * np.arange(24) / 24)[None, :]
    q0[2] = 0.02 * np.cos(2 * np.pi * np.arange(24) / 24)[:, None]
    q = torch.tensor(q0)[None]
    p = _params_head(L, 2)
    inv = p["inv_std"][None, :, None, None]

    def slope(x, dim):
        return L._minmod(x - L._shift(x, -1, dim), L._shift(x, 1, dim) - x)

    def head(x, s, sign):
        ratio = (x[:, :1] + sign * 0.5 * s[:, :1]) / x[:, :1]
        zh = (torch.log(torch.expm1(ratio)) - L.SOFTPLUS_SHIFT) * inv[:, :1]
        return torch.cat([zh, sign * 0.5 * s[:, 1:] * inv[:, 1:]], dim=1)

    def fake_cnn(params, x, round_bf16=True, shadow_f32=False):
        sx, sy = slope(x, 3), slope(x, 2)
        z = torch.zeros(x.shape[0], 72, x.shape[2], x.shape[3], dtype=F64)
        z[:, 0:3] = head(x, sx, -1.0)   # left
        z[:, 3:6] = head(x, sx, 1.0)    # right
        z[:, 6:9] = head(x, sy, -1.0)   # bottom
        z[:, 9:12] = head(x, sy, 1.0)   # top
        return z

    monkeypatch.setattr(L, "cnn", fake_cnn)
    Lq, nfb = L.direct_rhs(p, q, 1 / 24, 1 / 24)
    ref, _ = L.rhs(q, None, 1 / 24, 1 / 24)
    assert int(nfb.sum()) == 0
    assert torch.abs(Lq - ref).max() <= 1e-12 * torch.abs(ref).max()


def test_softplus_values(L):
    """softplus(0) = ln 2, softplus(c) = 1 for the shift c = ln(e - 1), the
    asymptotes x (large x) and e^x (very negative x), and no overflow."""
    x = torch.tensor([0.0, L.SOFTPLUS_SHIFT, 800.0, -40.0, -700.0], dtype=F64)
    y = L.softplus(x)
    assert abs(float(y[0]) - math.log(2.0)) <= 1e-16
    assert abs(float(y[1]) - 1.0) <= 2e-16
    assert float(y[2]) == 800.0
    assert abs(float(y[3]) / math.exp(-40.0) - 1.0) <= 1e-15
    assert 0.0 < float(y[4]) and abs(float(y[4]) / math.exp(-700.0) - 1.0) <= 1e-12


def test_direct_depths_positive_for_any_head(L):
    """The Softplus depth head of section 2.5.3 (third approach): a strongly
    negative height head (bias -300 in normalised units, -30 de-normalised)
    still gives positive face depths, so no face side falls back, and each
    depth is its cell's depth times e^(-30 + c) to first order; a random large
    head gives positive depths everywhere too."""
    q0 = I.random_smooth_swe(16, seed=10)
    q = torch.tensor(q0)[None]
    hb = [0.0] * 12
    for f in range(4):
        hb[3 * f] = -300.0
    p = _params_head(L, 11, head_bias=hb)
    faces = L.direct_faces(p, q)
    for Qf in faces:
        assert bool((Qf[:, 0] > 0).all())
        assert torch.allclose(Qf[:, 0], q[:, 0] * math.exp(-30.0 + L.SOFTPLUS_SHIFT), rtol=1e-12, atol=0)
        assert torch.equal(Qf[:, 1:], q[:, 1:])
    _, nfb = L.direct_rhs(p, q, 1 / 16, 1 / 16)
    assert int(nfb.sum()) == 0
    p = _params_head(L, 12, scale_last=50.0)
    for Qf in L.direct_faces(p, q):
        assert bool((Qf[:, 0] > 0).all())


def test_direct_step_conserves_and_keeps_uniform_states(L):
    """Any head: the periodic direct step conserves mass and momentum (each
    face's flux is shared by its two cells), and a uniform state stays
    unchanged (the network's output is then uniform, every face flux equal)."""
    q0 = I.random_smooth_swe(32, seed=7)
    q0[1] = 0.05 * np.sin(2 * np.pi * np.arange(32) / 32)[None, :]
    q = torch.tensor(q0)[None]
    p = _params_head(L, 3, scale_last=0.3)
    q1, st = L.direct_step(p, q, 1e-3, 1 / 32, 1 / 32)
    assert not bool(st["redone"].any())
    assert not torch.equal(q1, q)
    for v in range(3):
        a, b = float(q[0, v].sum()), float(q1[0, v].sum())
        assert abs(a - b) <= 1e-12 * float(q[0, 0].abs().sum()), v
    u = torch.zeros(1, 3, 16, 16, dtype=F64)
    u[:, 0], u[:, 1], u[:, 2] = 1.2, 0.1, -0.05
    Lu, _ = L.direct_rhs(p, u, 1 / 16, 1 / 16)
    assert torch.equal(Lu, torch.zeros_like(Lu))


def test_direct_all_faces_fall_back_gives_plain_scheme(L):
    """A height head so negative that the Softplus underflows to zero depth
    sends every side to its MINMOD state: the operator equals the plain one
    exactly, 4 sides per cell counted."""
    q0 = I.random_smooth_swe(16, seed=8)
    q = torch.tensor(q0)[None]
    hb = [0.0] * 12
    for f in range(4):
        hb[3 * f] = -1e4
    p = _params_head(L, 4, head_bias=hb)
    Lq, nfb = L.direct_rhs(p, q, 1 / 16, 1 / 16)
    ref, _ = L.rhs(q, None, 1 / 16, 1 / 16)
    assert int(nfb.sum()) == 2 * 2 * 16 * 16
    assert torch.equal(Lq, ref)


# ---- flux-limiter blend (section 2.5.3, second approach) --------------------

def test_limiter_minmod_values(L):
    """The MINMOD flux limiter phi(r) = max(0, min(1, r)) at textbook points:
    0 for r <= 0, r on (0, 1), 1 from r = 1 on; and the undefined ratio
    (q_{i+1} = q_i) takes the low-resolution flux."""
    a = torch.tensor([2.0, 1.0, -1.0, 1.0, 0.0, -3.0, -1.0, 0.0, 3.0], dtype=F64)
    b = torch.tensor([1.0, 2.0, 1.0, 0.0, 0.0, -2.0, -4.0, 5.0, -0.5], dtype=F64)
    want = torch.tensor([1.0, 0.5, 0.0, 0.0, 0.0, 1.0, 0.25, 0.0, 0.0], dtype=F64)
    assert torch.equal(L.limiter_minmod(a, b), want)


def _x_profile(hx, hux, hv, n):
    q = torch.zeros(1, 3, n, n, dtype=F64)
    q[0, 0] = torch.as_tensor(hx, dtype=F64)[None, :]
    q[0, 1] = torch.as_tensor(hux, dtype=F64)[None, :]
    q[0, 2] = hv
    return q


def _alpha(L, p, q):
    return L.coefficients(L.cnn(p, q), L.projector(1))


@pytest.mark.parametrize("flux,cflux", [("hlle", 0), ("rusanov", 1)])
def test_blend_at_extrema_is_first_order_classic(L, orc, flux, cflux):
    """Every cell an extremum along x (alternating values) and no variation
    along y: phi = 0 at every face, so the blended operator is the
    first-order scheme of the classic oracle whatever the network, while the
    unblended learned operator is not."""
    n = 32
    sgn = (-1.0) ** np.arange(n)
    q = _x_profile(1.0 + 0.1 * sgn, 0.05 + 0.02 * sgn, 0.01, n)
    p = _params_head(L, 5, scale_last=0.3)
    a = _alpha(L, p, q)
    Lb, _ = L.rhs(q, a, 1 / n, 1 / n, flux=flux, blend=True)
    Lh, _ = L.rhs(q, a, 1 / n, 1 / n, flux=flux)
    ref = orc.rhs(orc.Config(nx=n, ny=n, recon=orc.FIRST, flux=cflux), q[0].numpy())
    assert np.abs(Lb[0].numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(Lh[0].numpy() - ref).max() > 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("flux,cflux", [("hlle", 0), ("rusanov", 1)])
def test_blend_half_limiter_on_geometric_differences(L, orc, flux, cflux):
    """Successive differences doubling along x (q_{i+1} - q_i = 2^i / 4096 for
    i = 0..11): r = 1/2 at cells 1..11, so both faces of cells 2..11 take
    phi = 1/2 for h and hu and the blended operator there is the mean of the
    first-order and the learned ones; hv is uniform (phi = 0: first order).
    Pins the ratio's orientation (its inverse gives phi = 1)."""
    n = 32
    i = np.arange(n)
    h = np.where(i <= 12, 1.0 + (2.0 ** np.minimum(i, 12) - 1) / 4096, 0.0)
    h[13:] = h[12] - (h[12] - 1.0) * (i[13:] - 12) / 20
    hu = (h - 1.0) / 8 + 1 / 64
    q = _x_profile(h, hu, 1 / 32, n)
    p = _params_head(L, 6, scale_last=0.3)
    a = _alpha(L, p, q)
    Lb, _ = L.rhs(q, a, 1 / n, 1 / n, flux=flux, blend=True)
    Lh, _ = L.rhs(q, a, 1 / n, 1 / n, flux=flux)
    Ll = torch.tensor(orc.rhs(orc.Config(nx=n, ny=n, recon=orc.FIRST, flux=cflux), q[0].numpy()))[None]
    sc = float(Lh.abs().max())
    cells = slice(2, 12)
    assert torch.abs(Lb[:, :2, :, cells] - 0.5 * (Ll + Lh)[:, :2, :, cells]).max() <= 1e-12 * sc
    assert torch.abs(Lb[:, 2, :, cells] - Ll[:, 2, :, cells]).max() <= 1e-12 * sc
    assert torch.abs(Lh - Ll)[:, :2, :, cells].max() > 1e-4 * sc


@pytest.mark.parametrize("flux,cflux", [("hlle", 0), ("rusanov", 1)])
def test_blend_limiter_taken_at_the_low_index_cell(L, orc, flux, cflux):
    """A flat state that turns into a linear ramp at cell 8 (q_8 = q_7, then
    equal differences): cell 8's faces take phi(r_7) and phi(r_8), both 0,
    so its blended operator is first order; cells 10..30 have r = 1 at both
    faces and take the learned operator.  Taking face i+1/2's ratio at cell
    i+1 instead would give cell 8 phi = 1 on its right face."""
    n = 32
    i = np.arange(n)
    h = 1.0 + np.maximum(i - 8, 0) / 64
    q = _x_profile(h, (h - 1.0) / 2 + 1 / 32, 1 / 64, n)
    p = _params_head(L, 7, scale_last=0.3)
    a = _alpha(L, p, q)
    Lb, _ = L.rhs(q, a, 1 / n, 1 / n, flux=flux, blend=True)
    Lh, _ = L.rhs(q, a, 1 / n, 1 / n, flux=flux)
    Ll = torch.tensor(orc.rhs(orc.Config(nx=n, ny=n, recon=orc.FIRST, flux=cflux), q[0].numpy()))[None]
    sc = float(Lh.abs().max())
    assert torch.abs(Lb[..., 8] - Ll[..., 8]).max() <= 1e-12 * sc
    assert torch.abs(Lh[..., 8] - Ll[..., 8]).max() > 1e-4 * sc
    assert torch.abs(Lb[:, :2, :, 10:31] - Lh[:, :2, :, 10:31]).max() <= 1e-12 * sc


def test_blend_step_conserves_and_keeps_uniform_states(L):
    """The blended flux is still one flux per face: the periodic step
    conserves mass and momentum; a uniform state stays unchanged."""
    q0 = I.random_smooth_swe(32, seed=9)
    q0[1] = 0.05 * np.sin(2 * np.pi * np.arange(32) / 32)[None, :]
    q = torch.tensor(q0)[None]
    p = _params_head(L, 8, scale_last=0.3)
    q1, st = L.learned_step(p, q, 1e-3, 1 / 32, 1 / 32, blend=True)
    q1u, _ = L.learned_step(p, q, 1e-3, 1 / 32, 1 / 32)
    assert not bool(st["redone"].any())
    assert torch.abs(q1 - q1u).max() > 1e-9
    for v in range(3):
        assert abs(float(q[0, v].sum()) - float(q1[0, v].sum())) <= 1e-12 * float(q[0, 0].abs().sum()), v
    u = torch.zeros(1, 3, 16, 16, dtype=F64)
    u[:, 0], u[:, 1], u[:, 2] = 1.2, 0.1, -0.05
    Lu, _ = L.rhs(u, _alpha(L, p, u), 1 / 16, 1 / 16, blend=True)
    assert torch.abs(Lu).max() <= 1e-13


# ---- admissibility redo (section 5.2: a negative depth gives NaN) ----------

REDO_SCHEMES = ["learned", "direct", "blend"]


def _step(L, scheme, p, q, dt, n):
    if scheme == "direct":
        return L.direct_step(p, q, dt, 1 / n, 1 / n)
    return L.learned_step(p, q, dt, 1 / n, 1 / n, blend=scheme == "blend")


@pytest.mark.parametrize("scheme", REDO_SCHEMES)
def test_inadmissible_step_is_redone_with_the_plain_scheme(L, scheme):
    """A shallow state (depth about 0.1) and a large random head: the learned
    stages leave cells with non-positive depth, so the whole step is redone
    and its result is exactly the plain MINMOD Heun step of the same state;
    the plain step stays admissible."""
    n = 32
    q = torch.tensor(I.random_smooth_swe(n, seed=2))[None]
    q[:, 0] *= 0.1
    p = L.init_params(2, scale_last=10.0)
    qn, st = _step(L, scheme, p, q, 1e-3, n)
    qp = L.plain_step(q, 1e-3, 1 / n, 1 / n)
    assert bool(st["redone"][0])
    assert bool((qp[:, 0] > 0).all())
    assert torch.equal(qn, qp)


@pytest.mark.parametrize("scheme", REDO_SCHEMES)
def test_redo_is_per_solve(L, scheme):
    """In a batch, only the solve whose step is inadmissible is redone; the
    other (a weak hump at depth 1) keeps its learned result, equal to that
    solve stepped alone."""
    n = 32
    qa = torch.tensor(I.random_smooth_swe(n, seed=2))[None]
    qa[:, 0] *= 0.1
    qb = torch.tensor(I.random_smooth_swe(n, seed=3))[None]
    qb[:, 0] = 1.0 + 0.01 * (qb[:, 0] - 1.0)
    p = L.init_params(2, scale_last=10.0)
    qab, st = _step(L, scheme, p, torch.cat([qa, qb]), 1e-3, n)
    assert st["redone"].tolist() == [True, False]
    assert torch.equal(qab[:1], L.plain_step(qa, 1e-3, 1 / n, 1 / n))
    qb1, stb = _step(L, scheme, p, qb, 1e-3, n)
    assert not bool(stb["redone"][0])
    assert torch.allclose(qab[1:], qb1, rtol=0, atol=1e-14)


def test_block_average_brute_force(L):
    """Coarse cell (I, J) is the plain mean of the fine cells (f I + a, f J + c),
    a, c < f, summed by explicit loops."""
    g = torch.Generator().manual_seed(3)
    x = torch.rand(2, 3, 12, 8, generator=g, dtype=F64)
    f = 4
    c = L.block_average(x, f)
    assert c.shape == (2, 3, 3, 2)
    for b in range(2):
        for v in range(3):
            for I_ in range(3):
                for J in range(2):
                    acc = 0.0
                    for a in range(f):
                        for d in range(f):
                            acc += float(x[b, v, f * I_ + a, f * J + d])
                    assert abs(float(c[b, v, I_, J]) - acc / (f * f)) <= 1e-15
    # a field linear in x and y keeps its value at the coarse cell centres
    yy, xx = torch.meshgrid(torch.arange(16, dtype=F64) + 0.5, torch.arange(16, dtype=F64) + 0.5, indexing="ij")
    lin = (0.3 + 0.02 * xx - 0.05 * yy)[None]
    cy, cx = torch.meshgrid(4 * torch.arange(4, dtype=F64) + 2, 4 * torch.arange(4, dtype=F64) + 2, indexing="ij")
    assert torch.allclose(L.block_average(lin, 4)[0], 0.3 + 0.02 * cx - 0.05 * cy, atol=1e-14)
