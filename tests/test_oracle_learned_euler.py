"""Pins of the learned Euler oracle (oracle/learned_euler.py): special
coefficients that reduce the learned operator to the separately pinned
classic Euler oracle (first order, MINMOD), the positivity fallback on density
and on pressure, conservation and uniform states for any network, the
redo of an inadmissible step, and autograd gradients against central
differences."""
import numpy as np
import pytest
import torch

from paper_2602_08670_amd import inputs as I

F64 = torch.float64
FLUXES = [("hlle", 0), ("rusanov", 1)]


@pytest.fixture(scope="module")
def E():
    from oracle import learned_euler

    return learned_euler


def _state(n, seed):
    return I.random_smooth_euler(n, seed=seed)


def _onehot(n, own_left=2, own_right=3, scale=None):
    a = torch.zeros(1, 2, 2, 4, 6, n, n, dtype=F64)
    a[:, :, 0, :, own_left] = 1.0
    a[:, :, 1, :, own_right] = 1.0
    if scale is not None:
        a = a * torch.as_tensor(scale, dtype=F64)[None, None, None, :, None, None, None]
    return a


def test_generator_is_admissible_and_periodic():
    for seed in range(8):
        q = _state(32, seed)
        rho = q[0]
        p = 0.4 * (q[3] - 0.5 * (q[1] ** 2 + q[2] ** 2) / rho)
        assert rho.min() >= 0.2 - 1e-12 and p.min() >= 0.2 - 1e-12


@pytest.mark.parametrize("flux,cflux", FLUXES)
def test_one_hot_alpha_equals_first_order_classic(E, orc, flux, cflux):
    """alpha_L = e(cell i), alpha_R = e(cell i+1): the first-order scheme,
    equal to the classic Euler oracle with recon=FIRST (pins the Euler flux
    in both normal frames, the stencil indexing for four variables and the
    divergence)."""
    n = 32
    q0 = _state(n, 3)
    Lq, nfb = E.rhs(torch.tensor(q0)[None], _onehot(n), 1 / n, 1 / n, flux=flux)
    ref = orc.rhs(orc.Config(eqn=orc.EULER, nx=n, ny=n, recon=orc.FIRST, flux=cflux), q0)
    assert int(nfb) == 0
    assert np.abs(Lq[0].numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("flux,cflux", FLUXES)
def test_plain_minmod_equals_classic(E, orc, flux, cflux):
    n = 32
    q0 = _state(n, 4)
    q = torch.tensor(q0)[None]
    Lq, _ = E.rhs(q, None, 1 / n, 1 / n, flux=flux)
    ref = orc.rhs(orc.Config(eqn=orc.EULER, nx=n, ny=n, flux=cflux), q0)
    assert np.abs(Lq[0].numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    qs = E.plain_step(q, 1e-3, 1 / n, 1 / n, flux=flux)
    ref, *_ = orc.run(orc.Config(eqn=orc.EULER, nx=n, ny=n, flux=cflux, dt_fixed=1e-3), q0, None, 1)
    assert np.abs(qs[0].numpy() - ref).max() <= 1e-13 * np.abs(ref).max()


def test_density_fallback_gives_plain_scheme(E):
    """Coefficients that make every learned density negative send every face
    side to its MINMOD state: the operator equals the plain one exactly and
    every face side is counted."""
    n = 16
    q = torch.tensor(_state(n, 2))[None]
    Lq, nfb = E.rhs(q, -_onehot(n), 1 / n, 1 / n)
    ref, _ = E.rhs(q, None, 1 / n, 1 / n)
    assert int(nfb) == 2 * 2 * n * n
    assert torch.equal(Lq, ref)


def test_pressure_fallback_with_positive_density(E):
    """A drift of speed 2 (kinetic energy 2 rho); density and momenta
    reconstructed first order, the energy at 0.05 of the cell's: every
    learned density is positive and every learned pressure negative
    (0.05 E = p / 8 + rho / 10 < 2 rho), so every side falls back; with the
    energy kept none does.  A density-only check would keep these states."""
    n = 16
    q = torch.tensor(_state(n, 5))[None]
    rho = q[:, 0]
    p0 = E.pressure(q)
    q[:, 1], q[:, 2] = 1.6 * rho, 1.2 * rho
    q[:, 3] = p0 / 0.4 + 2.0 * rho
    a = _onehot(n, scale=[1.0, 1.0, 1.0, 0.05])
    QL, QR = E.learned_faces(q, a, axis=0)
    assert bool((QL[:, 0] > 0).all()) and bool((E.pressure(QL) <= 0).all())
    Lq, nfb = E.rhs(q, a, 1 / n, 1 / n)
    ref, _ = E.rhs(q, None, 1 / n, 1 / n)
    assert int(nfb) == 2 * 2 * n * n
    assert torch.equal(Lq, ref)
    _, nfb1 = E.rhs(q, _onehot(n), 1 / n, 1 / n)
    assert int(nfb1) == 0


def test_fallback_is_per_face_side(E):
    """Only the sides whose learned state is inadmissible fall back: negating
    the right-state coefficients of the x axis alone counts n^2 sides, and
    the x-axis fluxes then pair each face's first-order left state with its
    MINMOD right state (checked against those states put in by hand)."""
    n = 16
    q = torch.tensor(_state(n, 6))[None]
    a = _onehot(n)
    a[:, 0, 1] = -a[:, 0, 1]
    Lq, nfb = E.rhs(q, a, 1 / n, 1 / n)
    assert int(nfb) == n * n
    # the same operator from explicit states: x faces (first-order left,
    # MINMOD right), y faces first order
    _, MR = E.minmod_faces(q, 3)
    out = torch.zeros_like(q)
    for axis, dim, QL, QR in ((0, 3, q, MR), (1, 2, q, E.L._shift(q, 1, 2))):
        nm, tm = (1, 2) if axis == 0 else (2, 1)
        F = E.hlle((QL[:, 0], QL[:, nm], QL[:, tm], QL[:, 3]), (QR[:, 0], QR[:, nm], QR[:, tm], QR[:, 3]))
        Fc = [None] * 4
        Fc[0], Fc[nm], Fc[tm], Fc[3] = F
        Fc = torch.stack(Fc, dim=1)
        out = out - (Fc - E.L._shift(Fc, -1, dim)) * n
    assert torch.allclose(Lq, out, rtol=0, atol=1e-12 * float(out.abs().max()))


def test_conservation_and_uniform_state(E):
    """Any network: the periodic divergence sums to zero, and a uniform
    state (any drift) stays uniform (the constraint keeps sum alpha = 1)."""
    n = 16
    p = E.init_params(3, scale_last=0.05)
    q = torch.tensor(_state(n, 7))[None]
    qn, st = E.learned_step(p, q, 2e-3, 1 / n, 1 / n)
    assert not bool(st["redone"][0])
    tot0, tot1 = q.sum(dim=(2, 3)), qn.sum(dim=(2, 3))
    assert torch.allclose(tot0, tot1, rtol=1e-13, atol=0)
    u = torch.zeros(1, 4, n, n, dtype=F64)
    u[:, 0], u[:, 1], u[:, 2], u[:, 3] = 1.2, 0.3, -0.2, 3.0
    un, _ = E.learned_step(p, u, 2e-3, 1 / n, 1 / n)
    assert torch.allclose(un, u, rtol=0, atol=1e-13)


def test_zero_head_is_fromm(E):
    """A zero last layer gives alpha_base (Fromm) for every group."""
    n = 16
    p = E.init_params(1)
    z = E.L.cnn(p, torch.tensor(_state(n, 1))[None])
    assert z.shape == (1, 96, n, n) and float(z.abs().max()) == 0.0
    a = E.coefficients(z, E.L.projector(1))
    assert torch.equal(a[0, 1, 0, 3, :, 5, 7], E.L.ALPHA_BASE[0])
    assert torch.equal(a[0, 0, 1, 2, :, 0, 0], E.L.ALPHA_BASE[1])


def test_stage_two_fallbacks_not_counted_after_a_failed_stage_one(E):
    """When the first stage is already inadmissible the step is redone and
    only the first stage's fallback face sides are counted (the second stage
    runs on a safe copy and its count is dropped); when only the second
    stage fails both stages count."""
    n = 16
    q = torch.tensor(_state(n, 2))[None]
    kin = 0.5 * (q[:, 1] ** 2 + q[:, 2] ** 2) / q[:, 0]
    q[:, 3] = kin + 0.1 * (q[:, 3] - kin)
    P = E.L.projector(1)
    for scale, dt, first_fails in ((100.0, 1e-2, True), (30.0, 1e-2, False)):
        p = E.init_params(2, scale_last=scale)
        L0, f0 = E.rhs(q, E.coefficients(E.L.cnn(p, q), P), 1 / n, 1 / n)
        q1 = q + dt * L0
        assert bool(E.inadmissible_cells(q1)[0]) == first_fails
        _, st = E.learned_step(p, q, dt, 1 / n, 1 / n)
        assert bool(st["redone"][0])
        if first_fails:
            assert st["fallback_faces"] == int(f0)
        else:
            _, f1 = E.rhs(q1, E.coefficients(E.L.cnn(p, q1), P), 1 / n, 1 / n)
            assert st["fallback_faces"] == int(f0) + int(f1) and int(f1) > 0


def test_channel_layout(E):
    """Raw channel ((axis*2 + side)*4 + var)*6 + k feeds the coefficient group
    (axis, side, var): a bias on the channels of one group moves that group's
    coefficients and no other."""
    n = 8
    P = E.L.projector(1)
    for axis, side, var in ((0, 1, 3), (1, 0, 2), (1, 1, 0)):
        z = torch.zeros(1, 96, n, n, dtype=F64)
        c0 = ((axis * 2 + side) * 4 + var) * 6
        z[:, c0:c0 + 6] = torch.tensor([0.3, -0.2, 0.1, 0.4, -0.5, 0.2], dtype=F64)[None, :, None, None]
        a = E.coefficients(z, P)
        base = E.coefficients(torch.zeros_like(z), P)
        moved = (a - base).abs().amax(dim=(0, 4, 5, 6)) > 0  # (axis, side, var)
        assert moved.sum() == 1 and bool(moved[axis, side, var])


def test_inadmissible_step_is_redone_with_the_plain_scheme(E):
    """A low-pressure state, a large random head and a step near the CFL
    limit: the learned stages leave cells with non-positive pressure or
    density, so the step is redone and equals the plain MINMOD Heun step
    exactly (which stays admissible); in a batch the other solve (mild data,
    a small head) is not redone and equals itself stepped alone."""
    n = 16
    qa = torch.tensor(_state(n, 2))[None]
    rho = qa[:, 0]
    kin = 0.5 * (qa[:, 1] ** 2 + qa[:, 2] ** 2) / rho
    qa[:, 3] = kin + 0.1 * (qa[:, 3] - kin)  # pressure scaled down 10x
    p = E.init_params(2, scale_last=10.0)
    qn, st = E.learned_step(p, qa, 1e-2, 1 / n, 1 / n)
    qp = E.plain_step(qa, 1e-2, 1 / n, 1 / n)
    assert bool(st["redone"][0])
    assert not bool(E.inadmissible_cells(qp)[0])
    assert torch.equal(qn, qp)
    qb = torch.tensor(_state(n, 3))[None]
    pb = E.init_params(2, scale_last=0.01)
    qab, stab = E.learned_step(p, torch.cat([qa, qb]), 1e-2, 1 / n, 1 / n)
    assert stab["redone"].tolist()[0] is True
    assert torch.equal(qab[:1], qp)
    qab, stab = E.learned_step(pb, torch.cat([qa, qb]), 2e-3, 1 / n, 1 / n)
    qb1, _ = E.learned_step(pb, qb, 2e-3, 1 / n, 1 / n)
    assert stab["redone"].tolist()[1] is False
    assert torch.allclose(qab[1:], qb1, rtol=0, atol=1e-14)


def test_autograd_matches_central_differences(E):
    """Gradient of the two-step rollout loss with respect to sampled
    parameters and input cells, against central differences of the
    double-precision loss (no bfloat16 rounding, so the loss is smooth
    away from MINMOD and wave-speed switches)."""
    n = 16
    torch.manual_seed(0)
    p = E.init_params(4, scale_last=0.2)
    for l in range(len(p["w"])):
        p["w"][l].requires_grad_(True)
        p["b"][l].requires_grad_(True)
    q0 = torch.tensor(_state(n, 8))[None].requires_grad_(True)
    qs = [q0.detach()]
    for _ in range(2):
        qn, _ = E.plain_step(qs[-1], 2e-3, 1 / n, 1 / n), None
        qs.append(qn.detach() + 1e-3)
    targets = torch.stack(qs[1:], dim=1)
    scale = [0.1, 0.1, 0.1, 0.2]

    def loss_of():
        return E.rollout_loss(p, q0, targets, 2e-3, 1 / n, 1 / n, scale, round_bf16=False)

    loss = loss_of()
    gw = torch.autograd.grad(loss, [p["w"][0], p["w"][4], p["b"][4], q0])
    checks = [(p["w"][0], gw[0], (3, 2, 1, 0)), (p["w"][4], gw[1], (50, 7, 2, 1)),
              (p["b"][4], gw[2], (70,)), (q0, gw[3], (0, 3, 5, 9)), (q0, gw[3], (0, 0, 11, 2))]
    h = 1e-6
    for t, g, idx in checks:
        with torch.no_grad():
            old = t[idx].item()
            t[idx] = old + h
            lp = loss_of().item()
            t[idx] = old - h
            lm = loss_of().item()
            t[idx] = old
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[idx].item()) <= 1e-5 * max(abs(fd), 1e-8) + 1e-10, (idx, fd, g[idx].item())
