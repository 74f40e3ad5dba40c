"""Oracle of the learned-coefficient step for the 2D Euler equations.  TEST
INFRASTRUCTURE ONLY: used by tests/ and nothing in the product path.

Thesis "A Machine Learning accelerated geophysical fluid solver": section 6.2
names a data-driven discretisation of the Euler equations, with positivity of
density and energy, as future work.  This module carries the planar
shallow-water construction of oracle/learned.py over to the Euler system
(section 4.2: q = (rho, rho u, rho v, E), p = (gamma - 1)(E - |m|^2 / 2 rho)):

  - network: the same five 3x3 convolutions with ReLU and bfloat16 rounding,
    4 -> 32 -> 32 -> 32 -> 32 -> 96: per cell and axis two coefficient
    vectors (left and right state of the cell's high face) for each of the
    four conserved variables, channel ((axis*2 + side)*4 + var)*6 + k;
  - constraint (section 2.5.3, fourth approach): alpha = alpha_base + P z per
    group of six, exact for cell averages of linear data (oracle/learned.py);
  - numerical fluxes (eq 2.12, 2.16) of the Euler system in the face's normal
    frame, Einfeldt wave speeds from Roe averages clamped with zero;
  - positivity (the constraint of section 6.2): a learned face state whose
    density or pressure is not positive (or not finite) takes the MINMOD
    state of that side, which itself is the cell average when MINMOD gives
    an inadmissible state; a stage leaving a cell with rho <= 0 or p <= 0
    makes the solve redo the whole step with the plain MINMOD scheme;
  - Heun stages (eq 2.19) at a fixed step, periodic domain.
Gradients of rollout_loss come from automatic differentiation of these
double-precision operations (bfloat16 rounding passes gradients straight
through).
"""
from __future__ import annotations

import torch

from . import learned as L

F64 = torch.float64
NV = 4
LAYERS = [(4, 32), (32, 32), (32, 32), (32, 32), (32, 96)]
GAMMA = 1.4


def init_params(seed: int, scale_last: float = 0.0) -> dict:
    """Seeded parameters (He-scaled, bfloat16-valued weights, zero biases,
    last layer scaled by scale_last) with the normalisation of the smooth
    Euler workload (mean rho = 1, E = 2.5; unit-ish spreads)."""
    p = L.init_params(seed, scale_last=scale_last, layers=LAYERS)
    p["mean"] = torch.tensor([1.0, 0.0, 0.0, 2.5], dtype=F64)
    p["inv_std"] = torch.tensor([8.0, 4.0, 4.0, 2.0], dtype=F64)
    return p


def coefficients(z: torch.Tensor, P: torch.Tensor) -> torch.Tensor:
    """z (B, 96, H, W) -> alpha (B, axis, side, var, k, H, W) = alpha_base + P z."""
    B, C, H, W = z.shape
    zz = z.reshape(B, 2, 2, NV, 6, H, W)
    return L.ALPHA_BASE[None, None, :, None, :, None, None] + torch.einsum("kj,baswjhx->baswkhx", P, zz)


def pressure(Q: torch.Tensor, gamma: float = GAMMA) -> torch.Tensor:
    """p of states Q (B, 4, ...) (eq 2.4 in two dimensions)."""
    return (gamma - 1.0) * (Q[:, 3] - 0.5 * (Q[:, 1] ** 2 + Q[:, 2] ** 2) / Q[:, 0])


def admissible(Q: torch.Tensor, gamma: float = GAMMA) -> torch.Tensor:
    """rho > 0 and p > 0 (false for non-finite values), shape (B, 1, ...)."""
    with torch.no_grad():
        ok = (Q[:, 0] > 0) & (pressure(Q, gamma) > 0) & torch.isfinite(Q).all(dim=1)
    return ok[:, None]


def minmod_faces(q: torch.Tensor, dim: int, gamma: float = GAMMA):
    """MINMOD states of face i+1/2 (eq 2.18), each side replaced by its cell
    average when inadmissible."""
    qm1, q0, q1, q2 = L._shift(q, -1, dim), q, L._shift(q, 1, dim), L._shift(q, 2, dim)
    QL = q0 + 0.5 * L._minmod(q0 - qm1, q1 - q0)
    QR = q1 - 0.5 * L._minmod(q1 - q0, q2 - q1)
    QL = torch.where(admissible(QL, gamma), QL, q0)
    QR = torch.where(admissible(QR, gamma), QR, q1)
    return QL, QR


def learned_faces(q: torch.Tensor, alpha: torch.Tensor, axis: int):
    """Face states of face i+1/2 owned by cell i: Q_side,v = sum_k alpha[axis,
    side, v, k] q_v(i - 2 + k)."""
    dim = 3 if axis == 0 else 2
    st = torch.stack([L._shift(q, k - 2, dim) for k in range(6)], dim=2)  # (B, 4, 6, H, W)
    return (alpha[:, axis, 0] * st).sum(dim=2), (alpha[:, axis, 1] * st).sum(dim=2)


def _phys(r, mn, mt, E, gamma):
    u = mn / r
    p = (gamma - 1.0) * (E - 0.5 * (mn * mn + mt * mt) / r)
    return (mn, mn * u + p, mt * u, u * (E + p)), u, p


def hlle(sl, sr, gamma: float = GAMMA):
    """HLLE flux (eq 2.16) of normal-frame Euler states (rho, m_n, m_t, E),
    Einfeldt speeds: s_L = min(u_L - c_L, u~ - c~, 0), s_R = max(u_R + c_R,
    u~ + c~, 0) with sqrt(rho)-weighted Roe averages of u, v and H."""
    fl, ul, pl = _phys(*sl, gamma)
    fr, ur, pr = _phys(*sr, gamma)
    rl, rr = sl[0], sr[0]
    cl, cr = torch.sqrt(gamma * pl / rl), torch.sqrt(gamma * pr / rr)
    wl, wr = torch.sqrt(rl), torch.sqrt(rr)
    ua = (wl * ul + wr * ur) / (wl + wr)
    va = (wl * sl[2] / rl + wr * sr[2] / rr) / (wl + wr)
    Ha = (wl * (sl[3] + pl) / rl + wr * (sr[3] + pr) / rr) / (wl + wr)
    ca = torch.sqrt(torch.clamp((gamma - 1.0) * (Ha - 0.5 * (ua * ua + va * va)), min=0.0))
    sL = torch.clamp(torch.minimum(ul - cl, ua - ca), max=0.0)
    sR = torch.clamp(torch.maximum(ur + cr, ua + ca), min=0.0)
    return tuple((sR * a - sL * b + sL * sR * (y - x)) / (sR - sL) for a, b, x, y in zip(fl, fr, sl, sr))


def rusanov(sl, sr, gamma: float = GAMMA):
    """Rusanov flux (eq 2.12) with the largest |u| + c of the two face states."""
    fl, ul, pl = _phys(*sl, gamma)
    fr, ur, pr = _phys(*sr, gamma)
    a = torch.maximum(ul.abs() + torch.sqrt(gamma * pl / sl[0]), ur.abs() + torch.sqrt(gamma * pr / sr[0]))
    return tuple(0.5 * (x + y) - 0.5 * a * (d - c) for x, y, c, d in zip(fl, fr, sl, sr))


FLUXES = {"hlle": hlle, "rusanov": rusanov}


def rhs(q: torch.Tensor, alpha, dx: float, dy: float, gamma: float = GAMMA, flux: str = "hlle"):
    """L(q) with learned face states (alpha given) or the plain MINMOD
    states (alpha None).  Returns (L, per-solve face sides that fell back)."""
    fn = FLUXES[flux]
    out = torch.zeros_like(q)
    nfb = torch.zeros(q.shape[0], dtype=torch.int64)
    for axis, (dim, d) in enumerate(((3, dx), (2, dy))):
        ML, MR = minmod_faces(q, dim, gamma)
        if alpha is None:
            QL, QR = ML, MR
        else:
            QL, QR = learned_faces(q, alpha, axis)
            okl, okr = admissible(QL, gamma), admissible(QR, gamma)
            nfb = nfb + (~okl).flatten(1).sum(1) + (~okr).flatten(1).sum(1)
            QL = torch.where(okl, QL, ML)
            QR = torch.where(okr, QR, MR)
        nm, tm = (1, 2) if axis == 0 else (2, 1)
        F = fn((QL[:, 0], QL[:, nm], QL[:, tm], QL[:, 3]), (QR[:, 0], QR[:, nm], QR[:, tm], QR[:, 3]), gamma)
        Fc = [None] * 4
        Fc[0], Fc[nm], Fc[tm], Fc[3] = F
        Fc = torch.stack(Fc, dim=1)  # flux through face i+1/2, Cartesian order
        out = out - (Fc - L._shift(Fc, -1, dim)) / d
    return out, nfb


def inadmissible_cells(q: torch.Tensor, gamma: float = GAMMA) -> torch.Tensor:
    """Per solve: does any cell have rho <= 0 or p <= 0 (or a non-finite value)?"""
    return (~admissible(q, gamma)).flatten(1).any(dim=1)


def plain_step(q, dt, dx, dy, gamma=GAMMA, flux="hlle"):
    """Heun step (eq 2.19) of the plain MINMOD scheme at fixed dt."""
    L0, _ = rhs(q, None, dx, dy, gamma, flux)
    q1 = q + dt * L0
    L1, _ = rhs(q1, None, dx, dy, gamma, flux)
    return 0.5 * q + 0.5 * (q1 + dt * L1)


def learned_step(params, q, dt, dx, dy, gamma=GAMMA, flux="hlle", order=1, round_bf16=True):
    """One Heun step of the learned Euler scheme; the network runs on each
    stage's input.  Returns (q_next, stats) with stats = dict(fallback_faces,
    redone = per-solve flags of steps redone with the plain scheme).  The
    second stage's fallbacks are not counted for a solve whose first stage
    was already inadmissible."""
    P = L.projector(order)
    a0 = coefficients(L.cnn(params, q, round_bf16), P)
    L0, f0 = rhs(q, a0, dx, dy, gamma, flux)
    q1 = q + dt * L0
    bad1 = inadmissible_cells(q1, gamma)
    q1s = torch.where(bad1[:, None, None, None], q, q1)
    a1 = coefficients(L.cnn(params, q1s, round_bf16), P)
    L1, f1 = rhs(q1s, a1, dx, dy, gamma, flux)
    q2 = 0.5 * q + 0.5 * (q1s + dt * L1)
    bad = bad1 | inadmissible_cells(q2, gamma)
    if bool(bad.any()):
        qp = plain_step(q, dt, dx, dy, gamma, flux)
        q2 = torch.where(bad[:, None, None, None], qp, q2)
    nfb = f0 + torch.where(bad1, torch.zeros_like(f1), f1)
    return q2, {"fallback_faces": int(nfb.sum()), "redone": bad}


def rollout_loss(params, q0, targets, dt, dx, dy, scale, gamma=GAMMA, flux="hlle", round_bf16=True):
    """eq 2.28 for the Euler state: sum over t = 1..T of the MSE between the
    learned rollout and targets (B, T, 4, H, W), variable v divided by
    scale[v]."""
    q = q0
    loss = torch.zeros((), dtype=F64)
    s = torch.as_tensor(scale, dtype=F64)[None, :, None, None]
    for t in range(targets.shape[1]):
        q, _ = learned_step(params, q, dt, dx, dy, gamma, flux, round_bf16=round_bf16)
        loss = loss + (((q - targets[:, t]) / s) ** 2).mean()
    return loss
