"""Oracle of the learned-coefficient finite-volume step.  TEST INFRASTRUCTURE
ONLY: used by tests/, the smoke check and nothing in the product path.

Thesis "A Machine Learning accelerated geophysical fluid solver":
  - section 2.5.1 (eq 2.26-2.27): a network predicts the coefficients of a
    pseudo-linear stencil, value = sum_k alpha_k(u) u_k;
  - section 2.5.3, fourth approach (Fig 7): a CNN outputs "constraint alpha"
    per conserved component, which can be set up so the reconstruction is at
    least first-order accurate; the coefficients multiply the stencil values
    to give the face states Q_l, Q_r, which then enter the numerical flux
    (section 2.3.2) and the Heun update (eq 2.19);
  - eq 2.28: training loss = sum over T unrolled steps of the MSE between the
    coarse prediction and the coarsened high-resolution reference.

Readings (the thesis leaves these open):
  - stencil: the six cells i-2..i+3 around face i+1/2 (centres at
    -2.5..2.5 cell widths from the face); every cell owns its +x and +y face
    and carries two coefficient vectors per face (left state, right state)
    per conserved variable: 2 axes x 2 sides x 3 variables x 6 = 72 channels,
    channel index ((axis*2 + side)*3 + var)*6 + k;
  - constraint: exact for cell averages of polynomials of degree <= 1
    (sum alpha = 1, sum alpha x = 0), imposed by alpha = alpha_base + P z with
    P the orthogonal projector onto the null space of the 2 x 6 moment
    matrix; alpha_base = Fromm's stencils (L: q_i + (q_{i+1} - q_{i-1})/4,
    R: q_{i+1} - (q_{i+2} - q_i)/4);
  - network: 5 layers of 3x3 convolution (3 -> 32 -> 32 -> 32 -> 32 -> 72),
    ReLU between layers, periodic padding, per-channel affine normalisation
    of the input; BF16 weights and activations: the normalised input and
    every post-ReLU activation are rounded to bfloat16 (round to nearest
    even), weights are bfloat16 values, biases float; the last layer is not
    rounded.  Accumulation here is double precision;
  - positivity: a face side whose learned depth is <= 0 uses the MINMOD
    state of that side instead; if a stage produces a cell with h <= 0 the
    whole step of that solve is redone with the plain MINMOD scheme;
  - loss: MSE averaged over cells and variables, variable v scaled by 1/s_v,
    summed over the T unrolled steps.
Only the periodic shallow-water case is defined here (the learned workload).
Gradients come from automatic differentiation of these double-precision
operations (rounding to bfloat16 passes gradients straight through).
"""
from __future__ import annotations

import math

import torch

F64 = torch.float64
OFFSETS = torch.tensor([-2.5, -1.5, -0.5, 0.5, 1.5, 2.5], dtype=F64)
ALPHA_BASE = torch.tensor([[0.0, -0.25, 1.0, 0.25, 0.0, 0.0],    # left state of face i+1/2
                           [0.0, 0.0, 0.25, 1.0, -0.25, 0.0]],   # right state
                          dtype=F64)
LAYERS = [(3, 32), (32, 32), (32, 32), (32, 32), (32, 72)]


# ------------------------------------------------------------- constraint

def moment_matrix(order: int = 1) -> torch.Tensor:
    """Row p: the cell average of x^p over each stencil cell (cells of unit
    width centred at OFFSETS); sum_k alpha_k m_p(k) = [p == 0] makes the face
    value exact for polynomials of degree <= order."""
    rows = []
    for p in range(order + 1):
        hi = (OFFSETS + 0.5) ** (p + 1)
        lo = (OFFSETS - 0.5) ** (p + 1)
        rows.append((hi - lo) / (p + 1))
    return torch.stack(rows)


def projector(order: int = 1) -> torch.Tensor:
    A = moment_matrix(order)
    return torch.eye(6, dtype=F64) - A.T @ torch.linalg.solve(A @ A.T, A)


def coefficients(z: torch.Tensor, P: torch.Tensor) -> torch.Tensor:
    """z (B, 72, H, W) -> alpha (B, axis, side, var, k, H, W) = alpha_base + P z."""
    B, C, H, W = z.shape
    zz = z.reshape(B, 2, 2, 3, 6, H, W)
    return ALPHA_BASE[None, None, :, None, :, None, None] + torch.einsum("kj,baswjhx->baswkhx", P, zz)


# ------------------------------------------------------------------ network

def bf16(x: torch.Tensor, ste: bool = True) -> torch.Tensor:
    r = x.detach().to(torch.bfloat16).to(F64)
    return x + (r - x.detach()) if ste else r


def conv3x3_periodic(x: torch.Tensor, w: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """out[o, y, x] = b[o] + sum_{c, ky, kx} w[o, c, ky, kx] in[c, y + ky - 1, x + kx - 1],
    indices taken periodically."""
    out = b[None, :, None, None].expand(x.shape[0], -1, x.shape[2], x.shape[3])
    for ky in range(3):
        for kx in range(3):
            xs = torch.roll(x, shifts=(1 - ky, 1 - kx), dims=(2, 3))
            out = out + torch.einsum("oc,bchw->bohw", w[:, :, ky, kx], xs)
    return out


def cnn(params: dict, q: torch.Tensor, round_bf16: bool = True, shadow_f32: bool = False) -> torch.Tensor:
    """Raw coefficients z (B, 72, H, W) of states q (B, 3, H, W).

    shadow_f32: diagnostic only -- normalise and accumulate every convolution
    in float32 (as the GPU does) instead of float64; the distance between
    this and the double-precision result bounds what float32 accumulation
    alone changes through the bfloat16 rounding decisions."""
    rnd = bf16 if round_bf16 else (lambda t: t)
    W, bias = params["w"], params["b"]
    if shadow_f32:
        x = ((q.float() - params["mean"].float()[None, :, None, None])
             * params["inv_std"].float()[None, :, None, None]).double()
        x = rnd(x).float()
        for l in range(len(W) - 1):
            x = rnd(torch.relu(conv3x3_periodic(x, W[l].float(), bias[l].float())).double()).float()
        return conv3x3_periodic(x, W[-1].float(), bias[-1].float()).double()
    x = (q - params["mean"][None, :, None, None]) * params["inv_std"][None, :, None, None]
    x = rnd(x)
    for l in range(len(W) - 1):
        x = rnd(torch.relu(conv3x3_periodic(x, W[l], bias[l])))
    return conv3x3_periodic(x, W[-1], bias[-1])


def init_params(seed: int, hidden: int = 32, scale_last: float = 0.0, layers=None) -> dict:
    """Seeded parameters: He-scaled weights rounded to bfloat16, zero biases,
    last layer scaled by scale_last (0: the network starts at alpha_base).
    The mean/inv_std normalisation is (1, 0, 0) / (10, 10, 10) unless set."""
    g = torch.Generator().manual_seed(seed)
    layers = layers or [(3, hidden), (hidden, hidden), (hidden, hidden), (hidden, hidden), (hidden, 72)]
    w, b = [], []
    for i, (ci, co) in enumerate(layers):
        s = math.sqrt(2.0 / (9 * ci))
        t = torch.randn(co, ci, 3, 3, generator=g, dtype=F64) * s
        if i == len(layers) - 1:
            t = t * scale_last
        w.append(t.to(torch.bfloat16).to(F64))
        b.append(torch.zeros(co, dtype=F64))
    return {"w": w, "b": b, "mean": torch.tensor([1.0, 0.0, 0.0], dtype=F64),
            "inv_std": torch.tensor([10.0, 10.0, 10.0], dtype=F64)}


# ------------------------------------------------------- finite-volume parts

def _shift(x: torch.Tensor, k: int, dim: int) -> torch.Tensor:
    """y[i] = x[i + k] along dim, periodically."""
    return torch.roll(x, shifts=-k, dims=dim)


def _minmod(a, b):
    same = ((a > 0) & (b > 0)) | ((a < 0) & (b < 0))
    m = torch.where(a.abs() <= b.abs(), a, b)
    return torch.where(same, m, torch.zeros_like(a))


def minmod_faces(q: torch.Tensor, dim: int):
    """MINMOD face states of face i+1/2 (eq 2.18) with the cell-average
    safeguard for non-positive depth.  q (B, 3, H, W); returns QL, QR."""
    qm1, q0, q1, q2 = _shift(q, -1, dim), q, _shift(q, 1, dim), _shift(q, 2, dim)
    QL = q0 + 0.5 * _minmod(q0 - qm1, q1 - q0)
    QR = q1 - 0.5 * _minmod(q1 - q0, q2 - q1)
    QL = torch.where((QL[:, :1] > 0), QL, q0)
    QR = torch.where((QR[:, :1] > 0), QR, q1)
    return QL, QR


def learned_faces(q: torch.Tensor, alpha: torch.Tensor, axis: int):
    """Face states of face i+1/2 owned by cell i from its coefficients:
    Q_side = sum_k alpha[axis, side, v, k] q_v(i - 2 + k)."""
    dim = 3 if axis == 0 else 2
    st = torch.stack([_shift(q, k - 2, dim) for k in range(6)], dim=2)  # (B, 3, 6, H, W)
    QL = (alpha[:, axis, 0] * st).sum(dim=2)
    QR = (alpha[:, axis, 1] * st).sum(dim=2)
    return QL, QR


def hlle(hl, ml, tl, hr, mr, tr, g):
    """HLLE flux (eq 2.16) of normal-frame SWE states, Einfeldt speeds from
    the Roe average clamped with zero."""
    ul, ur = ml / hl, mr / hr
    cl, cr = torch.sqrt(g * hl), torch.sqrt(g * hr)
    wl, wr = torch.sqrt(hl), torch.sqrt(hr)
    ua = (wl * ul + wr * ur) / (wl + wr)
    ca = torch.sqrt(g * 0.5 * (hl + hr))
    sL = torch.clamp(torch.minimum(ul - cl, ua - ca), max=0.0)
    sR = torch.clamp(torch.maximum(ur + cr, ua + ca), min=0.0)
    fl = (ml, ml * ul + 0.5 * g * hl * hl, tl * ul)
    fr = (mr, mr * ur + 0.5 * g * hr * hr, tr * ur)
    dq = (hr - hl, mr - ml, tr - tl)
    return tuple((sR * a - sL * b + sL * sR * d) / (sR - sL) for a, b, d in zip(fl, fr, dq))


def rusanov(hl, ml, tl, hr, mr, tr, g):
    """Rusanov flux (eq 2.12) with the speed of the face states."""
    ul, ur = ml / hl, mr / hr
    a = torch.maximum(ul.abs() + torch.sqrt(g * hl), ur.abs() + torch.sqrt(g * hr))
    fl = (ml, ml * ul + 0.5 * g * hl * hl, tl * ul)
    fr = (mr, mr * ur + 0.5 * g * hr * hr, tr * ur)
    dq = (hr - hl, mr - ml, tr - tl)
    return tuple(0.5 * (x + y) - 0.5 * a * d for x, y, d in zip(fl, fr, dq))


FLUXES = {"hlle": hlle, "rusanov": rusanov}


def rhs(q: torch.Tensor, alpha, dx: float, dy: float, g: float = 9.81, flux: str = "hlle", blend: bool = False,
        limiter=None):
    """Spatial operator L(q) with learned face states (alpha given) or the
    plain MINMOD states (alpha None).  blend (learned only): each face's flux
    is the flux-limiter blend of section 2.5.3 (second approach), see
    blend_flux (limiter: its frozen-limiter / tape argument).  Returns (L, per-solve number of face sides that fell back to
    MINMOD)."""
    fn = FLUXES[flux]
    L = torch.zeros_like(q)
    nfb = torch.zeros(q.shape[0], dtype=torch.int64)
    for axis, (dim, d) in enumerate(((3, dx), (2, dy))):
        ML, MR = minmod_faces(q, dim)
        if alpha is None:
            QL, QR = ML, MR
        else:
            QL, QR = learned_faces(q, alpha, axis)
            okl, okr = QL[:, :1] > 0, QR[:, :1] > 0
            nfb = nfb + (~okl).flatten(1).sum(1) + (~okr).flatten(1).sum(1)
            QL = torch.where(okl, QL, ML)
            QR = torch.where(okr, QR, MR)
        nm, tm = (1, 2) if axis == 0 else (2, 1)
        F = fn(QL[:, 0], QL[:, nm], QL[:, tm], QR[:, 0], QR[:, nm], QR[:, tm], g)
        Fc = [None, None, None]
        Fc[0], Fc[nm], Fc[tm] = F
        Fc = torch.stack(Fc, dim=1)  # flux through face i+1/2, Cartesian order
        if blend and alpha is not None:
            Fc = blend_flux(q, Fc, dim, nm, tm, fn, g, limiter)
        L = L - (Fc - _shift(Fc, -1, dim)) / d
    return L, nfb


# ---- flux-limiter blend (section 2.5.3, second approach) ------------------
# The flux of face i+1/2 is pulled from a high-resolution flux (here: the
# learned face states' flux) towards the low-resolution one (the flux of the
# two cell averages) by a flux limiter of the ratio of successive gradients at
# cell i:  F = F_low - phi(r_i) (F_low - F_high),
# r_i = (q_i - q_{i-1}) / (q_{i+1} - q_i).  Readings: the limiter is MINMOD
# (the limiter the thesis uses throughout), phi(r) = max(0, min(1, r)); r is
# taken per conserved variable (h, hu, hv) and always at the face's low-index
# cell i, as printed, whatever the flow direction; where q_{i+1} = q_i the
# ratio is undefined and phi = 0 (the low-resolution flux).

def limiter_minmod(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """phi(r) of the MINMOD flux limiter for r = a / b (a = q_i - q_{i-1},
    b = q_{i+1} - q_i); 0 where b = 0."""
    nz = b != 0
    r = torch.where(nz, a / torch.where(nz, b, torch.ones_like(b)), torch.zeros_like(a))
    return torch.clamp(r, 0.0, 1.0)


def blend_flux(q, F_high, dim, nm, tm, fn, g, limiter=None):
    """Blended flux of every face i+1/2 along dim (Cartesian order, like
    F_high): the low-resolution flux is the numerical flux of the cell
    averages q_i and q_{i+1}.

    limiter: None (phi differentiated like every other operation), or a
    dict for training: {"frozen": True} treats phi as a constant in the
    gradient (the frozen-limiter adjoint: d phi / d q ~ 1 / (q_{i+1} - q_i)
    is unbounded where successive differences vanish, as on a flat
    background, and overflows there in single precision); with a "tape"
    list and "replay" False every phi is appended to the tape, with
    "replay" True the phis are taken from the tape in order instead (so a
    finite difference can hold them fixed)."""
    qa, qb = q, _shift(q, 1, dim)
    Fl = fn(qa[:, 0], qa[:, nm], qa[:, tm], qb[:, 0], qb[:, nm], qb[:, tm], g)
    F_low = [None, None, None]
    F_low[0], F_low[nm], F_low[tm] = Fl
    F_low = torch.stack(F_low, dim=1)
    if limiter is not None and limiter.get("replay"):
        phi = limiter["tape"][limiter["pos"]]
        limiter["pos"] += 1
    else:
        phi = limiter_minmod(q - _shift(q, -1, dim), _shift(q, 1, dim) - q)
        if limiter is not None and limiter.get("frozen"):
            phi = phi.detach()
        if limiter is not None and "tape" in limiter:
            limiter["tape"].append(phi.detach())
    return F_low - phi * (F_low - F_high)


def plain_step(q, dt, dx, dy, g=9.81, flux="hlle"):
    """Heun step (eq 2.19) of the plain MINMOD scheme at fixed dt."""
    L0, _ = rhs(q, None, dx, dy, g, flux)
    q1 = q + dt * L0
    L1, _ = rhs(q1, None, dx, dy, g, flux)
    return 0.5 * q + 0.5 * (q1 + dt * L1)


def learned_step(params, q, dt, dx, dy, g=9.81, flux="hlle", order=1, round_bf16=True, blend=False, limiter=None):
    """One Heun step of the learned scheme (blend: with the flux-limiter blend
    of its face fluxes, see blend_flux and its limiter argument).  The network runs on the input of
    each stage.  Returns (q_next, stats) with stats = dict(fallback_faces,
    redone = per-solve flags of steps redone with the plain scheme).  Face
    sides of the second stage are not counted for a solve whose first stage
    was already inadmissible (its step is redone either way)."""
    P = projector(order)
    a0 = coefficients(cnn(params, q, round_bf16), P)
    L0, f0 = rhs(q, a0, dx, dy, g, flux, blend, limiter)
    q1 = q + dt * L0
    bad1 = (q1[:, 0] <= 0).flatten(1).any(dim=1)
    # a solve whose first stage is already inadmissible is redone; evaluate the
    # second stage on a safe copy so nothing non-finite enters the graph
    q1s = torch.where(bad1[:, None, None, None], q, q1)
    a1 = coefficients(cnn(params, q1s, round_bf16), P)
    L1, f1 = rhs(q1s, a1, dx, dy, g, flux, blend, limiter)
    q2 = 0.5 * q + 0.5 * (q1s + dt * L1)
    bad = bad1 | (q2[:, 0] <= 0).flatten(1).any(dim=1)
    if bool(bad.any()):
        qp = plain_step(q, dt, dx, dy, g, flux)
        q2 = torch.where(bad[:, None, None, None], qp, q2)
    nfb = f0 + torch.where(bad1, torch.zeros_like(f1), f1)
    return q2, {"fallback_faces": int(nfb.sum()), "redone": bad}


# ---- direct face states (thesis section 5.3, planar shallow water) -------
# The network maps the cell averages to the states at the four faces of each
# cell, Q^l, Q^r, Q^b, Q^u (left, right, bottom, top); the flux of a face is
# the numerical flux of the states its two cells give it, so the face is
# shared and the scheme stays conservative.  Section 2.5.3 (third approach)
# splits the network's output into a height part and a momentum part and ends
# the height part in a Softplus so that every reconstructed depth is
# positive.  Reading of the output: channel 3f + v (f = l, r, b, u) belongs to
# face state f and variable v, in the input's normalised units (de-normalised
# by 1/inv_std_v);
#   depth     Q^f_h = q_h * softplus(z_{3f} / inv_std_h + c),  c = ln(e - 1),
#             softplus(c) = 1,
#   momentum  Q^f_m = q_m + z_{3f+m} / inv_std_m   (m = hu, hv),
# so a zero head is the first-order scheme and a face depth is positive
# wherever its cell's is (the Softplus part is the depth relative to the
# cell's own).  The other output channels are unused.

SOFTPLUS_SHIFT = math.log(math.e - 1.0)


def softplus(x: torch.Tensor) -> torch.Tensor:
    """ln(1 + e^x), evaluated without overflow."""
    return torch.logaddexp(x, torch.zeros_like(x))


def direct_faces(params, q, round_bf16=True):
    """(Ql, Qr, Qb, Qu), each (B, 3, H, W): the network's four face states of every cell."""
    z = cnn(params, q, round_bf16)
    sig = (1.0 / params["inv_std"])[None, :, None, None]
    out = []
    for f in range(4):
        zf = sig * z[:, 3 * f:3 * f + 3]
        depth = q[:, :1] * softplus(zf[:, :1] + SOFTPLUS_SHIFT)
        out.append(torch.cat([depth, q[:, 1:] + zf[:, 1:]], dim=1))
    return tuple(out)


def direct_rhs(params, q, dx, dy, g=9.81, flux="hlle", round_bf16=True):
    """L(q) of the direct face-state scheme: the flux of face i+1/2 from
    cell i's right state and cell i+1's left state (x), cell j's top state and
    cell j+1's bottom state (y).  A face side whose depth is not positive takes
    its MINMOD state (counted).  Returns (L, per-solve fallback face sides)."""
    fn = FLUXES[flux]
    Ql, Qr, Qb, Qu = direct_faces(params, q, round_bf16)
    L = torch.zeros_like(q)
    nfb = torch.zeros(q.shape[0], dtype=torch.int64)
    for axis, (dim, d, lo, hi) in enumerate(((3, dx, Qr, Ql), (2, dy, Qu, Qb))):
        ML, MR = minmod_faces(q, dim)
        QL, QR = lo, _shift(hi, 1, dim)  # face i+1/2: cell i's high side, cell i+1's low side
        okl, okr = QL[:, :1] > 0, QR[:, :1] > 0
        nfb = nfb + (~okl).flatten(1).sum(1) + (~okr).flatten(1).sum(1)
        QL = torch.where(okl, QL, ML)
        QR = torch.where(okr, QR, MR)
        nm, tm = (1, 2) if axis == 0 else (2, 1)
        F = fn(QL[:, 0], QL[:, nm], QL[:, tm], QR[:, 0], QR[:, nm], QR[:, tm], g)
        Fc = [None, None, None]
        Fc[0], Fc[nm], Fc[tm] = F
        Fc = torch.stack(Fc, dim=1)
        L = L - (Fc - _shift(Fc, -1, dim)) / d
    return L, nfb


def direct_step(params, q, dt, dx, dy, g=9.81, flux="hlle", round_bf16=True):
    """One Heun step of the direct face-state scheme, with the same
    admissibility rule as the learned step: a solve with a non-positive depth
    after either stage redoes the step with the plain scheme.  Returns
    (q_next, stats) as learned_step."""
    L0, f0 = direct_rhs(params, q, dx, dy, g, flux, round_bf16)
    q1 = q + dt * L0
    bad1 = (q1[:, 0] <= 0).flatten(1).any(dim=1)
    q1s = torch.where(bad1[:, None, None, None], q, q1)
    L1, f1 = direct_rhs(params, q1s, dx, dy, g, flux, round_bf16)
    q2 = 0.5 * q + 0.5 * (q1s + dt * L1)
    bad = bad1 | (q2[:, 0] <= 0).flatten(1).any(dim=1)
    if bool(bad.any()):
        qp = plain_step(q, dt, dx, dy, g, flux)
        q2 = torch.where(bad[:, None, None, None], qp, q2)
    nfb = f0 + torch.where(bad1, torch.zeros_like(f1), f1)
    return q2, {"fallback_faces": int(nfb.sum()), "redone": bad}


def rollout_loss(params, q0, targets, dt, dx, dy, scale, g=9.81, flux="hlle", round_bf16=True, direct=False,
                 blend=False, limiter=None):
    """eq 2.28: sum over t = 1..T of the MSE between the learned rollout and
    the reference targets (B, T, 3, H, W); variable v is divided by scale[v].
    direct: the rollout of the direct face-state scheme instead; blend: of the
    learned scheme with the flux-limiter blend of its face fluxes, trained
    with the limiter frozen in the gradient (blend_flux) unless a limiter
    dict is given."""
    if blend and limiter is None:
        limiter = {"frozen": True}
    q = q0
    loss = torch.zeros((), dtype=F64)
    s = torch.as_tensor(scale, dtype=F64)[None, :, None, None]
    for t in range(targets.shape[1]):
        if direct:
            q, _ = direct_step(params, q, dt, dx, dy, g, flux, round_bf16=round_bf16)
        else:
            q, _ = learned_step(params, q, dt, dx, dy, g, flux, round_bf16=round_bf16, blend=blend, limiter=limiter)
        loss = loss + (((q - targets[:, t]) / s) ** 2).mean()
    return loss


def block_average(q: torch.Tensor, f: int) -> torch.Tensor:
    """Exact cell-average coarsening (training targets of section 2.5.1 come
    from coarsened high-resolution runs): coarse cell (I, J) is the mean of
    the f x f fine cells it covers, q (..., H, W) with H, W multiples of f."""
    *lead, H, W = q.shape
    return q.reshape(*lead, H // f, f, W // f, f).mean(dim=(-3, -1))
