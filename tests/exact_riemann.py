"""Exact solutions of the 1D Riemann problems used as pins for the oracle.

Written from the mathematics of the exact Riemann solvers in E. F. Toro,
"Riemann Solvers and Numerical Methods for Fluid Dynamics" (ideal gas,
chapter 4) and "Shock-Capturing Methods for Free-Surface Shallow Flows"
(shallow water, chapter 5).  These are independent of the finite-volume
oracle: they only use the Rankine-Hugoniot and Riemann-invariant relations.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq


# ------------------------------------------------------------ shallow water

def swe_star(hl, ul, hr, ur, g=9.81):
    """Star depth and velocity of the SWE Riemann problem."""
    al, ar = np.sqrt(g * hl), np.sqrt(g * hr)

    def fk(h, hk, ak):
        if h <= hk:  # rarefaction: Riemann invariant u + 2c
            return 2.0 * (np.sqrt(g * h) - ak)
        return (h - hk) * np.sqrt(0.5 * g * (h + hk) / (h * hk))  # shock (Rankine-Hugoniot)

    f = lambda h: fk(h, hl, al) + fk(h, hr, ar) + ur - ul
    hs = brentq(f, 1e-14, 100.0 * max(hl, hr), xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (fk(hs, hr, ar) - fk(hs, hl, al))
    return hs, us


def swe_waves(hl, ul, hr, ur, g=9.81):
    """Wave speeds: (left head, left tail or shock, right shock or tail, right head)."""
    hs, us = swe_star(hl, ul, hr, ur, g)
    al, ar, a_s = np.sqrt(g * hl), np.sqrt(g * hr), np.sqrt(g * hs)
    if hs > hl:
        sl = ul - al * np.sqrt(0.5 * (hs + hl) * hs / hl ** 2)
        left = (sl, sl)
    else:
        left = (ul - al, us - a_s)
    if hs > hr:
        sr = ur + ar * np.sqrt(0.5 * (hs + hr) * hs / hr ** 2)
        right = (sr, sr)
    else:
        right = (us + a_s, ur + ar)
    return left + right, hs, us


def swe_sample(xi, hl, ul, hr, ur, g=9.81):
    """(h, u) of the self-similar solution at xi = (x - x0)/t (array)."""
    xi = np.asarray(xi, dtype=float)
    (lh, lt, rt, rh), hs, us = swe_waves(hl, ul, hr, ur, g)
    al, ar = np.sqrt(g * hl), np.sqrt(g * hr)
    h = np.empty_like(xi)
    u = np.empty_like(xi)
    left = xi < us
    # left family
    if hs > hl:
        m = left & (xi < lh)
        h[m], u[m] = hl, ul
        m = left & (xi >= lh)
        h[m], u[m] = hs, us
    else:
        m = left & (xi < lh)
        h[m], u[m] = hl, ul
        m = left & (xi > lt)
        h[m], u[m] = hs, us
        m = left & (xi >= lh) & (xi <= lt)
        a = (ul + 2.0 * al - xi[m]) / 3.0
        u[m] = (ul + 2.0 * al + 2.0 * xi[m]) / 3.0
        h[m] = a * a / g
    right = ~left
    if hs > hr:
        m = right & (xi > rt)
        h[m], u[m] = hr, ur
        m = right & (xi <= rt)
        h[m], u[m] = hs, us
    else:
        m = right & (xi > rh)
        h[m], u[m] = hr, ur
        m = right & (xi < rt)
        h[m], u[m] = hs, us
        m = right & (xi >= rt) & (xi <= rh)
        a = (-ur + 2.0 * ar + xi[m]) / 3.0
        u[m] = (ur - 2.0 * ar + 2.0 * xi[m]) / 3.0
        h[m] = a * a / g
    return h, u


# --------------------------------------------------------------- ideal gas

def euler_star(rl, ul, pl, rr, ur, pr, gamma=1.4):
    al, ar = np.sqrt(gamma * pl / rl), np.sqrt(gamma * pr / rr)
    gm = gamma - 1.0
    gp = gamma + 1.0

    def fk(p, rk, pk, ak):
        if p > pk:  # shock
            A = 2.0 / (gp * rk)
            B = gm / gp * pk
            return (p - pk) * np.sqrt(A / (p + B))
        return 2.0 * ak / gm * ((p / pk) ** (gm / (2.0 * gamma)) - 1.0)  # rarefaction

    f = lambda p: fk(p, rl, pl, al) + fk(p, rr, pr, ar) + ur - ul
    ps = brentq(f, 1e-14, 1e3 * max(pl, pr), xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (fk(ps, rr, pr, ar) - fk(ps, rl, pl, al))
    return ps, us


def euler_sample(xi, rl, ul, pl, rr, ur, pr, gamma=1.4):
    """(rho, u, p) of the self-similar solution at xi = (x - x0)/t."""
    xi = np.asarray(xi, dtype=float)
    ps, us = euler_star(rl, ul, pl, rr, ur, pr, gamma)
    gm, gp = gamma - 1.0, gamma + 1.0
    al, ar = np.sqrt(gamma * pl / rl), np.sqrt(gamma * pr / rr)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    left = xi < us
    if ps > pl:
        sl = ul - al * np.sqrt(gp / (2 * gamma) * ps / pl + gm / (2 * gamma))
        rsl = rl * (ps / pl + gm / gp) / (gm / gp * ps / pl + 1.0)
        m = left & (xi < sl)
        rho[m], u[m], p[m] = rl, ul, pl
        m = left & (xi >= sl)
        rho[m], u[m], p[m] = rsl, us, ps
    else:
        rsl = rl * (ps / pl) ** (1.0 / gamma)
        asl = al * (ps / pl) ** (gm / (2 * gamma))
        sh, st = ul - al, us - asl
        m = left & (xi < sh)
        rho[m], u[m], p[m] = rl, ul, pl
        m = left & (xi > st)
        rho[m], u[m], p[m] = rsl, us, ps
        m = left & (xi >= sh) & (xi <= st)
        base = 2.0 / gp + gm / (gp * al) * (ul - xi[m])
        rho[m] = rl * base ** (2.0 / gm)
        u[m] = 2.0 / gp * (al + gm / 2.0 * ul + xi[m])
        p[m] = pl * base ** (2.0 * gamma / gm)
    right = ~left
    if ps > pr:
        sr = ur + ar * np.sqrt(gp / (2 * gamma) * ps / pr + gm / (2 * gamma))
        rsr = rr * (ps / pr + gm / gp) / (gm / gp * ps / pr + 1.0)
        m = right & (xi > sr)
        rho[m], u[m], p[m] = rr, ur, pr
        m = right & (xi <= sr)
        rho[m], u[m], p[m] = rsr, us, ps
    else:
        rsr = rr * (ps / pr) ** (1.0 / gamma)
        asr = ar * (ps / pr) ** (gm / (2 * gamma))
        sh, st = ur + ar, us + asr
        m = right & (xi > sh)
        rho[m], u[m], p[m] = rr, ur, pr
        m = right & (xi < st)
        rho[m], u[m], p[m] = rsr, us, ps
        m = right & (xi >= st) & (xi <= sh)
        base = 2.0 / gp - gm / (gp * ar) * (ur - xi[m])
        rho[m] = rr * base ** (2.0 / gm)
        u[m] = 2.0 / gp * (-ar + gm / 2.0 * ur + xi[m])
        p[m] = pr * base ** (2.0 * gamma / gm)
    return rho, u, p


def cell_average(fn, n, sub=64, x0=0.5, t=1.0):
    """Average a sampled 1D field over the n cells of [0,1] with `sub` midpoint
    sub-samples per cell; fn maps xi = (x - x0)/t to values."""
    xs = (np.arange(n * sub) + 0.5) / (n * sub)
    vals = fn((xs - x0) / t)
    return vals.reshape(n, sub).mean(axis=1)
