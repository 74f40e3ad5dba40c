"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module holds no part of the solver's arithmetic: it only draws
initial states with numpy ``Generator(PCG64(seed))`` in a documented order and
returns them as float64 arrays in the solver layout ``[var][y][x]`` (x fastest).

Initial conditions follow the thesis's test problems (dam break of section
3.1.1, Gaussian hump of section 3.2.1, the Sod-type problem of section 4.1.1,
four-quadrant Riemann data of section 4.2) and the synthetic workloads built
on them: a Gaussian hump on a periodic unit square, a sum of seeded Gaussian
bumps over a bed of seeded Gaussians, seeded four-quadrant Euler data, and
multi-hump periodic states for the learned coarse solver.
"""
from __future__ import annotations

import numpy as np

G = 9.81
GAMMA = 1.4


def centres(n: int, length: float = 1.0) -> np.ndarray:
    """Cell-centre coordinates (i + 1/2) * L / n."""
    return (np.arange(n) + 0.5) * (length / n)


def gaussian_hump(n: int) -> np.ndarray:
    """h = 1 + 0.1 exp(-r^2 / 0.01) about (1/2, 1/2), u = v = 0, sampled at
    cell centres of an n x n periodic grid on [0,1]^2."""
    x = centres(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    h = 1.0 + 0.1 * np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / 0.01)
    q = np.zeros((3, n, n))
    q[0] = h
    return q


def _gauss_sum(n, rng, count, amp_lo, amp_hi):
    """Sum of `count` Gaussians A exp(-|x - c|^2 / w^2); per Gaussian the draws
    are A ~ U[amp_lo, amp_hi], w ~ U[0.02, 0.1], c ~ U[0,1]^2, in that order."""
    x = centres(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    f = np.zeros((n, n))
    for _ in range(count):
        a = rng.uniform(amp_lo, amp_hi)
        w = rng.uniform(0.02, 0.1)
        cx, cy = rng.uniform(0.0, 1.0, size=2)
        f += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (w * w))
    return f


def swe_bathy(n: int, seed: int = 0):
    """Shallow water over a bed: b = sum of 8 seeded Gaussians (amplitude
    U[0, 0.3], width U[0.02, 0.1]); free surface h + b = 1 + sum of 16 seeded
    Gaussian bumps (amplitude U[-0.1, 0.1], same width law); zero velocity.
    Returns (q[3,n,n], b[n,n])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = _gauss_sum(n, rng, 8, 0.0, 0.3)
    eta = 1.0 + _gauss_sum(n, rng, 16, -0.1, 0.1)
    h = eta - b
    if h.min() < 0.05:
        raise ValueError(f"seed {seed}: minimum depth {h.min():.3f} < 0.05")
    q = np.zeros((3, n, n))
    q[0] = h
    return q, b


def lake_at_rest(n: int, seed: int = 0, level: float = 1.0):
    """Flat free surface h + b = level over the seeded Gaussian bed, u = v = 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = _gauss_sum(n, rng, 8, 0.0, 0.3)
    q = np.zeros((3, n, n))
    q[0] = level - b
    return q, b


def euler_quadrants(n: int, seed: int = 0, gamma: float = GAMMA) -> np.ndarray:
    """Four-quadrant Riemann data split at (1/2, 1/2).  Per quadrant, in the
    order (x>=1/2,y>=1/2), (x<1/2,y>=1/2), (x<1/2,y<1/2), (x>=1/2,y<1/2), the
    draws are rho ~ U[0.1,1.5], p ~ U[0.1,1.5], u ~ U[-1,1], v ~ U[-1,1].
    Returns conserved (rho, rho u, rho v, E) with E = p/(gamma-1) + rho|u|^2/2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = centres(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    q = np.zeros((4, n, n))
    masks = [(X >= 0.5) & (Y >= 0.5), (X < 0.5) & (Y >= 0.5), (X < 0.5) & (Y < 0.5), (X >= 0.5) & (Y < 0.5)]
    for m in masks:
        rho = rng.uniform(0.1, 1.5)
        p = rng.uniform(0.1, 1.5)
        u = rng.uniform(-1.0, 1.0)
        v = rng.uniform(-1.0, 1.0)
        q[0][m] = rho
        q[1][m] = rho * u
        q[2][m] = rho * v
        q[3][m] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return q


def dam_break_x(nx: int, ny: int = 4, hl: float = 1.0, hr: float = 0.35, x0: float = 0.5) -> np.ndarray:
    """y-invariant dam break: h = hl for x < x0, hr otherwise, at rest."""
    x = centres(nx)
    q = np.zeros((3, ny, nx))
    q[0] = np.where(x < x0, hl, hr)[None, :]
    return q


def sod_x(nx: int, ny: int = 4, gamma: float = GAMMA, x0: float = 0.5) -> np.ndarray:
    """y-invariant Sod-type problem (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1)."""
    x = centres(nx)
    q = np.zeros((4, ny, nx))
    left = x < x0
    q[0] = np.where(left, 1.0, 0.125)[None, :]
    q[3] = np.where(left, 1.0, 0.1)[None, :] / (gamma - 1.0)
    return q


def random_smooth_swe(n: int, seed: int = 0, humps: int | None = None, periodic: bool = True) -> np.ndarray:
    """Multi-hump periodic SWE state for the learned coarse solver: K humps
    (K ~ U{1..4} unless given), each with amplitude +-U[0.05, 0.15], width
    w ~ U[0.005, 0.02] in exp(-r^2 / w), centre ~ U[0,1]^2, distance measured
    periodically.  h = 1 + sum, u = v = 0.  Draw order per hump: amplitude
    magnitude, sign, width, centre."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = int(rng.integers(1, 5)) if humps is None else humps
    x = centres(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    h = np.ones((n, n))
    for _ in range(k):
        a = rng.uniform(0.05, 0.15) * (1.0 if rng.uniform() < 0.5 else -1.0)
        w = rng.uniform(0.005, 0.02)
        cx, cy = rng.uniform(0.0, 1.0, size=2)
        dx = np.abs(X - cx)
        dy = np.abs(Y - cy)
        if periodic:
            dx = np.minimum(dx, 1.0 - dx)
            dy = np.minimum(dy, 1.0 - dy)
        h += a * np.exp(-(dx * dx + dy * dy) / w)
    q = np.zeros((3, n, n))
    q[0] = h
    return q


def random_smooth_euler(n: int, seed: int = 0, humps: int | None = None, gamma: float = GAMMA) -> np.ndarray:
    """Periodic smooth Euler state for the learned Euler step: a uniform
    drift (u, v) ~ U[-0.5, 0.5]^2 carrying K humps (K ~ U{1..4} unless
    given) of density and pressure, each hump with amplitudes +-U[0.05, 0.2]
    (density) and +-U[0.05, 0.2] (pressure) over rho = p = 1 (both stay
    >= 0.2), width w ~ U[0.005, 0.02] in exp(-r^2 / w), centre ~ U[0,1]^2,
    distance measured periodically.  Draw order: u, v, then per hump: density amplitude
    magnitude and sign, pressure amplitude magnitude and sign, width,
    centre.  Returns (rho, rho u, rho v, E)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u, v = rng.uniform(-0.5, 0.5, size=2)
    k = int(rng.integers(1, 5)) if humps is None else humps
    x = centres(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    rho = np.ones((n, n))
    p = np.ones((n, n))
    for _ in range(k):
        ar = rng.uniform(0.05, 0.2) * (1.0 if rng.uniform() < 0.5 else -1.0)
        ap = rng.uniform(0.05, 0.2) * (1.0 if rng.uniform() < 0.5 else -1.0)
        w = rng.uniform(0.005, 0.02)
        cx, cy = rng.uniform(0.0, 1.0, size=2)
        dx = np.abs(X - cx)
        dy = np.abs(Y - cy)
        dx = np.minimum(dx, 1.0 - dx)
        dy = np.minimum(dy, 1.0 - dy)
        e = np.exp(-(dx * dx + dy * dy) / w)
        rho += ar * e
        p += ap * e
    q = np.zeros((4, n, n))
    q[0] = rho
    q[1] = rho * u
    q[2] = rho * v
    q[3] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return q


def uniform_state(n: int, h: float = 1.0, u: float = 0.0, v: float = 0.0) -> np.ndarray:
    q = np.zeros((3, n, n))
    q[0] = h
    q[1] = h * u
    q[2] = h * v
    return q


def sphere_state(centres: np.ndarray, seed: int = 0, h0: float = 1.0, bumps: int = 4, u0: float = 0.0,
                 omega: float = 0.0, g: float = 1.0) -> np.ndarray:
    """Shallow water on the unit sphere in Cartesian form, sampled at given
    cell centres [3][ny][nx] (unit vectors): an eastward solid-body flow
    m = h u0 (z_hat x x) over the depth h0 - (omega u0 + u0^2/2) z^2 / g that
    balances it on a sphere rotating at omega (a steady state), plus `bumps`
    seeded Gaussian depth bumps A exp(-(angle to c)^2 / w^2), A ~ U[0.02, 0.08],
    w ~ U[0.15, 0.35], c uniform on the sphere (draw order per bump: A, w,
    then c as a normalised standard-normal 3-vector).  Returns [4][ny][nx]
    float64: h, hu, hv, hw."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, z = centres
    h = h0 - (omega * u0 + 0.5 * u0 * u0) * z * z / g
    for _ in range(bumps):
        a = rng.uniform(0.02, 0.08)
        w = rng.uniform(0.15, 0.35)
        c = rng.standard_normal(3)
        c = c / np.linalg.norm(c)
        ang = np.arccos(np.clip(c[0] * x + c[1] * y + c[2] * z, -1.0, 1.0))
        h = h + a * np.exp(-(ang * ang) / (w * w))
    q = np.zeros((4,) + x.shape)
    q[0] = h
    q[1] = h * u0 * (-y)
    q[2] = h * u0 * x
    return q
