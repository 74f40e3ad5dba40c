"""Reference (oracle) implementation of the finite-volume method and of the
learned-stencil step, used ONLY as test infrastructure.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.  The classic solver is plain double-precision C
(``fv_oracle.c``, loaded through ctypes); the learned path lives in
``learned.py`` (planar shallow water) and ``learned_euler.py`` (the Euler
system), both double-precision PyTorch CPU operations; the spherical
shallow-water solver is plain C (``sphere_oracle.c``, wrapped by
``sphere.py``).

Each function states the thesis passage it follows ("A Machine Learning
accelerated geophysical fluid solver": sections 2.3-2.5, 3.3, 5.3, 6.2,
eq 2.3-2.28, 3.1-3.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
SRC_PATH = os.path.join(HERE, "fv_oracle.c")
SPHERE_SRC_PATH = os.path.join(HERE, "sphere_oracle.c")

SWE, EULER = 0, 1
PERIODIC, WALL = 0, 1
HLLE, RUSANOV, ROE = 0, 1, 2
MINMOD, FIRST = 0, 1


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no fast-math, OpenMP row loops)."""
    newest = max(os.path.getmtime(SRC_PATH), os.path.getmtime(SPHERE_SRC_PATH))
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < newest:
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
                               "-o", tmp, SRC_PATH, SPHERE_SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Cfg(ctypes.Structure):
    _fields_ = [("eqn", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("flux", ctypes.c_int32),
                ("recon", ctypes.c_int32), ("rk_stages", ctypes.c_int32),
                ("shadow_f32", ctypes.c_int32), ("nthreads", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("cfl", ctypes.c_double),
                ("dt_fixed", ctypes.c_double), ("g", ctypes.c_double), ("gamma", ctypes.c_double)]


@dataclass
class Config:
    eqn: int = SWE
    nx: int = 64
    ny: int = 64
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    flux: int = HLLE
    recon: int = MINMOD
    rk_stages: int = 2
    shadow_f32: int = 0
    nthreads: int = 1
    lx: float = 1.0
    ly: float = 1.0
    cfl: float = 0.4
    dt_fixed: float = 0.0
    g: float = 9.81
    gamma: float = 1.4

    @property
    def nvar(self) -> int:
        return 3 if self.eqn == SWE else 4

    def _c(self) -> _Cfg:
        return _Cfg(self.eqn, self.nx, self.ny, self.bc_x, self.bc_y, self.flux, self.recon,
                    self.rk_stages, self.shadow_f32, self.nthreads, self.lx, self.ly, self.cfl,
                    self.dt_fixed, self.g, self.gamma)


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        d = ctypes.c_double
        dp = P(d)
        cp = P(_Cfg)
        _lib.orc_run.argtypes = [cp, dp, dp, ctypes.c_int64, dp, dp, dp]
        _lib.orc_run.restype = ctypes.c_int
        _lib.orc_step.argtypes = [cp, dp, dp, dp]
        _lib.orc_step.restype = ctypes.c_int
        _lib.orc_rhs.argtypes = [cp, dp, dp, dp]
        _lib.orc_rhs.restype = None
        _lib.orc_dt.argtypes = [cp, dp]
        _lib.orc_dt.restype = d
        _lib.orc_max_rate.argtypes = [cp, dp]
        _lib.orc_max_rate.restype = d
        _lib.orc_totals.argtypes = [cp, dp, dp]
        _lib.orc_totals.restype = None
        _lib.orc_numflux.argtypes = [cp, dp, dp, dp]
        _lib.orc_numflux.restype = None
        _lib.orc_physflux.argtypes = [cp, dp, dp]
        _lib.orc_physflux.restype = None
        _lib.orc_face_fluxes.argtypes = [cp, dp, dp, dp, dp]
        _lib.orc_face_fluxes.restype = None
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _state(cfg: Config, q) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64).copy()
    assert q.shape == (cfg.nvar, cfg.ny, cfg.nx), q.shape
    return q


def _bed(cfg: Config, b):
    if b is None:
        return None
    b = np.ascontiguousarray(b, dtype=np.float64)
    assert b.shape == (cfg.ny, cfg.nx)
    return b


def run(cfg: Config, q, b=None, nsteps: int = 1):
    """Advance ``nsteps`` full steps (section 2.3: eq 2.9/2.23 fluxes, eq 2.18
    reconstruction, eq 2.19/2.20 stages, eq 2.10 time step).  Returns
    ``(q, t, dt_min, dt_max, rc)``; rc = -4 when a cell became inadmissible."""
    q = _state(cfg, q)
    b = _bed(cfg, b)
    c = cfg._c()
    t, lo, hi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    rc = lib().orc_run(ctypes.byref(c), _dp(q), _dp(b), int(nsteps), ctypes.byref(t),
                       ctypes.byref(lo), ctypes.byref(hi))
    return q, t.value, lo.value, hi.value, rc


def rhs(cfg: Config, q, b=None) -> np.ndarray:
    """The spatial operator L(q) (flux divergence plus bed source)."""
    q = _state(cfg, q)
    b = _bed(cfg, b)
    L = np.zeros_like(q)
    c = cfg._c()
    lib().orc_rhs(ctypes.byref(c), _dp(q), _dp(b), _dp(L))
    return L


def dt(cfg: Config, q) -> float:
    c = cfg._c()
    return lib().orc_dt(ctypes.byref(c), _dp(_state(cfg, q)))


def max_rate(cfg: Config, q) -> float:
    c = cfg._c()
    return lib().orc_max_rate(ctypes.byref(c), _dp(_state(cfg, q)))


def totals(cfg: Config, q) -> np.ndarray:
    """Conserved totals per variable and the energy of eq 5.1."""
    out = np.zeros(cfg.nvar + 1)
    c = cfg._c()
    lib().orc_totals(ctypes.byref(c), _dp(_state(cfg, q)), _dp(out))
    return out


def numflux(cfg: Config, sl, sr) -> np.ndarray:
    """Numerical flux of two normal-frame states (eq 2.12, 2.14, 2.16)."""
    sl = np.ascontiguousarray(sl, dtype=np.float64)
    sr = np.ascontiguousarray(sr, dtype=np.float64)
    F = np.zeros(4)
    c = cfg._c()
    lib().orc_numflux(ctypes.byref(c), _dp(sl), _dp(sr), _dp(F))
    return F[: cfg.nvar]


def physflux(cfg: Config, s) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.float64)
    F = np.zeros(4)
    c = cfg._c()
    lib().orc_physflux(ctypes.byref(c), _dp(s), _dp(F))
    return F[: cfg.nvar]


def face_fluxes(cfg: Config, q, b=None):
    """Per-face numerical fluxes: Fx[v, j, i] at faces i-1/2 (i=0..nx) and
    Fy[v, j, i] at faces j-1/2 (j=0..ny)."""
    q = _state(cfg, q)
    b = _bed(cfg, b)
    Fx = np.zeros((cfg.nvar, cfg.ny, cfg.nx + 1))
    Fy = np.zeros((cfg.nvar, cfg.ny + 1, cfg.nx))
    c = cfg._c()
    lib().orc_face_fluxes(ctypes.byref(c), _dp(q), _dp(b), _dp(Fx), _dp(Fy))
    return Fx, Fy
