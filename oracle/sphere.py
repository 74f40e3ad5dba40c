"""Python access to the spherical shallow-water oracle (sphere_oracle.c).
TEST INFRASTRUCTURE ONLY: used by tests/ and nothing in the product path.

Thesis section 2.4 (logically rectangular grid on the sphere) and section 3.3
(shallow water in three-dimensional Cartesian form on the sphere, eq 3.1
correction, eq 3.2 source).  State layout [4][n][2n]: h, hu, hv, hw (Cartesian
momenta), rows along computational y, columns along computational x."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import lib as _orc_lib

HLLE, RUSANOV, ROE = 0, 1, 2
MINMOD, FIRST = 0, 1


class _Cfg(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("flux", ctypes.c_int32), ("recon", ctypes.c_int32),
                ("rk_stages", ctypes.c_int32), ("nthreads", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("cfl", ctypes.c_double), ("dt_fixed", ctypes.c_double), ("g", ctypes.c_double),
                ("omega", ctypes.c_double)]


@dataclass
class Config:
    n: int = 16
    flux: int = HLLE
    recon: int = MINMOD
    rk_stages: int = 2
    nthreads: int = 1
    cfl: float = 0.4
    dt_fixed: float = 0.0
    g: float = 1.0
    omega: float = 0.0

    def _c(self):
        return _Cfg(self.n, self.flux, self.recon, self.rk_stages, self.nthreads, 0, self.cfl, self.dt_fixed,
                    self.g, self.omega)


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _orc_lib()
        P = ctypes.POINTER
        d = ctypes.c_double
        dp = P(d)
        cp = P(_Cfg)
        _lib.sph_rhs.argtypes = [cp, dp, dp]
        _lib.sph_rhs.restype = None
        _lib.sph_run.argtypes = [cp, dp, ctypes.c_int64, dp]
        _lib.sph_run.restype = ctypes.c_int
        _lib.sph_dt.argtypes = [cp, dp]
        _lib.sph_dt.restype = d
        _lib.sph_geometry.argtypes = [cp, dp, dp, dp, dp]
        _lib.sph_geometry.restype = None
        _lib.sph_face.argtypes = [cp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        _lib.sph_face.restype = None
        _lib.sph_point.argtypes = [d, d, dp]
        _lib.sph_point.restype = None
        _lib.sph_totals.argtypes = [cp, dp, dp]
        _lib.sph_totals.restype = None
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _state(cfg, q):
    q = np.ascontiguousarray(q, dtype=np.float64).copy()
    assert q.shape == (4, cfg.n, 2 * cfg.n), q.shape
    return q


def point(xc, yc):
    p = np.zeros(3)
    lib().sph_point(float(xc), float(yc), _dp(p))
    return p


def geometry(cfg):
    """Cell centres [3][n][2n], areas, perimeters, and the sums of outward
    edge normals times edge lengths [3][n][2n]."""
    n = cfg.n
    c = np.zeros((3, n, 2 * n))
    a = np.zeros((n, 2 * n))
    p = np.zeros((n, 2 * n))
    N = np.zeros((3, n, 2 * n))
    lib().sph_geometry(ctypes.byref(cfg._c()), _dp(c), _dp(a), _dp(p), _dp(N))
    return c, a, p, N


def face(cfg, axis, i, j):
    out = np.zeros(10)
    lib().sph_face(ctypes.byref(cfg._c()), axis, i, j, _dp(out))
    return out[0:3], out[3:6], out[6:9], out[9]


def rhs(cfg, q):
    q = _state(cfg, q)
    L = np.zeros_like(q)
    lib().sph_rhs(ctypes.byref(cfg._c()), _dp(q), _dp(L))
    return L


def run(cfg, q, nsteps):
    """Advance nsteps full steps; returns (q, t, rc)."""
    q = _state(cfg, q)
    t = ctypes.c_double()
    rc = lib().sph_run(ctypes.byref(cfg._c()), _dp(q), int(nsteps), ctypes.byref(t))
    return q, t.value, rc


def dt(cfg, q):
    return lib().sph_dt(ctypes.byref(cfg._c()), _dp(_state(cfg, q)))


def totals(cfg, q):
    out = np.zeros(2)
    lib().sph_totals(ctypes.byref(cfg._c()), _dp(_state(cfg, q)), _dp(out))
    return out
