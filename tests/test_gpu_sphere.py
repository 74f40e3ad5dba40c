"""GPU shallow water on the sphere (sections 2.4 and 3.3) against the oracle
(oracle/sphere_oracle.c) through the C ABI (fv_sphere_*).

Tolerances as the planar path's: FP64 relative L2 <= 1e-12 per variable
(every flux x reconstruction x Runge-Kutta combination), FP32 smooth state
relative L2 <= 1e-5; a fluid at rest held to roundoff; mass conserved in
FP64 totals to 1e-13 (FP64) and 1e-6 (FP32)."""
import itertools

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
def S(orc):
    from oracle import sphere

    return sphere


def state(S, n, seed, u0=0.3, omega=0.5):
    cen, *_ = S.geometry(S.Config(n=n))
    return I.sphere_state(cen, seed=seed, u0=u0, omega=omega), cen


def test_centres_match_oracle(fv, S):
    q0, cen = state(S, 16, 1)
    s = fv.SphereSolver(q0, prec=fv.FV_F64, g=1.0)
    got = s.centres()
    s.close()
    print(f"[sphere] centres max diff {np.abs(got - cen).max():.2e}", flush=True)
    assert np.abs(got - cen).max() <= 1e-14


VARIANTS = list(itertools.product([0, 1, 2], [0, 1], [1, 2, 3]))


@pytest.mark.parametrize("flux,recon,rk", VARIANTS)
def test_fp64_parity(fv, S, flux, recon, rk):
    n, steps = 12, 15
    q0, _ = state(S, n, 2)
    kw = dict(flux=flux, recon=recon, rk_stages=rk, g=1.0, omega=0.5)
    print(f"[gpu] sphere FP64 n={n} {kw} x{steps}", flush=True)
    s = fv.SphereSolver(q0, prec=fv.FV_F64, **kw)
    s.run(steps)
    t, k = s.time()
    out = s.state()
    s.close()
    ref, t_ref, rc = S.run(S.Config(n=n, **kw), q0, steps)
    assert rc == 0 and k == steps
    assert abs(t - t_ref) <= 1e-13 * t_ref
    errs = rel_errors(out, ref)
    assert np.all(errs <= 1e-12), errs


@pytest.mark.parametrize("n", [49, 70])
def test_fp64_parity_ragged_tiles(fv, S, n):
    """Grids of several stage tiles (32 x 8 cells) with ragged last tiles in
    both directions: 98 x 49 cells leave 2 columns and 1 row, 140 x 70 leave
    12 columns and 6 rows; the tiles' halos cross the periodic seam and the
    mirrored edges y = -+1."""
    steps = 8
    q0, _ = state(S, n, 3)
    kw = dict(flux=0, recon=0, rk_stages=2, g=1.0, omega=0.5)
    print(f"[gpu] sphere FP64 n={n} {kw} x{steps}", flush=True)
    s = fv.SphereSolver(q0, prec=fv.FV_F64, **kw)
    s.run(steps)
    t, k = s.time()
    out = s.state()
    s.close()
    ref, t_ref, rc = S.run(S.Config(n=n, **kw), q0, steps)
    assert rc == 0 and k == steps
    assert abs(t - t_ref) <= 1e-13 * t_ref
    errs = rel_errors(out, ref)
    print(f"[sphere ragged] n={n} errs {errs}", flush=True)
    assert np.all(errs <= 1e-12), errs


def test_fp32_smooth_parity_and_mass(fv, S):
    n, steps = 48, 100
    q0, _ = state(S, n, 3)
    kw = dict(g=1.0, omega=0.5)
    s = fv.SphereSolver(q0, prec=fv.FV_F32, **kw)
    m0 = s.totals()
    s.run(steps)
    m1 = s.totals()
    t, k = s.time()
    out = s.state()
    s.close()
    c = S.Config(n=n, nthreads=8, **kw)
    ref, t_ref, rc = S.run(c, q0, steps)
    print(f"[sphere fp32] state rel L2 {state_rel(out, ref):.2e} per var {rel_errors(out, ref)}; "
          f"mass {m0[0]:.9e} -> {m1[0]:.9e}", flush=True)
    assert rc == 0 and k == steps and abs(t - t_ref) <= 1e-5 * t_ref
    assert state_rel(out, ref) <= 1e-5
    assert abs(m1[0] - m0[0]) <= 1e-6 * m0[0]
    to = S.totals(c, q0.astype(np.float32).astype(np.float64))
    assert abs(m0[0] - to[0]) <= 1e-12 * to[0] and abs(m0[1] - to[1]) <= 1e-12 * to[1]


def test_fluid_at_rest_and_mass_fp64(fv, S):
    n = 16
    q = np.zeros((4, n, 2 * n))
    q[0] = 1.3
    s = fv.SphereSolver(q, prec=fv.FV_F64, g=1.0, omega=0.7)
    s.run(20)
    out = s.state()
    s.close()
    assert np.abs(out[0] - 1.3).max() <= 1e-14 and np.abs(out[1:]).max() <= 1e-14
    q0, _ = state(S, n, 4)
    s = fv.SphereSolver(q0, prec=fv.FV_F64, g=1.0, omega=0.5)
    m0 = s.totals()[0]
    s.run(40)
    m1 = s.totals()[0]
    s.close()
    assert abs(m1 - m0) <= 1e-13 * m0


def test_inadmissible_initial_state_rejected(fv, S):
    q0, _ = state(S, 8, 5)
    q0[0, 3, 4] = -0.2
    with pytest.raises(fv.FvError) as e:
        fv.SphereSolver(q0, prec=fv.FV_F32, g=1.0)
    assert e.value.code == fv.FV_E_INADMISSIBLE
