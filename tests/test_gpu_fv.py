"""GPU <-> oracle parity of the classic finite-volume path, through the C ABI.

Tolerances: FP64 path relative L2 <= 1e-12 per variable; FP32 on smooth cases
relative L2 <= 1e-5 of the state vector, and per variable within twice the
error that FP32 storage alone causes (the oracle in FP32-shadow mode: double
arithmetic, state rounded to float after every stage); FP32 on shock cases
relative L1 <= 1e-4; conserved totals accumulated in FP64."""
import itertools
import math

import numpy as np
import pytest

from parity import max_rel, rel_errors, state_rel
from paper_2602_08670_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fv():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2602_08670_amd import fv as F

    return F


def gpu_run(fv, q0, b=None, nsteps=1, **kw):
    print(f"[gpu] shape={np.shape(q0)} bathy={b is not None} steps={nsteps} cfg={kw}", flush=True)
    s = fv.Solver(q0, b, **kw)
    s.run(nsteps)
    t, n = s.time()
    out = s.state()
    tot = s.totals()
    s.close()
    return out, t, n, tot


def orc_cfg(orc, q, **kw):
    nvar, ny, nx = np.shape(q)
    kw.setdefault("eqn", 0 if nvar == 3 else 1)
    return orc.Config(nx=nx, ny=ny, nthreads=8, **kw)


# ------------------------------------------------------------ FP64 path

def test_config1_fp64(fv, orc):
    """Gaussian hump 64^2, periodic, FP64, CFL 0.4, 200 steps: rel L2 <= 1e-12."""
    q0 = I.gaussian_hump(64)
    out, t, n, tot = gpu_run(fv, q0, nsteps=200, prec=fv.FV_F64)
    ref, t_ref, *_ = orc.run(orc_cfg(orc, q0), q0, None, 200)
    assert n == 200
    assert abs(t - t_ref) <= 1e-13 * t_ref
    assert max_rel(out, ref) <= 1e-12, rel_errors(out, ref)
    t0 = orc.totals(orc_cfg(orc, q0), q0)
    assert abs(tot[0] - t0[0]) <= 1e-13 * t0[0]


VARIANTS = list(itertools.product(
    ["swe", "swe_bed", "euler"], [0, 1, 2], [0, 1], [1, 2, 3], [(0, 0), (1, 1), (0, 1)]))


@pytest.mark.parametrize("eq,flux,recon,rk,bc", VARIANTS)
def test_variants_fp64_ragged(fv, orc, eq, flux, recon, rk, bc):
    """Every flux x reconstruction x RK x boundary combination in FP64 on a
    72 x 20 grid (ragged against the 64 x 8 tile), 15 steps: rel L2 <= 1e-12."""
    nx, ny = 72, 20
    b = None
    if eq == "euler":
        q0 = I.euler_quadrants(72, seed=3)[:, :20, :].copy()
    else:
        q, b = I.swe_bathy(72, seed=2)
        q0 = q[:, :20, :].copy()
        b = b[:20, :].copy()
        q0[1] = 0.05 * np.sin(np.arange(nx) / 5.0)[None, :]
        q0[2] = 0.03 * np.cos(np.arange(ny) / 3.0)[:, None]
        if eq == "swe":
            b = None
    kw = dict(flux=flux, recon=recon, rk_stages=rk, bc_x=bc[0], bc_y=bc[1])
    out, t, n, _ = gpu_run(fv, q0, b, nsteps=15, prec=fv.FV_F64, lx=1.0, ly=ny / nx, **kw)
    ref, t_ref, *_ , rc = orc.run(orc_cfg(orc, q0, lx=1.0, ly=ny / nx, **kw), q0, b, 15)
    assert rc == 0
    assert abs(t - t_ref) <= 1e-13 * t_ref
    assert max_rel(out, ref) <= 1e-12, rel_errors(out, ref)


@pytest.mark.parametrize("eqn,flux", [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1), (1, 2)])
def test_face_fluxes_tiny_grid(fv, orc, eqn, flux):
    """Face-by-face comparison on a 5 x 4 grid (FP64)."""
    rng = np.random.Generator(np.random.PCG64(9))
    if eqn == 0:
        q0 = np.stack([rng.uniform(0.5, 1.5, (4, 5)), rng.uniform(-0.5, 0.5, (4, 5)), rng.uniform(-0.5, 0.5, (4, 5))])
    else:
        r = rng.uniform(0.5, 1.5, (4, 5))
        u, v = rng.uniform(-0.5, 0.5, (2, 4, 5))
        p = rng.uniform(0.5, 1.5, (4, 5))
        q0 = np.stack([r, r * u, r * v, p / 0.4 + 0.5 * r * (u * u + v * v)])
    s = fv.Solver(q0, prec=fv.FV_F64, flux=flux, bc_x=fv.FV_BC_WALL, bc_y=fv.FV_BC_PERIODIC)
    fx, fy = s.face_fluxes()
    s.close()
    ox, oy = orc.face_fluxes(orc.Config(eqn=eqn, nx=5, ny=4, flux=flux, bc_x=1, bc_y=0), q0)
    assert np.abs(fx - ox).max() <= 1e-13 * np.abs(ox).max()
    assert np.abs(fy - oy).max() <= 1e-13 * np.abs(oy).max()


def test_lake_at_rest_fp64_and_fp32(fv):
    q0, b = I.lake_at_rest(128, seed=0)
    out, *_ = gpu_run(fv, q0, b, nsteps=200, prec=fv.FV_F64, bc_x=1, bc_y=1)
    assert np.abs(out[1:]).max() <= 1e-12 * math.sqrt(9.81)
    assert np.abs(out[0] + b - 1.0).max() <= 1e-13
    out, *_ = gpu_run(fv, q0, b, nsteps=200, prec=fv.FV_F32, bc_x=1, bc_y=1)
    b32 = b.astype(np.float32).astype(np.float64)
    assert np.abs(out[1:]).max() <= 1e-5
    assert np.abs(out[0] + b32 - (q0[0].astype(np.float32) + b32)).max() <= 1e-6


def test_conservation_periodic_fp32_fp64(fv):
    q0 = I.euler_quadrants(128, seed=4)
    for prec, tol in ((1, 1e-13), (0, 1e-6)):
        s = fv.Solver(q0, prec=prec)
        t0 = s.totals()
        s.run(100)
        t1 = s.totals()
        s.close()
        assert np.abs(t1[:4] - t0[:4]).max() <= tol * np.abs(t0[:4]).max(), (prec, t0, t1)


# ------------------------------------------------------------ FP32 path

def fp32_smooth_check(orc, out, q0, b, nsteps, **kw):
    ref, t_ref, *_ = orc.run(orc_cfg(orc, q0, **kw), q0, b, nsteps)
    c = orc_cfg(orc, q0, shadow_f32=1, **kw)
    b32 = None if b is None else b.astype(np.float32).astype(np.float64)
    shadow, *_ = orc.run(c, q0.astype(np.float32).astype(np.float64), b32, nsteps)
    floor = rel_errors(shadow, ref)
    got = rel_errors(out, ref)
    print(f"[fp32] state rel L2 {state_rel(out, ref):.2e}; per var {got} vs FP32-storage floor {floor}", flush=True)
    assert state_rel(out, ref) <= 1e-5
    assert np.all(got <= np.maximum(2.0 * floor, 1e-6)), (got, floor)
    return t_ref


def test_fp32_smooth_256(fv, orc):
    """Config-1 initial data at 256^2, FP32, 200 steps."""
    q0 = I.gaussian_hump(256)
    out, t, n, _ = gpu_run(fv, q0, nsteps=200, prec=fv.FV_F32)
    t_ref = fp32_smooth_check(orc, out, q0, None, 200)
    assert abs(t - t_ref) <= 1e-6 * t_ref


@pytest.mark.parametrize("flux", [0, 1, 2])
def test_fp32_euler_shock_256(fv, orc, flux):
    """Seeded four-quadrant Euler data at 256^2, walls, FP32, 100 steps:
    relative L1 <= 1e-4."""
    q0 = I.euler_quadrants(256, seed=0)
    out, t, n, _ = gpu_run(fv, q0, nsteps=100, prec=fv.FV_F32, flux=flux, bc_x=1, bc_y=1)
    ref, t_ref, *_ = orc.run(orc_cfg(orc, q0, flux=flux, bc_x=1, bc_y=1), q0, None, 100)
    assert abs(t - t_ref) <= 1e-5 * t_ref
    assert max_rel(out, ref, order=1) <= 1e-4, rel_errors(out, ref, 1)


def test_fp32_dam_break_2d_shock(fv, orc):
    """Stoker dam break along x on 512 x 8 in FP32: relative L1 <= 1e-4."""
    q0 = I.dam_break_x(512, 8)
    kw = dict(bc_x=1, bc_y=1, ly=8 / 512)
    out, *_ = gpu_run(fv, q0, nsteps=300, prec=fv.FV_F32, **kw)
    ref, *_ = orc.run(orc_cfg(orc, q0, **kw), q0, None, 300)
    assert max_rel(out, ref, order=1) <= 1e-4, rel_errors(out, ref, 1)


def test_fp32_swe_bathy_1024_full_size(fv, orc):
    """The 1024^2 shallow-water workload over the seeded bed, walls, in the
    launch configuration the benchmark times, for all of its 1000 steps: after
    10 steps against the oracle (FP32 smooth tolerance, per variable within 2x
    the FP32-storage floor), after 1000 steps against the oracle's 1000-step
    FP64 run (state relative L2 <= 1e-5, simulated time 1e-6), and the FP64
    totals of the GPU state (mass, both momenta, eq 5.1 energy) against the
    oracle's totals of its own state: mass to 2e-6 of its initial value, the
    energy and the momenta to 1e-6 of the energy."""
    q0, b = I.swe_bathy(1024, seed=0)
    kw = dict(bc_x=1, bc_y=1)
    s = fv.Solver(q0, b, prec=fv.FV_F32, **kw)
    m0 = s.totals()[0]
    s.run(10)
    out = s.state()
    fp32_smooth_check(orc, out, q0, b, 10, **kw)
    s.run(990)
    t, n = s.time()
    tot = s.totals()
    out = s.state()
    s.close()
    assert n == 1000
    assert abs(tot[0] - m0) <= 2e-6 * m0
    c = orc_cfg(orc, q0, **kw)
    c.nthreads = 16
    print("[oracle] 1024^2 shallow water over the bed, 1000 steps (FP64, 16 threads)", flush=True)
    ref, t_ref, *_, rc = orc.run(c, q0, b, 1000)
    assert rc == 0
    tref = orc.totals(c, ref)
    print(f"[fp32 1000 steps] state rel L2 {state_rel(out, ref):.2e}; per var {rel_errors(out, ref)}; "
          f"totals gpu {tot} oracle {tref}", flush=True)
    assert abs(t - t_ref) <= 1e-6 * t_ref
    assert state_rel(out, ref) <= 1e-5
    assert abs(tot[0] - tref[0]) <= 2e-6 * tref[0]
    assert np.abs(tot[1:] - tref[1:]).max() <= 1e-6 * tref[3]


@pytest.mark.parametrize("eqn", [0, 1])
def test_totals_every_output_matches_oracle(fv, orc, eqn):
    """fv_totals returns the nvar conserved totals and the eq 5.1 energy in
    FP64; each equals the oracle's totals of the same cell values to 1e-13 of
    the largest total (two FP64 sums in different orders): the initial state
    in FP64 and in FP32 (the FP32 values widened exactly), and the GPU's own
    state after 5 steps.  Shallow water: the config-1 hump moving at (0.3, -0.2);
    Euler: seeded four-quadrant data."""
    if eqn == 0:
        q0 = I.gaussian_hump(96)
        q0[1], q0[2] = 0.3 * q0[0], -0.2 * q0[0]
    else:
        q0 = I.euler_quadrants(96, seed=1)
    c = orc_cfg(orc, q0)
    for prec in (fv.FV_F64, fv.FV_F32):
        s = fv.Solver(q0, prec=prec)
        got = s.totals()
        qv = q0 if prec == fv.FV_F64 else q0.astype(np.float32).astype(np.float64)
        ref = orc.totals(c, qv)
        print(f"[totals eqn={eqn} prec={prec}] gpu {got} oracle {ref}", flush=True)
        assert got.shape == (q0.shape[0] + 1,)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), (got, ref)
        s.run(5)
        got = s.totals()
        ref = orc.totals(c, s.state())
        s.close()
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), (got, ref)


def test_fp32_euler_1024_full_size(fv, orc):
    """The 1024^2 four-quadrant Euler workload, 5 steps against the oracle
    (rel L1 <= 1e-4), then 500 steps with mass and energy conserved."""
    q0 = I.euler_quadrants(1024, seed=0)
    kw = dict(bc_x=1, bc_y=1)
    s = fv.Solver(q0, prec=fv.FV_F32, **kw)
    t0 = s.totals()
    s.run(5)
    out = s.state()
    ref, *_ = orc.run(orc_cfg(orc, q0, **kw), q0, None, 5)
    assert max_rel(out, ref, order=1) <= 1e-4, rel_errors(out, ref, 1)
    s.run(495)
    t1 = s.totals()
    t, n = s.time()
    s.close()
    assert n == 500
    assert abs(t1[0] - t0[0]) <= 2e-6 * t0[0]
    assert abs(t1[3] - t0[3]) <= 2e-6 * t0[3]


# ------------------------------------------------------- determinism / errors

def test_bitwise_repeatable(fv):
    q0, b = I.swe_bathy(200, seed=5)
    a, *_ = gpu_run(fv, q0, b, nsteps=50, prec=fv.FV_F32, bc_x=1, bc_y=1)
    c, *_ = gpu_run(fv, q0, b, nsteps=50, prec=fv.FV_F32, bc_x=1, bc_y=1)
    assert np.array_equal(a, c)


def test_inadmissible_initial_state_rejected(fv):
    q0 = I.gaussian_hump(32)
    q0[0, 3, 4] = -0.1
    with pytest.raises(fv.FvError) as e:
        fv.Solver(q0, prec=fv.FV_F32)
    assert e.value.code == fv.FV_E_INADMISSIBLE


def test_set_state_and_resume_bitwise(fv):
    """N steps straight equal N/2 steps, checkpoint (state + reference depth),
    a new handle, N/2 more steps; and fv_set_state on the same handle."""
    q0 = I.gaussian_hump(96)
    a, *_ = gpu_run(fv, q0, nsteps=40, prec=fv.FV_F32)
    s = fv.Solver(q0, prec=fv.FV_F32)
    s.run(20)
    mid = s.state()
    href = s.reference_depth()
    s.set_state(mid)
    s.run(20)
    c = s.state()
    s.close()
    s = fv.Solver(mid.astype(np.float32), prec=fv.FV_F32, h_ref=href)
    s.run(20)
    b = s.state()
    s.close()
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)
