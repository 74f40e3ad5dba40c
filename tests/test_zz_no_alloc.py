"""The allocation-free entry point (fv_run_noalloc: workspace in the library's
device array instead of the caller's) against fv_init + fv_run on the same
inputs: the same kernels run, so states, simulated time and step counts are
bit-identical.  Two calls in a row, the second on a smaller grid (the array
keeps the first call's contents), through the batched FP32 path and the
per-stage FP64 path, then a call whose initial state is not admissible."""
import numpy as np
import pytest
import torch

from paper_2602_08670_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fv():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2602_08670_amd import fv as F

    return F


def run_noalloc(fv, q0, b, steps, **kw):
    dt = torch.float64 if kw.get("prec", fv.FV_F32) == fv.FV_F64 else torch.float32
    q = torch.tensor(q0, dtype=dt, device="cuda").contiguous()
    bed = None if b is None else torch.tensor(b, dtype=dt, device="cuda").contiguous()
    info = torch.zeros(3, dtype=torch.float64, device="cuda")  # fv_run_info: t, steps, flag + reserved
    nvar, ny, nx = q0.shape
    cfg = fv.make_config(nx=nx, ny=ny, eqn=fv.FV_SWE if nvar == 3 else fv.FV_EULER, **kw)
    stream = torch.cuda.current_stream()
    print(f"[gpu] fv_run_noalloc {nvar}x{ny}x{nx} {kw} steps={steps}", flush=True)
    fv.fv_run_noalloc(cfg, q.data_ptr(), None if bed is None else bed.data_ptr(), steps, stream.cuda_stream,
                      info.data_ptr())
    torch.cuda.synchronize()
    raw = info.cpu().numpy()
    t = float(raw[0])
    n = int(raw[1:2].view(np.int64)[0])
    bad = int(raw[2:3].view(np.int32)[0])
    return q.double().cpu().numpy(), t, n, bad


def run_reference(fv, q0, b, steps, **kw):
    s = fv.Solver(q0, b, **kw)
    s.run(steps)
    out = s.state()
    t, n = s.time()
    s.close()
    return out, t, n


def test_noalloc_equals_workspace_path_twice_then_smaller(fv):
    q0, b = I.swe_bathy(1024, seed=0)
    kw = dict(prec=fv.FV_F32, bc_x=fv.FV_BC_WALL, bc_y=fv.FV_BC_WALL, h_ref=1.0)
    got, t, n, bad = run_noalloc(fv, q0, b, 30, **kw)
    ref, t_ref, n_ref = run_reference(fv, q0, b, 30, **kw)
    print(f"[noalloc 1024^2 bed] t {t} vs {t_ref}, steps {n} vs {n_ref}", flush=True)
    assert bad == 0 and n == n_ref == 30 and t == t_ref
    assert np.array_equal(got, ref)

    q0 = I.euler_quadrants(96, seed=2)[:, :80].copy()
    kw = dict(prec=fv.FV_F64, flux=fv.FV_FLUX_RUSANOV, rk_stages=3, ly=80 / 96)
    got, t, n, bad = run_noalloc(fv, q0, None, 25, **kw)
    ref, t_ref, n_ref = run_reference(fv, q0, None, 25, **kw)
    print(f"[noalloc 80x96 Euler FP64 RK3] t {t} vs {t_ref}, steps {n} vs {n_ref}", flush=True)
    assert bad == 0 and n == n_ref == 25 and t == t_ref
    assert np.array_equal(got, ref)


def test_noalloc_reports_inadmissible_initial_state(fv):
    """A negative depth in the initial state: the flag comes back through the
    device record, no step is taken and the state is left as it was."""
    q0 = I.gaussian_hump(64)
    q0[0, 5, 7] = -0.1
    got, t, n, bad = run_noalloc(fv, q0, None, 5, prec=fv.FV_F32, h_ref=1.0)
    assert bad == 1 and n == 0 and t == 0.0
    assert np.array_equal(got, q0.astype(np.float32).astype(np.float64))
