"""Thin Python binding of libfv (include/fv.h): argument marshalling only.

Every entry point keeps the C name (fv_init, fv_step, fv_run, ...).  Device
memory and streams come from PyTorch; all computation runs in the HIP
kernels of libfv.so.  If the library is not built the import of this module
raises immediately -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfv.so")

FV_OK, FV_E_INVALID, FV_E_NOMEM, FV_E_HIP, FV_E_INADMISSIBLE, FV_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
FV_SWE, FV_EULER = 0, 1
FV_F32, FV_F64 = 0, 1
FV_BC_PERIODIC, FV_BC_WALL = 0, 1
FV_FLUX_HLLE, FV_FLUX_RUSANOV, FV_FLUX_ROE = 0, 1, 2
FV_RECON_MINMOD, FV_RECON_FIRST = 0, 1


class FvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fv status {code}: {msg}")
        self.code = code


class fv_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("eqn", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("bc_x", ctypes.c_int32),
                ("bc_y", ctypes.c_int32), ("flux", ctypes.c_int32), ("recon", ctypes.c_int32),
                ("rk_stages", ctypes.c_int32), ("learned", ctypes.c_int32), ("lx", ctypes.c_double),
                ("ly", ctypes.c_double), ("cfl", ctypes.c_double), ("dt_fixed", ctypes.c_double),
                ("g", ctypes.c_double), ("gamma", ctypes.c_double), ("h_ref", ctypes.c_double)]


def make_config(eqn=FV_SWE, prec=FV_F32, nx=64, ny=64, bc_x=FV_BC_PERIODIC, bc_y=FV_BC_PERIODIC,
                flux=FV_FLUX_HLLE, recon=FV_RECON_MINMOD, rk_stages=2, lx=1.0, ly=1.0, cfl=0.4,
                dt_fixed=0.0, g=9.81, gamma=1.4, h_ref=0.0, learned=0) -> fv_config:
    return fv_config(ctypes.sizeof(fv_config), eqn, prec, nx, ny, bc_x, bc_y, flux, recon, rk_stages, learned,
                     lx, ly, cfl, dt_fixed, g, gamma, h_ref)


class fv_sphere_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("prec", ctypes.c_int32), ("n", ctypes.c_int32),
                ("flux", ctypes.c_int32), ("recon", ctypes.c_int32), ("rk_stages", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("pad", ctypes.c_int32), ("cfl", ctypes.c_double),
                ("dt_fixed", ctypes.c_double), ("g", ctypes.c_double), ("omega", ctypes.c_double)]


class fv_euler_learned_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("B", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("flux", ctypes.c_int32), ("order", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("gamma", ctypes.c_double),
                ("dt", ctypes.c_double), ("mean", ctypes.c_float * 4), ("inv_std", ctypes.c_float * 4)]


def make_euler_learned_config(B, nx, ny, dt, flux=FV_FLUX_HLLE, order=1, lx=1.0, ly=1.0, gamma=1.4,
                              mean=(1.0, 0.0, 0.0, 2.5), inv_std=(8.0, 4.0, 4.0, 2.0)) -> fv_euler_learned_config:
    return fv_euler_learned_config(ctypes.sizeof(fv_euler_learned_config), B, nx, ny, flux, order, lx, ly, gamma,
                                   dt, (ctypes.c_float * 4)(*mean), (ctypes.c_float * 4)(*inv_std))


class fv_euler_train_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("B", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("T", ctypes.c_int32), ("flux", ctypes.c_int32), ("lx", ctypes.c_double),
                ("ly", ctypes.c_double), ("gamma", ctypes.c_double), ("dt", ctypes.c_double),
                ("scale", ctypes.c_float * 4), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


def make_euler_train_config(B, nx, ny, T, dt, flux=FV_FLUX_HLLE, lx=1.0, ly=1.0, gamma=1.4,
                            scale=(0.1, 0.1, 0.1, 0.2), lr=1e-3, beta1=0.9, beta2=0.999,
                            eps=1e-8) -> fv_euler_train_config:
    return fv_euler_train_config(ctypes.sizeof(fv_euler_train_config), B, nx, ny, T, flux, lx, ly, gamma, dt,
                                 (ctypes.c_float * 4)(*scale), lr, beta1, beta2, eps)


def make_sphere_config(n, prec=FV_F32, flux=FV_FLUX_HLLE, recon=FV_RECON_MINMOD, rk_stages=2, cfl=0.4,
                       dt_fixed=0.0, g=1.0, omega=0.0) -> fv_sphere_config:
    return fv_sphere_config(ctypes.sizeof(fv_sphere_config), prec, n, flux, recon, rk_stages, 0, 0, cfl, dt_fixed,
                            g, omega)


class fv_run_info(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("steps", ctypes.c_int64), ("inadmissible", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class fv_model_desc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("hidden", ctypes.c_int32), ("order", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("mean", ctypes.c_float * 3), ("inv_std", ctypes.c_float * 3)]


class fv_learned_stats(ctypes.Structure):
    _fields_ = [("fallback_faces", ctypes.c_int64), ("redone_steps", ctypes.c_int64)]


class fv_train_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("B", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("T", ctypes.c_int32), ("flux", ctypes.c_int32), ("lx", ctypes.c_double),
                ("ly", ctypes.c_double), ("dt", ctypes.c_double), ("g", ctypes.c_double), ("h_ref", ctypes.c_double),
                ("scale", ctypes.c_float * 3), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("direct", ctypes.c_int32),
                ("blend", ctypes.c_int32)]


class fv_server_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_solves", ctypes.c_int32),
                ("steps_per_round", ctypes.c_int32), ("direct", ctypes.c_int32), ("max_items", ctypes.c_uint64),
                ("model", ctypes.c_void_p), ("learned_split", ctypes.c_int32), ("learned_layered", ctypes.c_int32),
                ("act_pixels", ctypes.c_uint64), ("max_bypass", ctypes.c_int32), ("reserved0", ctypes.c_int32)]


class fv_request(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("eqn", ctypes.c_int32), ("n", ctypes.c_int32),
                ("bc", ctypes.c_int32), ("steps", ctypes.c_int64), ("cfl", ctypes.c_double), ("g", ctypes.c_double),
                ("gamma", ctypes.c_double), ("h_ref", ctypes.c_double), ("q0", ctypes.c_void_p),
                ("bed", ctypes.c_void_p), ("learned", ctypes.c_int32), ("reserved1", ctypes.c_int32),
                ("dt_fixed", ctypes.c_double), ("lx", ctypes.c_double)]


class fv_request_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("rounds_queued", ctypes.c_int32), ("steps_done", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("sim_time", ctypes.c_double), ("fallback_faces", ctypes.c_int64), ("redone_steps", ctypes.c_int64)]


class fv_server_stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("graph_replays", ctypes.c_int64), ("grid_updates", ctypes.c_int64),
                ("graphs_captured", ctypes.c_int32), ("layered_rounds", ctypes.c_int32), ("host_launch_s", ctypes.c_double),
                ("host_wait_s", ctypes.c_double), ("host_capture_s", ctypes.c_double),
                ("host_admit_s", ctypes.c_double), ("host_retire_s", ctypes.c_double)]


def make_model_desc(mean=(1.0, 0.0, 0.0), inv_std=(10.0, 10.0, 10.0), order=1, hidden=32) -> fv_model_desc:
    d = fv_model_desc()
    d.struct_size = ctypes.sizeof(fv_model_desc)
    d.hidden = hidden
    d.order = order
    d.reserved0 = 0
    for i in range(3):
        d.mean[i] = mean[i]
        d.inv_std[i] = inv_std[i]
    return d


def _load():
    # libfv must bind to the HIP runtime instance that owns the device memory
    # and streams it is handed: PyTorch ships its own libamdhip64 (same
    # soname), so it is loaded first and the library's dependency resolves to it.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    cp = ctypes.POINTER(fv_config)
    sig = {
        "fv_nvar": ([cp], ctypes.c_int),
        "fv_workspace_bytes": ([cp], ctypes.c_size_t),
        "fv_init": ([cp, vp, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)], st),
        "fv_step": ([vp], st),
        "fv_run": ([vp, i64], st),
        "fv_time": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)], st),
        "fv_totals": ([vp, ctypes.POINTER(ctypes.c_double)], st),
        "fv_get_state": ([vp, vp, ctypes.c_int], st),
        "fv_set_state": ([vp, vp, ctypes.c_int], st),
        "fv_state_ptr": ([vp], vp),
        "fv_reference_depth": ([vp], ctypes.c_double),
        "fv_set_stream": ([vp, vp], st),
        "fv_face_fluxes": ([vp, vp, vp], st),
        "fv_destroy": ([vp], None),
        "fv_noalloc_bytes": ([cp], ctypes.c_size_t),
        "fv_sphere_workspace_bytes": ([ctypes.POINTER(fv_sphere_config)], ctypes.c_size_t),
        "fv_sphere_init": ([ctypes.POINTER(fv_sphere_config), vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)], st),
        "fv_sphere_run": ([vp, i64], st),
        "fv_sphere_time": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)], st),
        "fv_sphere_centres": ([vp, vp], st),
        "fv_sphere_totals": ([vp, ctypes.POINTER(ctypes.c_double)], st),
        "fv_sphere_destroy": ([vp], None),
        "fv_run_noalloc": ([cp, vp, vp, i64, vp, vp], st),
        "fv_euler_net_param_count": ([], ctypes.c_size_t),
        "fv_euler_learned_workspace_bytes": ([ctypes.POINTER(fv_euler_learned_config)], ctypes.c_size_t),
        "fv_euler_learned_create": ([ctypes.POINTER(fv_euler_learned_config), vp, vp, ctypes.c_size_t, vp,
                                     ctypes.POINTER(vp)], st),
        "fv_euler_learned_update": ([vp], st),
        "fv_euler_learned_forward": ([vp, vp, vp], st),
        "fv_euler_learned_forward_tiled": ([vp, vp, vp], st),
        "fv_euler_learned_step": ([vp, vp, i64], st),
        "fv_euler_learned_stats": ([vp, vp, vp, vp], st),
        "fv_euler_learned_destroy": ([vp], None),
        "fv_euler_train_workspace_bytes": ([ctypes.POINTER(fv_euler_train_config)], ctypes.c_size_t),
        "fv_euler_train_create": ([ctypes.POINTER(fv_euler_train_config), vp, vp, vp, vp, vp, ctypes.c_size_t,
                                   ctypes.POINTER(vp)], st),
        "fv_euler_train_step": ([vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(fv_learned_stats)], st),
        "fv_euler_train_input_grad": ([vp, vp], st),
        "fv_euler_adam_step": ([vp], st),
        "fv_euler_train_set_lr": ([vp, ctypes.c_float], st),
        "fv_euler_train_destroy": ([vp], None),
        "fv_model_param_count": ([], ctypes.c_size_t),
        "fv_model_workspace_bytes": ([ctypes.POINTER(fv_model_desc)], ctypes.c_size_t),
        "fv_model_create": ([ctypes.POINTER(fv_model_desc), vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)], st),
        "fv_model_update": ([vp], st),
        "fv_model_destroy": ([vp], None),
        "fv_model_forward_scratch_bytes": ([ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_size_t),
        "fv_model_forward": ([vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_size_t], st),
        "fv_model_forward_tiled": ([vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp], st),
        "fv_learned_step": ([vp, vp, i64, ctypes.POINTER(fv_learned_stats)], st),
        "fv_direct_step": ([vp, vp, i64, ctypes.POINTER(fv_learned_stats)], st),
        "fv_blend_step": ([vp, vp, i64, ctypes.POINTER(fv_learned_stats)], st),
        "fv_train_workspace_bytes": ([ctypes.POINTER(fv_train_config)], ctypes.c_size_t),
        "fv_train_create": ([ctypes.POINTER(fv_train_config), vp, vp, vp, vp, vp, ctypes.c_size_t,
                             ctypes.POINTER(vp)], st),
        "fv_train_step": ([vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(fv_learned_stats)], st),
        "fv_train_input_grad": ([vp, vp], st),
        "fv_train_state": ([vp, ctypes.c_int, vp], st),
        "fv_adam_step": ([vp], st),
        "fv_train_set_lr": ([vp, ctypes.c_float], st),
        "fv_train_destroy": ([vp], None),
        "fv_coarsen": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp], st),
        "fv_server_pool_overhead": ([ctypes.POINTER(fv_server_config)], ctypes.c_size_t),
        "fv_request_bytes": ([ctypes.POINTER(fv_request)], ctypes.c_size_t),
        "fv_server_create": ([ctypes.POINTER(fv_server_config), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)], st),
        "fv_server_submit": ([vp, ctypes.POINTER(fv_request), ctypes.POINTER(i64)], st),
        "fv_server_round": ([vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], st),
        "fv_server_info": ([vp, i64, ctypes.POINTER(fv_request_info)], st),
        "fv_server_get_stats": ([vp, ctypes.POINTER(fv_server_stats)], st),
        "fv_server_result": ([vp, i64, vp], st),
        "fv_server_release": ([vp, i64], st),
        "fv_server_destroy": ([vp], None),
        "fv_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def _check(rc: int):
    if rc != FV_OK:
        raise FvError(rc, lib.fv_last_error().decode())


# --------------------------------------------------------------- C-ABI names

def fv_nvar(cfg: fv_config) -> int:
    return lib.fv_nvar(ctypes.byref(cfg))


def fv_workspace_bytes(cfg: fv_config) -> int:
    n = lib.fv_workspace_bytes(ctypes.byref(cfg))
    if n == 0:
        raise FvError(FV_E_INVALID, lib.fv_last_error().decode())
    return n


def fv_init(cfg: fv_config, q_ptr: int, bathy_ptr: int | None, ws_ptr: int, ws_bytes: int, stream: int = 0):
    h = ctypes.c_void_p()
    _check(lib.fv_init(ctypes.byref(cfg), q_ptr, bathy_ptr, ws_ptr, ws_bytes, stream, ctypes.byref(h)))
    return h


def fv_step(h):
    _check(lib.fv_step(h))


def fv_run(h, nsteps: int):
    _check(lib.fv_run(h, int(nsteps)))


def fv_time(h):
    t, s = ctypes.c_double(), ctypes.c_int64()
    _check(lib.fv_time(h, ctypes.byref(t), ctypes.byref(s)))
    return t.value, s.value


def fv_totals(h, nvar: int) -> np.ndarray:
    out = np.zeros(nvar + 1)
    _check(lib.fv_totals(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def fv_get_state(h, dst_ptr: int, dst_is_host: int):
    _check(lib.fv_get_state(h, dst_ptr, dst_is_host))


def fv_set_state(h, src_ptr: int, src_is_host: int):
    _check(lib.fv_set_state(h, src_ptr, src_is_host))


def fv_state_ptr(h) -> int:
    return lib.fv_state_ptr(h)


def fv_reference_depth(h) -> float:
    return lib.fv_reference_depth(h)


def fv_set_stream(h, stream: int):
    _check(lib.fv_set_stream(h, stream))


def fv_face_fluxes(h, fx_ptr: int, fy_ptr: int):
    _check(lib.fv_face_fluxes(h, fx_ptr, fy_ptr))


def fv_destroy(h):
    lib.fv_destroy(h)


def fv_sphere_workspace_bytes(cfg: fv_sphere_config) -> int:
    n = lib.fv_sphere_workspace_bytes(ctypes.byref(cfg))
    if n == 0:
        raise FvError(FV_E_INVALID, lib.fv_last_error().decode())
    return n


def fv_sphere_init(cfg: fv_sphere_config, q_ptr: int, ws_ptr: int, ws_bytes: int, stream: int = 0):
    h = ctypes.c_void_p()
    _check(lib.fv_sphere_init(ctypes.byref(cfg), q_ptr, ws_ptr, ws_bytes, stream, ctypes.byref(h)))
    return h


def fv_sphere_run(h, nsteps: int):
    _check(lib.fv_sphere_run(h, int(nsteps)))


def fv_sphere_time(h):
    t, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib.fv_sphere_time(h, ctypes.byref(t), ctypes.byref(n)))
    return t.value, n.value


def fv_sphere_centres(h, dst_ptr: int):
    _check(lib.fv_sphere_centres(h, dst_ptr))


def fv_sphere_totals(h) -> np.ndarray:
    out = (ctypes.c_double * 2)()
    _check(lib.fv_sphere_totals(h, out))
    return np.array(out[:])


def fv_sphere_destroy(h):
    lib.fv_sphere_destroy(h)


def fv_noalloc_bytes(cfg: fv_config) -> int:
    return lib.fv_noalloc_bytes(ctypes.byref(cfg))


def fv_run_noalloc(cfg: fv_config, q_ptr: int, bathy_ptr: int | None, nsteps: int, stream: int = 0,
                   info_ptr: int | None = None):
    _check(lib.fv_run_noalloc(ctypes.byref(cfg), q_ptr, bathy_ptr, nsteps, stream, info_ptr))


FV_NOALLOC_SCRATCH_BYTES = 64 << 20


def fv_last_error() -> str:
    return lib.fv_last_error().decode()


def fv_model_param_count() -> int:
    return lib.fv_model_param_count()


def fv_model_workspace_bytes(desc: fv_model_desc) -> int:
    n = lib.fv_model_workspace_bytes(ctypes.byref(desc))
    if n == 0:
        raise FvError(FV_E_INVALID, "invalid model description")
    return n


def fv_model_create(desc: fv_model_desc, params_ptr: int, ws_ptr: int, ws_bytes: int, stream: int = 0):
    h = ctypes.c_void_p()
    _check(lib.fv_model_create(ctypes.byref(desc), params_ptr, ws_ptr, ws_bytes, stream, ctypes.byref(h)))
    return h


def fv_model_update(m):
    _check(lib.fv_model_update(m))


def fv_model_destroy(m):
    lib.fv_model_destroy(m)


def fv_model_forward_scratch_bytes(B: int, nx: int, ny: int) -> int:
    return lib.fv_model_forward_scratch_bytes(B, nx, ny)


def fv_model_forward(m, q_ptr: int, B: int, nx: int, ny: int, z_ptr: int, scratch_ptr: int, scratch_bytes: int):
    _check(lib.fv_model_forward(m, q_ptr, B, nx, ny, z_ptr, scratch_ptr, scratch_bytes))


def fv_model_forward_tiled(m, q_ptr: int, B: int, nx: int, ny: int, z_ptr: int):
    _check(lib.fv_model_forward_tiled(m, q_ptr, B, nx, ny, z_ptr))


def fv_learned_step(h, m, nsteps: int, want_stats: bool = True):
    st = fv_learned_stats()
    _check(lib.fv_learned_step(h, m, int(nsteps), ctypes.byref(st) if want_stats else None))
    return (st.fallback_faces, st.redone_steps) if want_stats else None


def fv_direct_step(h, m, nsteps: int, want_stats: bool = True):
    st = fv_learned_stats()
    _check(lib.fv_direct_step(h, m, int(nsteps), ctypes.byref(st) if want_stats else None))
    return (st.fallback_faces, st.redone_steps) if want_stats else None


def fv_blend_step(h, m, nsteps: int, want_stats: bool = True):
    st = fv_learned_stats()
    _check(lib.fv_blend_step(h, m, int(nsteps), ctypes.byref(st) if want_stats else None))
    return (st.fallback_faces, st.redone_steps) if want_stats else None


def fv_train_workspace_bytes(cfg: fv_train_config) -> int:
    n = lib.fv_train_workspace_bytes(ctypes.byref(cfg))
    if n == 0:
        raise FvError(FV_E_INVALID, lib.fv_last_error().decode())
    return n


def fv_train_create(cfg, model_h, grads_ptr, m_ptr, v_ptr, ws_ptr, ws_bytes):
    h = ctypes.c_void_p()
    _check(lib.fv_train_create(ctypes.byref(cfg), model_h, grads_ptr, m_ptr, v_ptr, ws_ptr, ws_bytes,
                               ctypes.byref(h)))
    return h


def fv_train_step(h, q0_ptr, tgt_ptr, T):
    loss = ctypes.c_double()
    st = fv_learned_stats()
    _check(lib.fv_train_step(h, q0_ptr, tgt_ptr, int(T), ctypes.byref(loss), ctypes.byref(st)))
    return loss.value, (st.fallback_faces, st.redone_steps)


def fv_train_input_grad(h, dst_ptr):
    _check(lib.fv_train_input_grad(h, dst_ptr))


def fv_train_state(h, t, dst_ptr):
    _check(lib.fv_train_state(h, int(t), dst_ptr))


def fv_adam_step(h):
    _check(lib.fv_adam_step(h))


def fv_train_set_lr(h, lr: float):
    _check(lib.fv_train_set_lr(h, float(lr)))


def fv_train_destroy(h):
    lib.fv_train_destroy(h)


def fv_coarsen(fine_ptr, nvar, nx, ny, factor, coarse_ptr, stream=0):
    _check(lib.fv_coarsen(fine_ptr, nvar, nx, ny, factor, coarse_ptr, stream))


def make_train_config(B, nx, ny, T, dt, lx=1.0, ly=1.0, g=9.81, h_ref=1.0, flux=FV_FLUX_HLLE,
                      scale=(0.05, 0.05, 0.05), lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                      direct=False, blend=False) -> fv_train_config:
    c = fv_train_config()
    c.struct_size = ctypes.sizeof(fv_train_config)
    c.B, c.nx, c.ny, c.T, c.flux = B, nx, ny, T, flux
    c.lx, c.ly, c.dt, c.g, c.h_ref = lx, ly, dt, g, h_ref
    for i in range(3):
        c.scale[i] = scale[i]
    c.lr, c.beta1, c.beta2, c.eps = lr, beta1, beta2, eps
    c.direct, c.blend = 1 if direct else 0, 1 if blend else 0
    return c


class Trainer:
    """Unrolled-loss training of a Model on batches of coarse windows."""

    def __init__(self, model: "Model", cfg: fv_train_config):
        import torch

        self.model = model
        self.cfg = cfg
        n = fv_model_param_count()
        dev = model.device
        self.grads = torch.zeros(n, dtype=torch.float32, device=dev)
        self.m = torch.zeros(n, dtype=torch.float32, device=dev)
        self.v = torch.zeros(n, dtype=torch.float32, device=dev)
        nb = fv_train_workspace_bytes(cfg)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        self.h = fv_train_create(cfg, model.h, self.grads.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                 self.ws.data_ptr(), nb)

    def step(self, q0, targets):
        """q0 [B,3,ny,nx], targets [T,B,3,ny,nx] (torch CUDA float32)."""
        q0 = q0.contiguous()
        targets = targets.contiguous()
        return fv_train_step(self.h, q0.data_ptr(), targets.data_ptr(), targets.shape[0])

    def input_grad(self):
        import torch

        c = self.cfg
        out = torch.empty((c.B, 3, c.ny, c.nx), dtype=torch.float32, device=self.model.device)
        fv_train_input_grad(self.h, out.data_ptr())
        return out

    def state(self, t):
        import torch

        c = self.cfg
        out = torch.empty((c.B, 3, c.ny, c.nx), dtype=torch.float32, device=self.model.device)
        fv_train_state(self.h, t, out.data_ptr())
        return out

    def adam(self):
        fv_adam_step(self.h)

    def set_lr(self, lr: float):
        fv_train_set_lr(self.h, lr)

    def close(self):
        if self.h is not None:
            fv_train_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def coarsen(fine, factor):
    """Block average of a torch CUDA float32 state [nvar, ny, nx] by factor."""
    import torch

    nvar, ny, nx = fine.shape
    out = torch.empty((nvar, ny // factor, nx // factor), dtype=torch.float32, device=fine.device)
    fv_coarsen(fine.contiguous().data_ptr(), nvar, nx, ny, factor, out.data_ptr(),
               torch.cuda.current_stream(fine.device).cuda_stream)
    return out


def make_request(q0, steps, bed=None, bc=FV_BC_WALL, cfl=0.4, g=9.81, gamma=1.4, h_ref=0.0, learned=False,
                 dt_fixed=0.0, lx=0.0):
    """Request over host arrays (kept referenced by the returned tuple until
    fv_server_submit copied them).  learned=True: a learned solve (periodic,
    no bed) of `steps` steps of dt_fixed with the server's model."""
    q0 = np.ascontiguousarray(q0, dtype=np.float32)
    nvar, n, n2 = q0.shape
    assert n == n2
    b = None if bed is None else np.ascontiguousarray(bed, dtype=np.float32)
    if learned:
        bc = FV_BC_PERIODIC
    r = fv_request(ctypes.sizeof(fv_request), FV_SWE if nvar == 3 else FV_EULER, n, bc, int(steps), cfl, g, gamma,
                   h_ref, q0.ctypes.data, None if b is None else b.ctypes.data, 1 if learned else 0, 0,
                   float(dt_fixed), float(lx))
    return r, (q0, b)


class Server:
    """Continuous-batching server over a torch-allocated device pool."""

    def __init__(self, pool_bytes: int, max_solves: int = 1024, steps_per_round: int = 24,
                 max_items: int = 1 << 18, device="cuda", stream=None, model=None, direct=False,
                 learned_split: int = 0, learned_layered: int = 0, act_pixels: int | None = None,
                 max_bypass: int = 0):
        """direct: launch every kernel of a round directly instead of replaying
        the round's captured graph (same results).  learned_split: network
        tiles in a round's first step from which the round runs the network
        pass and the learned stage as separate launches (0: the library's
        default).  learned_layered: 16 x 16 tiles from which such a round's
        network pass runs layer by layer (0: the library's default, -1:
        never); act_pixels: cells of its activation scratch, 128 bytes each
        out of the pool (None: with a model, an eighth of the pool up to 64 Mi
        cells; without, none).  max_bypass: rounds a queued request may go
        without fitting before nothing behind it is admitted (0: the
        library's default, -1: never)."""
        import torch

        self.model = model  # kept alive while the server runs
        if model is not None:
            torch.cuda.synchronize()  # the model's packed weights are ready
        if act_pixels is None:
            act_pixels = min(pool_bytes // 8 // 128, 1 << 26) if model is not None else 0
        self.cfg = fv_server_config(ctypes.sizeof(fv_server_config), max_solves, steps_per_round,
                                    1 if direct else 0, max_items, None if model is None else model.h,
                                    int(learned_split), int(learned_layered), int(act_pixels), int(max_bypass), 0)
        # zero-filled: the pool's pages are mapped here rather than by the
        # first rounds that reach them
        self.pool = torch.zeros(pool_bytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        h = ctypes.c_void_p()
        _check(lib.fv_server_create(ctypes.byref(self.cfg), self.pool.data_ptr(), pool_bytes,
                                    self.stream.cuda_stream, ctypes.byref(h)))
        self.h = h

    @staticmethod
    def request_bytes(req: fv_request) -> int:
        return lib.fv_request_bytes(ctypes.byref(req))

    def submit(self, q0, steps, bed=None, **kw) -> int:
        r, keep = make_request(q0, steps, bed, **kw)
        rid = ctypes.c_int64()
        _check(lib.fv_server_submit(self.h, ctypes.byref(r), ctypes.byref(rid)))
        del keep
        return rid.value

    def round(self):
        a, q = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.fv_server_round(self.h, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def info(self, rid: int) -> fv_request_info:
        inf = fv_request_info()
        _check(lib.fv_server_info(self.h, rid, ctypes.byref(inf)))
        return inf

    def stats(self) -> fv_server_stats:
        out = fv_server_stats()
        _check(lib.fv_server_get_stats(self.h, ctypes.byref(out)))
        return out

    def result(self, rid: int, shape):
        out = np.empty(shape, dtype=np.float32)
        _check(lib.fv_server_result(self.h, rid, out.ctypes.data))
        return out

    def release(self, rid: int):
        _check(lib.fv_server_release(self.h, rid))

    def close(self):
        if self.h is not None:
            lib.fv_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def params_to_vector(weights, biases) -> np.ndarray:
    """Master parameter vector from per-layer W (co, ci, 3, 3) and b (co)."""
    parts = []
    for w, b in zip(weights, biases):
        parts.append(np.asarray(w, dtype=np.float32).ravel())
        parts.append(np.asarray(b, dtype=np.float32).ravel())
    return np.concatenate(parts)


class Model:
    """Network parameters (torch FP32 master vector on the device) and the
    packed weights of libfv."""

    def __init__(self, params, desc: fv_model_desc | None = None, device="cuda", stream=None):
        import torch

        self.desc = desc if desc is not None else make_model_desc()
        self.device = torch.device(device)
        p = torch.as_tensor(np.asarray(params, dtype=np.float32), device=self.device).contiguous()
        if p.numel() != fv_model_param_count():
            raise ValueError(f"expected {fv_model_param_count()} parameters, got {p.numel()}")
        self.params = p
        n = fv_model_workspace_bytes(self.desc)
        self.ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = fv_model_create(self.desc, self.params.data_ptr(), self.ws.data_ptr(), n, self.stream.cuda_stream)

    def update(self):
        fv_model_update(self.h)

    def forward(self, q):
        """z [B, ny, nx, 72] for states q [B, 3, ny, nx] (torch CUDA float32)."""
        import torch

        B, _, ny, nx = q.shape
        z = torch.empty((B, ny, nx, 72), dtype=torch.float32, device=self.device)
        nb = fv_model_forward_scratch_bytes(B, nx, ny)
        sc = torch.empty(nb, dtype=torch.uint8, device=self.device)
        fv_model_forward(self.h, q.data_ptr(), B, nx, ny, z.data_ptr(), sc.data_ptr(), nb)
        return z

    def forward_tiled(self, q):
        """The same z from the one-launch tiled pass (nx, ny multiples of 8)."""
        import torch

        B, _, ny, nx = q.shape
        z = torch.empty((B, ny, nx, 72), dtype=torch.float32, device=self.device)
        fv_model_forward_tiled(self.h, q.data_ptr(), B, nx, ny, z.data_ptr())
        return z

    def close(self):
        if self.h is not None:
            fv_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------ torch-backed handle

class Solver:
    """A solve whose state, bed and workspace are torch CUDA tensors."""

    def __init__(self, q0, bathy=None, device="cuda", stream=None, **cfg_kw):
        import torch

        q0 = np.asarray(q0)
        nvar, ny, nx = q0.shape
        cfg_kw.setdefault("eqn", FV_SWE if nvar == 3 else FV_EULER)
        self.cfg = make_config(nx=nx, ny=ny, **cfg_kw)
        self.dtype = torch.float64 if self.cfg.prec == FV_F64 else torch.float32
        self.nvar = nvar
        self.device = torch.device(device)
        self.q = torch.tensor(q0, dtype=self.dtype, device=self.device).contiguous()
        self.bed = None if bathy is None else torch.tensor(np.asarray(bathy), dtype=self.dtype,
                                                           device=self.device).contiguous()
        nbytes = fv_workspace_bytes(self.cfg)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = fv_init(self.cfg, self.q.data_ptr(), None if self.bed is None else self.bed.data_ptr(),
                         self.ws.data_ptr(), nbytes, self.stream.cuda_stream)

    def step(self):
        fv_step(self.h)

    def run(self, nsteps: int):
        fv_run(self.h, nsteps)

    def time(self):
        return fv_time(self.h)

    def totals(self) -> np.ndarray:
        return fv_totals(self.h, self.nvar)

    def state(self) -> np.ndarray:
        out = np.empty((self.nvar, self.cfg.ny, self.cfg.nx),
                       dtype=np.float64 if self.cfg.prec == FV_F64 else np.float32)
        fv_get_state(self.h, out.ctypes.data, 1)
        return out.astype(np.float64)

    def set_state(self, q):
        src = np.ascontiguousarray(q, dtype=np.float64 if self.cfg.prec == FV_F64 else np.float32)
        fv_set_state(self.h, src.ctypes.data, 1)

    def reference_depth(self) -> float:
        return fv_reference_depth(self.h)

    def learned_step(self, model: "Model", nsteps: int, want_stats: bool = True):
        return fv_learned_step(self.h, model.h, nsteps, want_stats)

    def direct_step(self, model: "Model", nsteps: int, want_stats: bool = True):
        """Steps of the direct face-state scheme (the model's channels 0..11)."""
        return fv_direct_step(self.h, model.h, nsteps, want_stats)

    def blend_step(self, model: "Model", nsteps: int, want_stats: bool = True):
        """Learned steps with the flux-limiter blend of the face fluxes."""
        return fv_blend_step(self.h, model.h, nsteps, want_stats)

    def face_fluxes(self):
        import torch

        fx = torch.empty((self.nvar, self.cfg.ny, self.cfg.nx + 1), dtype=self.dtype, device=self.device)
        fy = torch.empty((self.nvar, self.cfg.ny + 1, self.cfg.nx), dtype=self.dtype, device=self.device)
        fv_face_fluxes(self.h, fx.data_ptr(), fy.data_ptr())
        return fx.double().cpu().numpy(), fy.double().cpu().numpy()

    def close(self):
        if self.h is not None:
            fv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EulerLearned:
    """Learned Euler step over B periodic solves; parameters, workspace and
    states are torch CUDA tensors (argument marshalling only)."""

    def __init__(self, params, B, nx, ny, dt, device="cuda", stream=None, **cfg_kw):
        import torch

        self.device = torch.device(device)
        self.cfg = make_euler_learned_config(B, nx, ny, dt, **cfg_kw)
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32), device=self.device).contiguous()
        assert self.params.numel() == lib.fv_euler_net_param_count()
        nb = lib.fv_euler_learned_workspace_bytes(ctypes.byref(self.cfg))
        if nb == 0:
            raise FvError(-1, lib.fv_last_error().decode())
        self.ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib.fv_euler_learned_create(ctypes.byref(self.cfg), self.params.data_ptr(), self.ws.data_ptr(), nb,
                                           self.stream.cuda_stream, ctypes.byref(h)))
        self.h = h

    def update(self):
        _check(lib.fv_euler_learned_update(self.h))

    def forward(self, q):
        """Raw coefficients [B, ny, nx, 96] of the states q [B, 4, ny, nx]."""
        import torch

        c = self.cfg
        q = q.contiguous()
        z = torch.empty((c.B, c.ny, c.nx, 96), dtype=torch.float32, device=self.device)
        _check(lib.fv_euler_learned_forward(self.h, q.data_ptr(), z.data_ptr()))
        return z

    def forward_tiled(self, q):
        """The same in one launch (nx, ny multiples of 8); bit-identical."""
        import torch

        c = self.cfg
        q = q.contiguous()
        z = torch.empty((c.B, c.ny, c.nx, 96), dtype=torch.float32, device=self.device)
        _check(lib.fv_euler_learned_forward_tiled(self.h, q.data_ptr(), z.data_ptr()))
        return z

    def step(self, q, nsteps: int):
        """nsteps learned Heun steps of q [B, 4, ny, nx] (float32, contiguous, in place)."""
        assert q.is_contiguous()
        _check(lib.fv_euler_learned_step(self.h, q.data_ptr(), int(nsteps)))

    def stats(self):
        """(fallback face sides, redone steps, frozen, rc) per solve, numpy arrays;
        rc is FV_E_INADMISSIBLE when a solve is frozen."""
        B = self.cfg.B
        fb, rd = np.zeros(B, dtype=np.int64), np.zeros(B, dtype=np.int64)
        fr = np.zeros(B, dtype=np.int32)
        rc = lib.fv_euler_learned_stats(self.h, fb.ctypes.data, rd.ctypes.data, fr.ctypes.data)
        return fb, rd, fr, rc

    def close(self):
        if self.h is not None:
            lib.fv_euler_learned_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EulerTrainer:
    """Unrolled-loss training of an EulerLearned network (its master
    parameters are updated in place by adam())."""

    def __init__(self, net: EulerLearned, cfg: fv_euler_train_config):
        import torch

        self.net = net
        self.cfg = cfg
        n = lib.fv_euler_net_param_count()
        self.grads = torch.zeros(n, dtype=torch.float32, device=net.device)
        self.m = torch.zeros(n, dtype=torch.float32, device=net.device)
        self.v = torch.zeros(n, dtype=torch.float32, device=net.device)
        nb = lib.fv_euler_train_workspace_bytes(ctypes.byref(cfg))
        if nb == 0:
            raise FvError(-1, lib.fv_last_error().decode())
        self.ws = torch.empty(nb, dtype=torch.uint8, device=net.device)
        h = ctypes.c_void_p()
        _check(lib.fv_euler_train_create(ctypes.byref(cfg), net.h, self.grads.data_ptr(), self.m.data_ptr(),
                                         self.v.data_ptr(), self.ws.data_ptr(), nb, ctypes.byref(h)))
        self.h = h

    def step(self, q0, targets):
        """q0 [B,4,ny,nx], targets [T,B,4,ny,nx] (torch CUDA float32) -> (loss, (fallbacks, redone))."""
        q0 = q0.contiguous()
        targets = targets.contiguous()
        loss = ctypes.c_double()
        stats = fv_learned_stats()
        _check(lib.fv_euler_train_step(self.h, q0.data_ptr(), targets.data_ptr(), targets.shape[0],
                                       ctypes.byref(loss), ctypes.byref(stats)))
        return loss.value, (stats.fallback_faces, stats.redone_steps)

    def input_grad(self):
        import torch

        c = self.cfg
        out = torch.empty((c.B, 4, c.ny, c.nx), dtype=torch.float32, device=self.net.device)
        _check(lib.fv_euler_train_input_grad(self.h, out.data_ptr()))
        return out

    def adam(self):
        _check(lib.fv_euler_adam_step(self.h))

    def set_lr(self, lr: float):
        _check(lib.fv_euler_train_set_lr(self.h, lr))

    def close(self):
        if self.h is not None:
            lib.fv_euler_train_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SphereSolver:
    """Shallow water on the sphere: state and workspace are torch CUDA tensors."""

    def __init__(self, q0, device="cuda", stream=None, **cfg_kw):
        import torch

        q0 = np.asarray(q0)
        assert q0.ndim == 3 and q0.shape[0] == 4 and q0.shape[2] == 2 * q0.shape[1], q0.shape
        self.cfg = make_sphere_config(q0.shape[1], **cfg_kw)
        self.dtype = torch.float64 if self.cfg.prec == FV_F64 else torch.float32
        self.device = torch.device(device)
        self.q = torch.tensor(q0, dtype=self.dtype, device=self.device).contiguous()
        nbytes = fv_sphere_workspace_bytes(self.cfg)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = fv_sphere_init(self.cfg, self.q.data_ptr(), self.ws.data_ptr(), nbytes, self.stream.cuda_stream)

    def run(self, nsteps: int):
        fv_sphere_run(self.h, nsteps)

    def time(self):
        return fv_sphere_time(self.h)

    def totals(self) -> np.ndarray:
        return fv_sphere_totals(self.h)

    def centres(self) -> np.ndarray:
        import torch

        n = self.cfg.n
        out = torch.empty((3, n, 2 * n), dtype=self.dtype, device=self.device)
        fv_sphere_centres(self.h, out.data_ptr())
        return out.double().cpu().numpy()

    def state(self) -> np.ndarray:
        import torch

        torch.cuda.synchronize(self.device)
        return self.q.double().cpu().numpy()

    def close(self):
        if self.h is not None:
            fv_sphere_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
