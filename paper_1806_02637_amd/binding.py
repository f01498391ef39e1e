"""ctypes binding of libecc.so: one Python function per C entry point of
include/ecc.h, with the same name and argument order.  Argument marshalling
only -- every step of the path runs in the HIP kernels behind the library.

Pointers are passed as Python ints (``tensor.data_ptr()``, ``ctypes`` buffers
or 0 for NULL); streams as the integer handle of a hipStream_t.  A non-zero
status raises ``EccError`` with the library's message.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libecc.so")

ECC_OK, ECC_E_ARG, ECC_E_BUDGET, ECC_E_HIP, ECC_E_STATE, ECC_E_NOSCAN = 0, -1, -2, -3, -4, -5
ECC_F32, ECC_BF16, ECC_F16 = 0, 1, 2
ECC_GEOM_F32, ECC_GEOM_F64 = 0, 1
ECC_KAPPA_OBJECT, ECC_KAPPA_DETECTOR = 0, 1
ECC_NOALLOC_SCRATCH_BYTES = 64 << 20
DTYPES = {"f32": ECC_F32, "bf16": ECC_BF16, "f16": ECC_F16}

# every symbol include/ecc.h declares
SYMBOLS = (
    "ecc_last_error", "ecc_create", "ecc_destroy", "ecc_scan_load", "ecc_scan_build_sinograms",
    "ecc_scan_set_sinograms", "ecc_scan_read_sinogram", "ecc_scan_free", "ecc_scan_bytes", "ecc_workspace_bytes",
    "ecc_cost", "ecc_cost_counts", "ecc_cost_noalloc", "ecc_cost_grad", "ecc_cost_pinv", "ecc_scan_info",
    "ecc_spline_motion", "ecc_spline_motion_grad",
    "ecc_fdk_workspace_bytes", "ecc_fdk",
    "ecc_server_create", "ecc_server_submit", "ecc_server_poll", "ecc_server_wait", "ecc_server_request_bytes",
    "ecc_server_set_work_cap", "ecc_server_destroy",
)
# the measurement probe of include/ecc_probe.h
PROBE_SYMBOLS = ("ecc_probe_gather",)


class EccError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func} -> {status}: {msg}")
        self.status = status


class EvalParams(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("geom", ctypes.c_int32), ("R_mm", ctypes.c_double), ("c", ctypes.c_double),
                ("kappa_range", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class EccVolume(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("voxel_mm", ctypes.c_double)]


class RequestStats(ctypes.Structure):
    _fields_ = [("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("slot", ctypes.c_int32), ("status", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_U64 = ctypes.c_uint64

_SIGNATURES = {
    "ecc_last_error": ([], ctypes.c_char_p),
    "ecc_create": ([ctypes.POINTER(_P), ctypes.c_int, _U64], _I32),
    "ecc_destroy": ([_P], _I32),
    "ecc_scan_load": ([_P, ctypes.POINTER(_I32), _I32, _I32, _I32, _P, _P, _P, _I32], _I32),
    "ecc_scan_build_sinograms": ([_P, _I32, _I32, _I32, ctypes.c_double, _I32, _P], _I32),
    "ecc_scan_set_sinograms": ([_P, _I32, _I32, _I32, _P, _I32, _I32], _I32),
    "ecc_scan_read_sinogram": ([_P, _I32, _I32, _P], _I32),
    "ecc_scan_free": ([_P, _I32], _I32),
    "ecc_scan_bytes": ([_P, _I32, ctypes.POINTER(_U64)], _I32),
    "ecc_workspace_bytes": ([_P, _I32, _I32, _I32, ctypes.POINTER(_U64)], _I32),
    "ecc_cost": ([_P, _I32, _I32, _P, ctypes.POINTER(EvalParams), _P, _P, _P, _U64, _P], _I32),
    "ecc_cost_counts": ([_P, _I32, _I32, _P, ctypes.POINTER(EvalParams), _P, _P, _P, _P, _U64, _P], _I32),
    "ecc_cost_noalloc": ([_P, _I32, _I32, _P, ctypes.POINTER(EvalParams), _P, _P, _P], _I32),
    "ecc_cost_grad": ([_P, _I32, _I32, _P, ctypes.POINTER(EvalParams), _P, _P, _P, _P, _U64, _P], _I32),
    "ecc_cost_pinv": ([_P, _I32, _I32, _P, _P, ctypes.POINTER(EvalParams), _P, _P, _P, _U64, _P], _I32),
    "ecc_scan_info": ([_P, _I32] + [ctypes.POINTER(_I32)] * 5, _I32),
    "ecc_spline_motion": ([_P, _I32, _I32, _I32, _P, _P, _P, _P], _I32),
    "ecc_spline_motion_grad": ([_P, _I32, _I32, _I32, _P, _P, _P, _P, _P], _I32),
    "ecc_fdk_workspace_bytes": ([_P, _I32, ctypes.POINTER(_U64)], _I32),
    "ecc_fdk": ([_P, _I32, _P, _P, ctypes.POINTER(EccVolume), _P, _P, _U64, _P], _I32),
    "ecc_server_create": ([_P, ctypes.POINTER(_P), _I32, _U64], _I32),
    "ecc_server_submit": ([_P, _I32, _I32, _P, ctypes.POINTER(EvalParams), _I32, ctypes.POINTER(ctypes.c_int64)],
                          _I32),
    "ecc_server_poll": ([_P, ctypes.c_int64, ctypes.POINTER(_I32)], _I32),
    "ecc_server_wait": ([_P, ctypes.c_int64, _P, _P, ctypes.POINTER(RequestStats)], _I32),
    "ecc_server_request_bytes": ([_P, _I32, _I32, _I32, ctypes.POINTER(_U64)], _I32),
    "ecc_server_set_work_cap": ([_P, ctypes.c_double], _I32),
    "ecc_server_destroy": ([_P], _I32),
    "ecc_probe_gather": ([_P, _U64, _I32, _I32, _I32, _P, _P], _I32),
}


def load_library(path: str = LIB_PATH):
    """Opens libecc.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with paper_1806_02637_amd.build.build() "
                               "(the engine has no CPU fallback)")
        lib = ctypes.CDLL(path)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _check(status: int, func: str):
    if status != ECC_OK:
        raise EccError(status, func, ecc_last_error())


def ecc_last_error() -> str:
    return load_library().ecc_last_error().decode()


def ecc_create(hip_device: int = 0, hbm_budget_bytes: int = 0) -> int:
    out = _P()
    _check(load_library().ecc_create(ctypes.byref(out), hip_device, hbm_budget_bytes), "ecc_create")
    return out.value


def ecc_destroy(ctx: int):
    _check(load_library().ecc_destroy(ctx), "ecc_destroy")


def ecc_scan_load(ctx: int, n_views: int, W: int, H: int, P_ptr: int, intr_ptr: int, images_ptr: int,
                  images_on_device: int) -> int:
    sid = _I32()
    _check(load_library().ecc_scan_load(ctx, ctypes.byref(sid), n_views, W, H, P_ptr, intr_ptr, images_ptr,
                                        images_on_device), "ecc_scan_load")
    return sid.value


def ecc_scan_build_sinograms(ctx: int, scan_id: int, n_alpha: int, n_t: int, ds_px: float, dtype: int,
                             stream: int = 0):
    _check(load_library().ecc_scan_build_sinograms(ctx, scan_id, n_alpha, n_t, ds_px, dtype, stream),
           "ecc_scan_build_sinograms")


def ecc_scan_set_sinograms(ctx: int, scan_id: int, n_alpha: int, n_t: int, sino_ptr: int, sino_on_device: int,
                           dtype: int):
    _check(load_library().ecc_scan_set_sinograms(ctx, scan_id, n_alpha, n_t, sino_ptr, sino_on_device, dtype),
           "ecc_scan_set_sinograms")


def ecc_scan_read_sinogram(ctx: int, scan_id: int, view: int, out_ptr: int):
    _check(load_library().ecc_scan_read_sinogram(ctx, scan_id, view, out_ptr), "ecc_scan_read_sinogram")


def ecc_scan_free(ctx: int, scan_id: int):
    _check(load_library().ecc_scan_free(ctx, scan_id), "ecc_scan_free")


def ecc_scan_bytes(ctx: int, scan_id: int) -> int:
    out = _U64()
    _check(load_library().ecc_scan_bytes(ctx, scan_id, ctypes.byref(out)), "ecc_scan_bytes")
    return out.value


def ecc_workspace_bytes(ctx: int, scan_id: int, B: int, with_grad: int) -> int:
    out = _U64()
    _check(load_library().ecc_workspace_bytes(ctx, scan_id, B, with_grad, ctypes.byref(out)), "ecc_workspace_bytes")
    return out.value


def ecc_cost(ctx: int, scan_id: int, B: int, theta_ptr: int, params: EvalParams, out_cost_ptr: int,
             out_pair_ptr: int, workspace_ptr: int, workspace_bytes: int, stream: int = 0):
    _check(load_library().ecc_cost(ctx, scan_id, B, theta_ptr, ctypes.byref(params), out_cost_ptr, out_pair_ptr,
                                   workspace_ptr, workspace_bytes, stream), "ecc_cost")


def ecc_cost_counts(ctx: int, scan_id: int, B: int, theta_ptr: int, params: EvalParams, out_cost_ptr: int,
                    out_pair_ptr: int, out_count_ptr: int, workspace_ptr: int, workspace_bytes: int, stream: int = 0):
    _check(load_library().ecc_cost_counts(ctx, scan_id, B, theta_ptr, ctypes.byref(params), out_cost_ptr,
                                          out_pair_ptr, out_count_ptr, workspace_ptr, workspace_bytes, stream),
           "ecc_cost_counts")


def ecc_cost_noalloc(ctx: int, scan_id: int, B: int, theta_ptr: int, params: EvalParams, out_cost_ptr: int,
                     out_pair_ptr: int, stream: int = 0):
    _check(load_library().ecc_cost_noalloc(ctx, scan_id, B, theta_ptr, ctypes.byref(params), out_cost_ptr,
                                           out_pair_ptr, stream), "ecc_cost_noalloc")


def ecc_cost_grad(ctx: int, scan_id: int, B: int, theta_ptr: int, params: EvalParams, out_cost_ptr: int,
                  grad_ptr: int, out_pair_grad_ptr: int, workspace_ptr: int, workspace_bytes: int, stream: int = 0):
    _check(load_library().ecc_cost_grad(ctx, scan_id, B, theta_ptr, ctypes.byref(params), out_cost_ptr, grad_ptr,
                                        out_pair_grad_ptr, workspace_ptr, workspace_bytes, stream), "ecc_cost_grad")


def ecc_cost_pinv(ctx: int, scan_id: int, B: int, theta_ptr: int, pinv_ptr: int, params: EvalParams,
                  out_cost_ptr: int, out_pair_ptr: int, workspace_ptr: int, workspace_bytes: int, stream: int = 0):
    _check(load_library().ecc_cost_pinv(ctx, scan_id, B, theta_ptr, pinv_ptr, ctypes.byref(params), out_cost_ptr,
                                        out_pair_ptr, workspace_ptr, workspace_bytes, stream), "ecc_cost_pinv")


def ecc_scan_info(ctx: int, scan_id: int):
    vals = [_I32() for _ in range(5)]
    _check(load_library().ecc_scan_info(ctx, scan_id, *[ctypes.byref(v) for v in vals]), "ecc_scan_info")
    return tuple(v.value for v in vals)


def ecc_fdk_workspace_bytes(ctx: int, scan_id: int) -> int:
    out = _U64()
    _check(load_library().ecc_fdk_workspace_bytes(ctx, scan_id, ctypes.byref(out)), "ecc_fdk_workspace_bytes")
    return int(out.value)


def ecc_fdk(ctx: int, scan_id: int, theta_ptr: int, images_ptr: int, vol: EccVolume, out_ptr: int,
            workspace_ptr: int, workspace_bytes: int, stream: int = 0):
    _check(load_library().ecc_fdk(ctx, scan_id, theta_ptr, images_ptr, ctypes.byref(vol), out_ptr, workspace_ptr,
                                  workspace_bytes, stream), "ecc_fdk")


def ecc_spline_motion(ctx: int, B: int, n_views: int, n_nodes: int, node_x_ptr: int, nodes_ptr: int,
                      theta_ptr: int, stream: int = 0):
    _check(load_library().ecc_spline_motion(ctx, B, n_views, n_nodes, node_x_ptr, nodes_ptr, theta_ptr, stream),
           "ecc_spline_motion")


def ecc_spline_motion_grad(ctx: int, B: int, n_views: int, n_nodes: int, node_x_ptr: int, nodes_ptr: int,
                           grad_theta_ptr: int, grad_nodes_ptr: int, stream: int = 0):
    _check(load_library().ecc_spline_motion_grad(ctx, B, n_views, n_nodes, node_x_ptr, nodes_ptr, grad_theta_ptr,
                                                 grad_nodes_ptr, stream), "ecc_spline_motion_grad")


def ecc_server_create(ctx: int, n_slots: int, arena_bytes: int) -> int:
    out = _P()
    _check(load_library().ecc_server_create(ctx, ctypes.byref(out), n_slots, arena_bytes), "ecc_server_create")
    return out.value


def ecc_server_submit(srv: int, scan_id: int, B: int, theta_host_ptr: int, params: EvalParams,
                      with_grad: int) -> int:
    rid = ctypes.c_int64()
    _check(load_library().ecc_server_submit(srv, scan_id, B, theta_host_ptr, ctypes.byref(params), with_grad,
                                            ctypes.byref(rid)), "ecc_server_submit")
    return rid.value


def ecc_server_poll(srv: int, request_id: int) -> bool:
    done = _I32()
    _check(load_library().ecc_server_poll(srv, request_id, ctypes.byref(done)), "ecc_server_poll")
    return bool(done.value)


def ecc_server_wait(srv: int, request_id: int, cost_host_ptr: int, grad_host_ptr: int) -> RequestStats:
    st = RequestStats()
    _check(load_library().ecc_server_wait(srv, request_id, cost_host_ptr, grad_host_ptr, ctypes.byref(st)),
           "ecc_server_wait")
    return st


def ecc_server_set_work_cap(srv: int, work_cap: float):
    _check(load_library().ecc_server_set_work_cap(srv, float(work_cap)), "ecc_server_set_work_cap")


def ecc_server_request_bytes(srv: int, scan_id: int, B: int, with_grad: int) -> int:
    out = _U64()
    _check(load_library().ecc_server_request_bytes(srv, scan_id, B, with_grad, ctypes.byref(out)),
           "ecc_server_request_bytes")
    return out.value


def ecc_server_destroy(srv: int):
    _check(load_library().ecc_server_destroy(srv), "ecc_server_destroy")


def ecc_probe_gather(buf_ptr: int, nbytes: int, pattern: int, iters: int, n_blocks: int, out_ptr: int,
                     stream: int = 0):
    _check(load_library().ecc_probe_gather(buf_ptr, nbytes, pattern, iters, n_blocks, out_ptr, stream),
           "ecc_probe_gather")
