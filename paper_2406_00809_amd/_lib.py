"""ctypes binding of libgnp.so (include/gnp.h).  Argument marshalling only:
every step of the computation runs in the HIP library.

torch is imported first so that libgnp binds to the same HIP runtime as
PyTorch (both need the soname libamdhip64.so.7); PyTorch supplies device
memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (must precede loading libgnp)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgnp.so")

GNP_OK, GNP_EINVAL, GNP_ENOMEM, GNP_EDEVICE, GNP_ENUMERIC, GNP_EBUSY = range(6)
STATUS_NAMES = {0: "GNP_OK", 1: "GNP_EINVAL", 2: "GNP_ENOMEM", 3: "GNP_EDEVICE",
                4: "GNP_ENUMERIC", 5: "GNP_EBUSY"}
GNP_F64, GNP_F32, GNP_BF16 = 0, 1, 2

# every exported entry point: name -> (restype, argtypes)
VP, I32P, F64P = C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)


class TrainOpts(C.Structure):
    _fields_ = [("steps", C.c_int), ("batch", C.c_int), ("lr", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("seed", C.c_uint64), ("prec", C.c_int), ("sampler_m", C.c_int),
                ("sampler_count", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("mismatch", C.c_int), ("breakdowns", C.c_int),
                ("rel_res_true", C.c_double), ("rel_res_est", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("rejected", C.c_int64), ("queued", C.c_int64), ("active", C.c_int64),
                ("max_active", C.c_int64), ("latency_p50_s", C.c_double),
                ("latency_p99_s", C.c_double), ("latency_mean_s", C.c_double),
                ("solves_per_s", C.c_double), ("hbm_budget", C.c_size_t),
                ("hbm_used", C.c_size_t), ("hbm_peak", C.c_size_t),
                ("workspaces_allocated", C.c_int64), ("workspaces_reused", C.c_int64),
                ("workspaces_evicted", C.c_int64), ("converged", C.c_int64),
                ("converged_per_s", C.c_double), ("conv_latency_p50_s", C.c_double),
                ("conv_latency_p99_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SIGNATURES = {
    "gnp_last_error": (C.c_char_p, []),
    "gnp_version": (C.c_char_p, []),
    "gnp_system_create": (C.c_int, [C.c_int64, C.c_int64, VP, VP, VP, C.c_int, VP,
                                    C.POINTER(VP)]),
    "gnp_system_destroy": (None, [VP]),
    "gnp_system_gamma": (C.c_int, [VP, F64P, F64P]),
    "gnp_system_export": (C.c_int, [VP, VP, VP, VP, VP, VP]),
    "gnp_system_n": (C.c_int64, [VP]),
    "gnp_system_nnz": (C.c_int64, [VP]),
    "gnp_spmv": (C.c_int, [VP, VP, VP, C.c_int, VP]),
    "gnp_model_create": (C.c_int, [VP, C.c_int, C.c_int, C.c_int, VP, C.c_uint64,
                                   C.POINTER(VP)]),
    "gnp_model_destroy": (None, [VP]),
    "gnp_system_set_values": (C.c_int, [VP, VP, VP]),
    "gnp_model_nparams": (C.c_size_t, [VP]),
    "gnp_model_set_scaling": (C.c_int, [VP, C.c_int]),
    "gnp_params_get": (C.c_int, [VP, VP, C.c_size_t]),
    "gnp_params_set": (C.c_int, [VP, VP, C.c_size_t]),
    "gnp_params_set_device": (C.c_int, [VP, VP, C.c_size_t, VP]),
    "gnp_apply": (C.c_int, [VP, VP, VP, C.c_int, C.c_int, VP]),
    "gnp_apply_noalloc": (C.c_int, [VP, VP, VP, C.c_int, C.c_int, VP]),
    "gnp_apply_layers": (C.c_int, [VP, VP, VP, VP, C.c_int, C.c_int, VP]),
    "fgmres_solve": (C.c_int, [VP, VP, VP, VP, C.c_int, C.c_double, C.c_int, C.c_int, VP,
                               C.POINTER(SolveInfo), VP]),
    "fgmres_solve_batch": (C.c_int, [VP, VP, VP, VP, C.c_int, C.c_int, C.c_double, C.c_int,
                                     C.c_int, VP, VP]),
    "fgmres_solve_jacobi": (C.c_int, [VP, VP, VP, C.c_int, C.c_double, C.c_int, C.c_int, VP,
                                      C.POINTER(SolveInfo), VP]),
    "fgmres_solve_gmres": (C.c_int, [VP, VP, VP, C.c_int, C.c_double, C.c_int, C.c_int,
                                     C.c_double, C.c_int, VP, C.POINTER(SolveInfo), VP]),
    "fgmres_step_times": (C.c_int, [VP, VP, C.c_int]),
    "gnp_system_set_timeout": (C.c_int, [VP, C.c_double]),
    "gnp_auc": (C.c_int, [VP, VP, C.c_int, C.c_double, VP, VP]),
    "gnp_train": (C.c_int, [VP, C.POINTER(TrainOpts), VP, VP, C.POINTER(C.c_int), VP]),
    "gnp_loss_grad": (C.c_int, [VP, VP, C.c_int, C.c_int, F64P, VP, VP]),
    "gnp_forward_save": (C.c_int, [VP, VP, VP, C.c_int, C.c_int, VP]),
    "gnp_backward": (C.c_int, [VP, VP, VP, VP]),
    "gnp_time_layer": (C.c_int, [VP, C.c_int, C.c_int, C.c_int, F64P, VP]),
    "gnp_time_layer_cold": (C.c_int, [VP, C.c_int, C.c_int, C.c_int, VP, C.c_size_t, F64P,
                                      F64P, VP]),
    "gnp_time_spmv": (C.c_int, [VP, VP, VP, C.c_int, C.c_int, F64P, VP]),
    "gnp_server_create": (C.c_int, [C.c_size_t, C.c_int, C.c_int, C.c_int, C.c_int,
                                    C.POINTER(VP)]),
    "gnp_server_register": (C.c_int, [VP, VP, VP, C.POINTER(C.c_int)]),
    "gnp_server_workspace_bytes": (C.c_int, [VP, C.c_int, C.POINTER(C.c_size_t)]),
    "gnp_server_submit": (C.c_int, [VP, C.c_int, VP, C.c_double, C.c_int,
                                    C.POINTER(C.c_uint64)]),
    "gnp_server_poll": (C.c_int, [VP, C.c_uint64, VP, C.POINTER(SolveInfo), F64P]),
    "gnp_server_drain": (C.c_int, [VP, C.c_double]),
    "gnp_server_update_system": (C.c_int, [VP, C.c_int, VP, VP, VP, C.POINTER(C.c_int)]),
    "gnp_server_get_stats": (C.c_int, [VP, C.POINTER(ServerStats)]),
    "gnp_server_destroy": (None, [VP]),
    "gnp_sampler_create": (C.c_int, [VP, C.c_int, C.c_uint64, C.c_int, VP, C.POINTER(VP)]),
    "gnp_sampler_info": (C.c_int, [VP, C.POINTER(C.c_int), VP, VP, VP]),
    "gnp_sampler_draw": (C.c_int, [VP, C.c_uint32, C.c_int, VP, VP]),
    "gnp_sampler_destroy": (None, [VP]),
}

_lib = None


class GNPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libgnp.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2406_00809_amd.build`")
    L = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status: int):
    if status != GNP_OK:
        msg = load().gnp_last_error()
        raise GNPError(status, msg.decode() if msg else "")
