"""ctypes binding of libhprqp.so (the C ABI in include/hprqp.h).

Argument marshalling only: PyTorch supplies device memory and the stream;
every step of the solver runs in the library's HIP kernels.  There is no
fallback: if the library is missing or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhprqp.so")

_vp = C.c_void_p


class hprqp_problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("qkind", C.c_int32),
                ("q_rowptr", _vp), ("q_col", _vp), ("q_val", _vp), ("q_nnz", C.c_int64),
                ("kron_p", C.c_int32), ("kron_s", C.c_int32), ("kron_B", _vp), ("kron_C", _vp),
                ("lr_rank", C.c_int32), ("lr_d", _vp), ("lr_F", _vp),
                ("c", _vp), ("L", _vp), ("U", _vp),
                ("a_rowptr", _vp), ("a_col", _vp), ("a_val", _vp), ("a_nnz", C.c_int64),
                ("l", _vp), ("u", _vp),
                ("l1_weight", C.c_double),
                ("gram_p", C.c_int32), ("gram_rowptr", _vp), ("gram_col", _vp), ("gram_val", _vp),
                ("gram_nnz", C.c_int64), ("kron_S", _vp), ("kron_T", _vp)]


class hprqp_options(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int64), ("time_limit_s", C.c_double),
                ("check_every", C.c_int32), ("sigma0", C.c_double),
                ("lambda_A", C.c_double), ("lambda_Q", C.c_double),
                ("power_start_A", _vp), ("power_start_Q", _vp),
                ("alpha1", C.c_double), ("alpha2", C.c_double), ("alpha3", C.c_double),
                ("enable_restart", C.c_int32), ("enable_sigma_update", C.c_int32),
                ("use_graph", C.c_int32), ("spmv_autotune", C.c_int32),
                ("trace_iters", C.c_int32), ("trace_host", C.POINTER(C.c_double)),
                ("log_cap", C.c_int32), ("check_log_host", C.POINTER(C.c_double)),
                ("profile_kernels", C.c_int32), ("precondition", C.c_int32), ("ruiz_iters", C.c_int32),
                ("spmv_lanes", C.c_int32), ("method", C.c_int32), ("kron_kernel", C.c_int32),
                ("small_path", C.c_int32), ("batch_threads", C.c_int32)]


class hprqp_info(C.Structure):
    _fields_ = [("term", C.c_int32), ("iters", C.c_int64), ("restarts", C.c_int32), ("n_log", C.c_int32),
                ("sigma", C.c_double), ("sigma0", C.c_double), ("lambda_A", C.c_double),
                ("lambda_Q", C.c_double), ("eta_p", C.c_double), ("eta_d", C.c_double),
                ("eta_gap", C.c_double), ("pobj", C.c_double), ("dobj", C.c_double),
                ("R_last", C.c_double), ("t_setup_s", C.c_double), ("t_solve_s", C.c_double),
                ("t_precond_s", C.c_double), ("qwx_gap", C.c_double)]


class hprqp_state(C.Structure):
    _fields_ = [("k", C.c_int64), ("restarts", C.c_int32), ("reserved", C.c_int32), ("sigma", C.c_double),
                ("R0ref", C.c_double), ("alpha3", C.c_double), ("y", C.c_void_p), ("w", C.c_void_p),
                ("x", C.c_void_p)]


EXPORTS = ("hprqp_default_options", "hprqp_create", "hprqp_solve", "hprqp_solve_resume", "hprqp_residuals", "hprqp_residuals_noalloc",
           "hprqp_apply",
           "hprqp_power_info", "hprqp_scaling", "hprqp_kernel_stats", "hprqp_set_options", "hprqp_destroy", "hprqp_batch_create", "hprqp_solve_batch",
           "hprqp_batch_last_kernel_s", "hprqp_batch_shapes", "hprqp_batch_set_priority", "hprqp_stream_copy", "hprqp_batch_destroy", "hprqp_last_error")

_lib = None


def load():
    """Load libhprqp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with `python -m paper_2507_02470_amd.build`")
    lib = C.CDLL(LIB_PATH)
    lib.hprqp_default_options.argtypes = [C.POINTER(hprqp_options)]
    lib.hprqp_default_options.restype = None
    lib.hprqp_create.argtypes = [C.POINTER(hprqp_problem), C.POINTER(hprqp_options), _vp, C.POINTER(_vp)]
    lib.hprqp_solve.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(hprqp_info)]
    lib.hprqp_solve_resume.argtypes = [_vp, C.POINTER(hprqp_state), C.POINTER(hprqp_state), _vp, _vp, _vp, _vp,
                                       C.POINTER(hprqp_info)]
    lib.hprqp_solve_resume.restype = C.c_int
    lib.hprqp_residuals.argtypes = [_vp, _vp, _vp, _vp, _vp, C.POINTER(hprqp_info)]
    lib.hprqp_residuals_noalloc.argtypes = [C.POINTER(hprqp_problem), _vp, _vp, _vp, _vp, C.POINTER(hprqp_info), _vp]
    lib.hprqp_apply.argtypes = [_vp, C.c_int32, _vp, _vp]
    lib.hprqp_power_info.argtypes = [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    lib.hprqp_scaling.argtypes = [_vp, _vp, _vp]
    lib.hprqp_scaling.restype = C.c_int
    lib.hprqp_kernel_stats.argtypes = [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    lib.hprqp_kernel_stats.restype = C.c_int
    lib.hprqp_set_options.argtypes = [_vp, C.POINTER(hprqp_options)]
    lib.hprqp_set_options.restype = C.c_int
    lib.hprqp_destroy.argtypes = [_vp]
    lib.hprqp_destroy.restype = None
    lib.hprqp_last_error.restype = C.c_char_p
    lib.hprqp_stream_copy.argtypes = [_vp, _vp, C.c_int64, _vp, C.POINTER(C.c_double)]
    lib.hprqp_stream_copy.restype = C.c_int
    if hasattr(lib, "hprqp_batch_create"):
        lib.hprqp_batch_create.argtypes = [C.c_int32, C.POINTER(hprqp_problem), C.POINTER(hprqp_options), _vp,
                                           C.POINTER(_vp)]
        lib.hprqp_solve_batch.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(hprqp_info)]
        lib.hprqp_batch_last_kernel_s.argtypes = [_vp]
        lib.hprqp_batch_last_kernel_s.restype = C.c_double
        lib.hprqp_batch_shapes.argtypes = [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        lib.hprqp_batch_shapes.restype = C.c_int
        lib.hprqp_batch_set_priority.argtypes = [_vp, _vp]
        lib.hprqp_batch_set_priority.restype = C.c_int
        lib.hprqp_batch_destroy.argtypes = [_vp]
        lib.hprqp_batch_destroy.restype = None
    for name in ("hprqp_create", "hprqp_solve", "hprqp_residuals", "hprqp_residuals_noalloc", "hprqp_apply",
                 "hprqp_power_info",
                 "hprqp_kernel_stats",
                 "hprqp_batch_create", "hprqp_solve_batch"):
        if hasattr(lib, name):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_SHAPE", 3: "ERR_BOUNDS", 4: "ERR_HIP", 5: "ERR_OOM", 6: "ERR_UNSUPPORTED"}
TERM = {0: "solved", 1: "max_iter", 2: "time_limit", 3: "numerical"}


class HPRQPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def check(status: int):
    if status != 0:
        raise HPRQPError(status, load().hprqp_last_error().decode())
