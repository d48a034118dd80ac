"""ctypes declarations of the C ABI in include/saamg.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_NAME = "libsaamg.so"

AMG_OK = 0
AMG_NOT_CONVERGED = 1
AMG_ERR_ARG = -1
AMG_ERR_SINGULAR_BLOCK = -2
AMG_ERR_NOT_SPD = -3
AMG_ERR_OOM = -4
AMG_ERR_HIP = -5
AMG_ERR_BREAKDOWN = -6
AMG_ERR_UNSUPPORTED = -7

STATUS_NAMES = {
    0: "AMG_OK", 1: "AMG_NOT_CONVERGED", -1: "AMG_ERR_ARG", -2: "AMG_ERR_SINGULAR_BLOCK",
    -3: "AMG_ERR_NOT_SPD", -4: "AMG_ERR_OOM", -5: "AMG_ERR_HIP", -6: "AMG_ERR_BREAKDOWN",
    -7: "AMG_ERR_UNSUPPORTED",
}

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
KRYLOV = {"cg": 0, "fcg": 1, "ir": 2}
SETUP_PATHS = {"block": 0, "scalar": 1}
SMOOTHERS = {"jacobi": 0, "learned": 1, "spai0": 2, "ilu0": 3}
MAX_LEVELS = 16
MLP_PARAMS = 10374


class AmgParams(C.Structure):
    _fields_ = [
        ("eps_strong", C.c_double), ("eps_decay", C.c_double), ("omega_p", C.c_double),
        ("omega_j", C.c_double), ("npre", C.c_int32), ("npost", C.c_int32),
        ("coarse_enough", C.c_int32), ("max_levels", C.c_int32), ("use_nullspace", C.c_int32),
        ("precision", C.c_int32), ("krylov", C.c_int32), ("maxiter", C.c_int32),
        ("check_every", C.c_int32), ("max_restarts", C.c_int32), ("use_graphs", C.c_int32),
        ("nthreads", C.c_int32), ("autotune", C.c_int32), ("smoother", C.c_int32),
        ("accept_recurrence", C.c_int32), ("smoother_levels", C.c_int32), ("setup_path", C.c_int32),
        ("setup_device", C.c_int32),
    ]


class AmgBsr3(C.Structure):
    _fields_ = [("nb", C.c_int32), ("nnzb", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class AmgSolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("fell_back", C.c_int32), ("rel_true_residual", C.c_double),
                ("solve_ms", C.c_double)]


class AmgStats(C.Structure):
    _fields_ = [
        ("levels", C.c_int32), ("nb", C.c_int32 * MAX_LEVELS), ("nnzb_A", C.c_int64 * MAX_LEVELS),
        ("nnzb_P", C.c_int64 * MAX_LEVELS), ("n_agg", C.c_int32 * MAX_LEVELS),
        ("omega_j", C.c_double * MAX_LEVELS), ("n_coarse", C.c_int32),
        ("operator_complexity", C.c_double), ("setup_ms", C.c_double),
        ("device_bytes", C.c_double), ("vcycle_bytes", C.c_double), ("iter_bytes", C.c_double),
        ("layout_A", C.c_int32 * MAX_LEVELS), ("layout_P", C.c_int32 * MAX_LEVELS),
        ("layout_R", C.c_int32 * MAX_LEVELS),
        ("layout_AM", C.c_int32 * MAX_LEVELS), ("layout_G", C.c_int32 * MAX_LEVELS),
        ("setup_phase_ms", C.c_double * 11),
    ]


# (name, restype, argtypes) of every exported entry point
SIGNATURES = [
    ("amg_default_params", None, [C.POINTER(AmgParams)]),
    ("amg_last_error", C.c_char_p, []),
    ("amg_hierarchy_build", C.c_int, [C.POINTER(AmgBsr3), C.c_void_p, C.POINTER(AmgParams),
                                      C.POINTER(C.c_void_p)]),
    ("amg_hierarchy_free", None, [C.c_void_p]),
    ("amg_hierarchy_build_device", C.c_int, [C.POINTER(AmgBsr3), C.c_void_p, C.POINTER(AmgParams), C.c_void_p,
                                             C.POINTER(C.c_void_p)]),
    ("amg_hierarchy_stats", C.c_int, [C.c_void_p, C.POINTER(AmgStats)]),
    ("amg_hierarchy_level_shape", C.c_int, [C.c_void_p, C.c_int32, C.c_int32,
                                            C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                            C.POINTER(C.c_int64)]),
    ("amg_hierarchy_export", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                       C.c_void_p, C.c_void_p]),
    ("amg_setup", C.c_int, [C.POINTER(AmgBsr3), C.c_void_p, C.POINTER(AmgParams), C.c_void_p,
                            C.POINTER(C.c_void_p)]),
    ("amg_upload", C.c_int, [C.c_void_p, C.POINTER(AmgParams), C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    ("amg_destroy", None, [C.c_void_p]),
    ("amg_stats", C.c_int, [C.c_void_p, C.POINTER(AmgStats)]),
    ("amg_solve", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                            C.POINTER(AmgSolveInfo)]),
    ("amg_vcycle", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("amg_debug_apply", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    ("amg_true_residual", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.POINTER(C.c_double)]),
    ("amg_true_residual_noalloc", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.POINTER(C.c_double)]),
    ("amg_time_op", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                              C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("amg_solve_multi", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_double,
                                  C.POINTER(AmgSolveInfo)]),
    ("amg_setup_batch", C.c_int, [C.c_int32, C.POINTER(AmgBsr3), C.POINTER(C.c_void_p),
                                  C.POINTER(AmgParams), C.c_void_p, C.POINTER(C.c_void_p)]),
    ("amg_solve_batch", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.c_double, C.POINTER(AmgSolveInfo)]),
    ("amg_batch_destroy", None, [C.c_void_p]),
    ("amg_vcycle_batch", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    ("amg_vcycle_multi", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    ("amg_smoother_set_weights", C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_int32,
                                           C.POINTER(C.c_int32)]),
    ("amg_mlp_loss_grad", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_int32,
                                    C.POINTER(C.c_double), C.c_void_p]),
    ("amg_mlp_adam", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                               C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float]),
    ("amg_training_errors", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]),
]

_lib = None


def library_path() -> str:
    return os.path.join(_HERE, LIB_NAME)


def load(path: str | None = None):
    """Load the HIP library (built in-tree by the package build step).

    Raises RuntimeError if it has not been built: there is no fallback path.
    """
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or library_path()
    try:  # share PyTorch's HIP runtime when it is installed (one runtime per process)
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(p)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


class AmgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(lib, status: int, allow_not_converged: bool = True) -> int:
    if status == AMG_OK or (status == AMG_NOT_CONVERGED and allow_not_converged):
        return status
    raise AmgError(status, lib.amg_last_error().decode())
