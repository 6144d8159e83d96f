"""ctypes declarations of libpmg.so (include/pmg.h).  Argument marshalling
only: every computation runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmg.so")

PMG_OK = 0
PMG_ERR_INVALID_ARG = -1
PMG_ERR_UNSUPPORTED = -2
PMG_ERR_DEGENERATE = -3
PMG_ERR_HIP = -4
PMG_ERR_OOM = -5
PMG_ERR_BREAKDOWN = -6
PMG_WARN_NOT_CONVERGED = 1

PMG_FP64 = 0
PMG_FP32 = 1
PMG_BF16_FP32ACC = 2
PMG_BF16X3_FP32ACC = 3
PMG_PATCH_INTERIOR = 0
PMG_PATCH_WITH_BOUNDARY = 1
PMG_COARSE_ARITHMETIC = 0
PMG_COARSE_GEOMETRIC = 1
PMG_COARSE_HARMONIC = 2
PMG_BOUNDS_LANCZOS = 0
PMG_BOUNDS_FIXED = 1

PMG_SMOOTHER_CHEBYSHEV = 0
PMG_SMOOTHER_CARTESIAN = 1

PMG_Q_N_PATCHES = 0
PMG_Q_N_COLORS = 1
PMG_Q_N_LEVELS = 2
PMG_Q_N_DOFS = 3
PMG_Q_N_INTERIOR_DOFS = 4
PMG_Q_DEVICE_BYTES = 5
PMG_Q_N_BOUNDARY_PATCHES = 6
PMG_Q_LOCAL_DOFS = 7
PMG_Q_TUNED_GRID = 8
PMG_Q_TUNED_MAP = 9
PMG_BQ_N_INSTANCES = 0
PMG_BQ_CAPTURES = 1
PMG_BQ_REPLAYS = 2
PMG_Q_COLOR_OFFSET = 16
PMG_Q_LEVEL_DEGREE = 32
PMG_Q_LEVEL_SIZE = 48

EXPORTS = [
    "pmg_default_opts", "pmg_patch_setup", "pmg_patch_smooth", "pmg_patch_smooth_colors",
    "pmg_patch_residual", "pmg_patch_apply", "pmg_patch_local_solve", "pmg_patch_pcg",
    "pmg_set_smoother", "gmg_set_post_direction", "gmg_gmres_solve", "pmg_patch_smooth_additive",
    "gmg_set_additive",
    "pmg_get_inv_diag",
    "pmg_get_bounds", "pmg_set_bounds", "pmg_get_patch_vertices", "pmg_query",
    "pmg_patch_destroy", "gmg_setup", "gmg_apply", "gmg_vcycle", "gmg_cg_solve", "gmg_query",
    "gmg_level_smoother", "gmg_destroy", "pmg_last_error", "pmg_patches_setup",
    "pmg_patch_features", "pmg_mlp_param_count", "pmg_mlp_create", "pmg_mlp_get_params",
    "pmg_mlp_set_params", "pmg_mlp_fit_standardizer", "pmg_mlp_get_standardizer",
    "pmg_mlp_set_standardizer", "pmg_mlp_predict", "pmg_mlp_gradient", "pmg_mlp_train",
    "pmg_mlp_destroy", "pmg_set_bounds_mlp", "pmg_set_launch", "pmg_autotune",
    "pmg_batch_setup", "pmg_batch_instance", "pmg_batch_smooth", "pmg_batch_smooth_eager",
    "pmg_batch_autotune", "pmg_batch_query", "pmg_batch_destroy", "pmg_mlp_save", "pmg_mlp_load",
    "pmg_mlp_fit_bounds", "pmg_patch_pcg_noalloc",
    "pmg_simplex_numbering", "pmg_simplex_setup", "pmg_simplex_query", "pmg_simplex_set_bounds",
    "pmg_simplex_get_inv_diag", "pmg_simplex_apply", "pmg_simplex_local_solve", "pmg_simplex_pcg",
    "pmg_simplex_destroy",
]


class PmgMesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_cells", ctypes.c_int32),
                ("vertices", ctypes.POINTER(ctypes.c_double))]


class PmgOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("levels", ctypes.c_int32 * 8), ("cheb_degree", ctypes.c_int32),
                ("n_vcycles", ctypes.c_int32), ("bounds", ctypes.c_int32),
                ("lanczos_steps", ctypes.c_int32), ("cheb_safety", ctypes.c_double),
                ("cheb_range", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("stream", ctypes.c_void_p), ("patch_set", ctypes.c_int32),
                ("coarse_mean", ctypes.c_int32)]


class PmgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libpmg status {status}: {message}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libpmg.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2510_17785_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    F = ctypes.POINTER(ctypes.c_float)
    i32 = ctypes.c_int32
    sig = {
        "pmg_default_opts": [ctypes.POINTER(PmgOpts)],
        "pmg_patch_setup": [ctypes.POINTER(PmgMesh), D, i32, ctypes.POINTER(PmgOpts),
                            ctypes.POINTER(P)],
        "pmg_patch_smooth": [P, P, P, i32],
        "pmg_patch_smooth_colors": [P, P, P, i32, i32],
        "pmg_patch_residual": [P, P, P, P],
        "pmg_patch_apply": [P, i32, P, P],
        "pmg_patch_local_solve": [P, P, P],
        "pmg_patch_pcg": [P, P, P, ctypes.c_double, i32, P, P],
        "pmg_patch_pcg_noalloc": [P, P, P, ctypes.c_double, i32, P, P],
        "pmg_simplex_numbering": [i32, ctypes.POINTER(i32), i32, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "pmg_simplex_setup": [i32, ctypes.c_int64, D, ctypes.POINTER(i32), D, i32, ctypes.POINTER(PmgOpts),
                              ctypes.POINTER(P)],
        "pmg_simplex_query": [P, i32, ctypes.POINTER(ctypes.c_int64)],
        "pmg_simplex_set_bounds": [P, D],
        "pmg_simplex_get_inv_diag": [P, i32, P],
        "pmg_simplex_apply": [P, i32, P, P],
        "pmg_simplex_local_solve": [P, P, P],
        "pmg_simplex_pcg": [P, P, P, ctypes.c_double, i32, P, P],
        "pmg_simplex_destroy": [P],
        "pmg_set_smoother": [P, i32, ctypes.c_double],
        "pmg_patch_smooth_additive": [P, P, P, ctypes.c_double],
        "gmg_set_post_direction": [P, i32],
        "gmg_set_additive": [P, ctypes.c_double],
        "gmg_gmres_solve": [P, P, P, ctypes.c_double, i32, ctypes.POINTER(i32),
                            ctypes.POINTER(ctypes.c_double)],
        "pmg_get_inv_diag": [P, i32, P],
        "pmg_get_bounds": [P, D],
        "pmg_set_bounds": [P, D],
        "pmg_get_patch_vertices": [P, ctypes.POINTER(ctypes.c_int32)],
        "pmg_query": [P, i32, ctypes.POINTER(ctypes.c_int64)],
        "pmg_patch_destroy": [P],
        "gmg_setup": [ctypes.POINTER(PmgMesh), D, i32, ctypes.POINTER(PmgOpts), ctypes.POINTER(P)],
        "gmg_apply": [P, P, P],
        "gmg_vcycle": [P, P, P],
        "gmg_cg_solve": [P, P, P, ctypes.c_double, i32, ctypes.POINTER(i32),
                         ctypes.POINTER(ctypes.c_double)],
        "gmg_query": [P, i32, ctypes.POINTER(ctypes.c_int64)],
        "gmg_level_smoother": [P, i32, ctypes.POINTER(P)],
        "gmg_destroy": [P],
        "pmg_last_error": [],
        "pmg_patches_setup": [i32, ctypes.c_int64, D, D, i32, ctypes.POINTER(PmgOpts),
                              ctypes.POINTER(P)],
        "pmg_patch_features": [P, P],
        "pmg_mlp_param_count": [i32, i32, ctypes.POINTER(ctypes.c_int64)],
        "pmg_mlp_create": [i32, i32, F, ctypes.c_int64, P, ctypes.POINTER(P)],
        "pmg_mlp_get_params": [P, F],
        "pmg_mlp_set_params": [P, F],
        "pmg_mlp_fit_standardizer": [P, P, ctypes.c_int64],
        "pmg_mlp_get_standardizer": [P, F, F],
        "pmg_mlp_set_standardizer": [P, F, F],
        "pmg_mlp_predict": [P, P, ctypes.c_int64, P],
        "pmg_mlp_gradient": [P, P, P, ctypes.c_int64, F, ctypes.POINTER(ctypes.c_double)],
        "pmg_mlp_train": [P, P, P, ctypes.c_int64, P, i32, i32, ctypes.c_float, D],
        "pmg_mlp_destroy": [P],
        "pmg_mlp_fit_bounds": [P, P, P, ctypes.c_int64, P, ctypes.c_int64, i32, i32, ctypes.c_float, D, F, D],
        "pmg_set_bounds_mlp": [P, P, ctypes.c_double, ctypes.c_double,
                               ctypes.POINTER(ctypes.c_int64)],
        "pmg_set_launch": [P, i32, i32],
        "pmg_autotune": [P, P, P, F],
        "pmg_batch_setup": [ctypes.POINTER(PmgMesh), ctypes.POINTER(D), ctypes.POINTER(i32), i32,
                            ctypes.POINTER(PmgOpts), ctypes.POINTER(P)],
        "pmg_batch_instance": [P, i32, ctypes.POINTER(P)],
        "pmg_batch_smooth": [P, ctypes.POINTER(P), ctypes.POINTER(P), i32],
        "pmg_batch_smooth_eager": [P, ctypes.POINTER(P), ctypes.POINTER(P), i32],
        "pmg_batch_autotune": [P, ctypes.POINTER(P), ctypes.POINTER(P)],
        "pmg_batch_query": [P, i32, ctypes.POINTER(ctypes.c_int64)],
        "pmg_batch_destroy": [P],
        "pmg_mlp_save": [P, ctypes.c_double, ctypes.c_char_p],
        "pmg_mlp_load": [ctypes.c_char_p, ctypes.c_int64, P, ctypes.POINTER(P),
                         ctypes.POINTER(ctypes.c_double)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name == "pmg_last_error" else ctypes.c_int
    _lib = lib
    return lib


def check(status: int) -> int:
    if status < 0:
        msg = load().pmg_last_error().decode(errors="replace")
        raise PmgError(status, msg)
    return status
