"""ctypes mirror of include/rmg.h and loader of the in-tree HIP library.

The library must have been built (``__graft_entry__.build()`` or
``python -m paper_1903_08741_amd.build_lib``); there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RMG_LIBRARY") or os.path.join(HERE, "librmg.so")

RMG_OK, RMG_EINVAL, RMG_ENOMEM, RMG_EHIP, RMG_ENOTCONV = 0, -1, -2, -3, -4
SAMPLE_OK, SAMPLE_MAXITER, SAMPLE_NONFINITE = 0, 1, 2
GARDNER, VGM, LINEAR = 0, 1, 2
QOI_MEAN_SATURATION, QOI_BOTTOM_OUTFLUX = 0, 1
FP64, MIXED = 0, 1
CYCLE_V, CYCLE_W = 1, 2
FLAG_FORCE_STREAMING = 1
FLAG_EAGER = 2
FLAG_STATE_GLOBAL = 4
FLAG_NO_AUTOTUNE = 8
FLAG_TILES_16 = 16
FLAG_WHOLE_WHERE_FITS = 32
FLAG_COARSE_TOP_32 = 64
FLAG_CONFINE = 128
FLAG_NO_CONFINE = 256

COST_WORK, COST_TIME = 0, 1

EXPORTED = ("rmg_struct_size", "rmg_ctx_create", "rmg_ctx_destroy", "rmg_last_error",
            "rmg_ctx_set_workspace_limit", "rmg_ctx_tune_dump", "sample_fields", "picard_mg_solve", "picard_mg_solve_noalloc",
            "mlmc_level_estimate",
            "rmg_set_kernel_timing", "rmg_get_kernel_timing", "pc_mlmc", "rmg_mlmc_optimal_samples",
            "picard_mg_adjoint", "picard_mg_outflux")


class Marginal(C.Structure):
    _fields_ = [("shift", C.c_double), ("log_mean", C.c_double), ("scale", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("model", C.c_int32), ("n_steps", C.c_int32), ("qoi", C.c_int32), ("init_profile", C.c_int32),
                ("theta_r", C.c_double), ("theta_s", C.c_double), ("gardner_a", C.c_double),
                ("linear_c0", C.c_double), ("vg_alpha_shift", C.c_double), ("vg_n_shift", C.c_double),
                ("h_top", C.c_double), ("h_bottom", C.c_double), ("h_init", C.c_double), ("dt", C.c_double),
                ("init_rate", C.c_double)]


class SolverOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("cycle", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("cycles_per_picard", C.c_int32), ("max_picard", C.c_int32), ("coarsest_n", C.c_int32),
                ("flags", C.c_int32), ("fallback_cycles", C.c_int32), ("fallback_max_picard", C.c_int32),
                ("eps_mg", C.c_double), ("eps_picard", C.c_double)]


class SampleStats(C.Structure):
    _fields_ = [("picard_its", C.c_int32), ("mg_cycles", C.c_int32), ("steps_done", C.c_int32),
                ("status", C.c_int32), ("final_dp_inf", C.c_double), ("attempts", C.c_int32),
                ("reserved", C.c_int32)]


class DD(C.Structure):
    _fields_ = [("hi", C.c_double), ("lo", C.c_double)]


class LevelSums(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_failed", C.c_int64), ("picard_its", C.c_int64),
                ("mg_cycles", C.c_int64), ("mg_cycles_coarse", C.c_int64), ("n_retried", C.c_int64),
                ("sY", DD), ("sY2", DD), ("sQf", DD), ("sQf2", DD),
                ("sQc", DD), ("sQc2", DD)]


class Level(C.Structure):
    _fields_ = [("n_fine", C.c_int32), ("n_coarse", C.c_int32), ("n_samples", C.c_int64),
                ("fine", Problem), ("coarse", Problem), ("d_basis_fine", C.c_void_p),
                ("d_basis_coarse", C.c_void_p), ("d_xi", C.c_void_p)]


class PcLevel(C.Structure):
    _fields_ = [("n_fine", C.c_int32), ("n_coarse", C.c_int32), ("n_warmup", C.c_int64),
                ("fine", Problem), ("coarse", Problem), ("d_basis_fine", C.c_void_p),
                ("d_basis_coarse", C.c_void_p)]


class PcOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("bias_rate", C.c_double), ("cost_model", C.c_int32),
                ("max_rounds", C.c_int32), ("max_pairs", C.c_int64), ("max_pairs_per_call", C.c_int64)]


class PcLevelOut(C.Structure):
    _fields_ = [("drawn", C.c_int64), ("target", C.c_int64), ("W", C.c_double), ("V", C.c_double),
                ("mean", C.c_double), ("sums", LevelSums)]


class PcResult(C.Structure):
    _fields_ = [("mean", C.c_double), ("var", C.c_double), ("sampling_err2", C.c_double),
                ("bias", C.c_double), ("total_cost", C.c_double), ("wall_ms", C.c_double),
                ("rounds", C.c_int32), ("converged", C.c_int32), ("calls", C.c_int64),
                ("bias_pairs", C.c_int64)]


# int (*rmg_xi_source)(void* user, int level, int64_t first, int64_t count, double* h_xi)
XiSource = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.POINTER(C.c_double))


class KernelTiming(C.Structure):
    _fields_ = [("launches", C.c_int64), ("cells", C.c_int64), ("total_ms", C.c_double),
                ("algo_bytes", C.c_double)]


TIME_NONE, TIME_SMOOTHER_DOWN, TIME_COARSE, TIME_FINE = 0, 1, 2, 4

STRUCTS = {"rmg_kernel_timing": KernelTiming, "rmg_problem": Problem, "rmg_solver_opts": SolverOpts, "rmg_sample_stats": SampleStats,
           "rmg_level_sums": LevelSums, "rmg_level": Level, "rmg_marginal": Marginal,
           "rmg_pc_level": PcLevel, "rmg_pc_opts": PcOpts, "rmg_pc_level_out": PcLevelOut,
           "rmg_pc_result": PcResult}

_lib = None


def lib():
    """Load librmg.so once and declare the exported signatures; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first "
                           "(there is no fallback implementation)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int, C.c_int64
    L.rmg_struct_size.argtypes = [C.c_char_p]
    L.rmg_struct_size.restype = i64
    L.rmg_ctx_create.argtypes = [C.POINTER(vp), i32, C.c_char_p]
    L.rmg_ctx_create.restype = i32
    L.rmg_ctx_set_workspace_limit.argtypes = [vp, i64]
    L.rmg_ctx_set_workspace_limit.restype = i32
    L.rmg_ctx_tune_dump.argtypes = [vp, C.c_char_p, i64]
    L.rmg_ctx_tune_dump.restype = i64
    L.rmg_ctx_destroy.argtypes = [vp]
    L.rmg_ctx_destroy.restype = None
    L.rmg_last_error.argtypes = [vp]
    L.rmg_last_error.restype = C.c_char_p
    L.sample_fields.argtypes = [vp, i32, i32, i32, vp, vp, C.POINTER(Marginal), i64, vp, vp]
    L.sample_fields.restype = i32
    L.picard_mg_solve.argtypes = [vp, i32, C.POINTER(Problem), C.POINTER(SolverOpts), vp, i64, vp, vp, vp,
                                  vp, vp]
    L.picard_mg_solve.restype = i32
    L.picard_mg_solve_noalloc.argtypes = L.picard_mg_solve.argtypes
    L.picard_mg_solve_noalloc.restype = i32
    L.mlmc_level_estimate.argtypes = [vp, i32, C.POINTER(Level), i32, i32, C.POINTER(Marginal),
                                      C.POINTER(SolverOpts), C.POINTER(LevelSums), vp, vp]
    L.mlmc_level_estimate.restype = i32
    L.picard_mg_adjoint.argtypes = [vp, i32, C.POINTER(Problem), C.POINTER(SolverOpts), i32, vp,
                                    C.POINTER(Marginal), vp, i64, i32, C.c_double, vp, vp, vp, vp, vp]
    L.picard_mg_adjoint.restype = i32
    L.picard_mg_outflux.argtypes = [vp, i32, C.POINTER(Problem), C.POINTER(SolverOpts), i32, vp,
                                    C.POINTER(Marginal), vp, i64, vp, vp, vp, vp]
    L.picard_mg_outflux.restype = i32
    L.pc_mlmc.argtypes = [vp, i32, C.POINTER(PcLevel), i32, i32, C.POINTER(Marginal), C.POINTER(SolverOpts),
                          C.POINTER(PcOpts), XiSource, vp, C.POINTER(PcLevelOut), C.POINTER(PcResult), vp]
    L.pc_mlmc.restype = i32
    L.rmg_mlmc_optimal_samples.argtypes = [i32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                                           C.POINTER(C.c_int64)]
    L.rmg_mlmc_optimal_samples.restype = i32
    L.rmg_set_kernel_timing.argtypes = [vp, i32]
    L.rmg_set_kernel_timing.restype = i32
    L.rmg_get_kernel_timing.argtypes = [vp, i32, C.POINTER(KernelTiming)]
    L.rmg_get_kernel_timing.restype = i32
    for name, cls in STRUCTS.items():
        got = L.rmg_struct_size(name.encode())
        if got != C.sizeof(cls):
            raise RuntimeError(f"ABI mismatch: {name} is {got} bytes in the library, {C.sizeof(cls)} here")
    _lib = L
    return L
