"""ctypes declarations of the C ABI in include/qrvie.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqrvie.so")

MAX_LEVELS = 24
OK, ERR_INVALID_ARG, ERR_GEOMETRY, ERR_OUT_OF_MEMORY, ERR_DEVICE, NOT_CONVERGED, ERR_QUEUE_FULL = range(7)
PREC_C128, PREC_C64, PREC_BF16X2, PREC_C64_ONLY, PREC_C64_F32 = 0, 1, 2, 3, 4
SOLVE_FP64, SOLVE_MIXED_IR, SOLVE_BLOCK, SOLVE_BLOCK_IR = 0, 1, 2, 3


class C128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class ArrayDescC(C.Structure):
    _fields_ = [("n", C.c_int32), ("centers", C.POINTER(C.c_double)), ("radius", C.POINTER(C.c_double)),
                ("height", C.POINTER(C.c_double)), ("eps_r", C.POINTER(C128)), ("n_eps", C.c_int32),
                ("lattice_ij", C.POINTER(C.c_int32)), ("pitch", C.c_double), ("wavelength", C.c_double),
                ("cells_per_particle", C.c_int32), ("shape", C.c_int32), ("grid", C.c_int32)]


class CompressOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("far_prec", C.c_int32), ("near_prec", C.c_int32),
                ("max_block_rows", C.c_int64), ("share_transpose", C.c_int32), ("seed", C.c_uint64),
                ("verbose", C.c_int32), ("chunk_bytes", C.c_int64), ("compression", C.c_int32),
                ("aca_start", C.c_int32), ("aca_stop", C.c_double)]


class OpStats(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_blocks", C.c_int64), ("n_blocks_level", C.c_int64 * MAX_LEVELS),
                ("min_rank_level", C.c_int32 * MAX_LEVELS), ("max_rank_level", C.c_int32 * MAX_LEVELS),
                ("mean_rank_level", C.c_double * MAX_LEVELS), ("n_self_types", C.c_int32),
                ("n_qr_entries", C.c_int64), ("gain", C.c_double), ("max_block_rel_err", C.c_double),
                ("apply_bytes", C.c_int64), ("device_bytes", C.c_int64), ("t_assembly_s", C.c_double),
                ("t_compression_s", C.c_double), ("t_precond_setup_s", C.c_double),
                ("apply_bytes_c64", C.c_int64), ("n_aca", C.c_int64), ("n_aca_resumed", C.c_int64),
                ("n_aca_retried", C.c_int64), ("n_aca_sketch", C.c_int64)]


class BlockInfo(C.Structure):
    _fields_ = [("level", C.c_int32), ("m", C.c_int32), ("n", C.c_int32), ("rank", C.c_int32),
                ("row_first", C.c_int32), ("row_count", C.c_int32), ("col_first", C.c_int32),
                ("col_count", C.c_int32), ("rel_err", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("max_iter", C.c_int32), ("mode", C.c_int32), ("tol", C.c_double),
                ("use_x0", C.c_int32), ("inner_tol", C.c_double), ("verbose", C.c_int32),
                ("block_width", C.c_int32), ("inner_fp32", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("rel_res_prec", C.c_double), ("rel_res_true", C.c_double), ("n_apply", C.c_int32),
                ("n_prec", C.c_int32), ("t_apply_s", C.c_double), ("t_prec_s", C.c_double),
                ("t_krylov_s", C.c_double), ("t_total_s", C.c_double), ("n_reorth", C.c_int32),
                ("n_refine", C.c_int32), ("basis_ortho", C.c_double)]


class ServerOptsC(C.Structure):
    _fields_ = [("slots", C.c_int32), ("hbm_budget", C.c_size_t), ("eps", C.c_double), ("restart", C.c_int32),
                ("max_iter", C.c_int32), ("mode", C.c_int32), ("block_width", C.c_int32), ("op_cache", C.c_int32),
                ("seed", C.c_uint64), ("tune_tiles", C.c_int32), ("max_bypass", C.c_int32)]


TUNE_VARIANTS = 8


class BlockTune(C.Structure):
    _fields_ = [("nrhs_tile", C.c_int32), ("n_variants", C.c_int32), ("u", C.c_int32 * TUNE_VARIANTS),
                ("rows_per_wave", C.c_int32 * TUNE_VARIANTS), ("ms", (C.c_double * TUNE_VARIANTS) * 3),
                ("mismatches", (C.c_int64 * TUNE_VARIANTS) * 3), ("chosen", C.c_int32 * 3)]


class ServerStatsC(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64), ("refused", C.c_int64),
                ("running", C.c_int64), ("queued", C.c_int64), ("ops_built", C.c_int64), ("cache_hits", C.c_int64),
                ("evictions", C.c_int64), ("rhs_solved", C.c_int64), ("latency_p50_s", C.c_double),
                ("latency_p99_s", C.c_double), ("queue_wait_p50_s", C.c_double), ("makespan_s", C.c_double),
                ("requests_per_s", C.c_double), ("rhs_solves_per_s", C.c_double), ("peak_bytes", C.c_size_t),
                ("in_use_bytes", C.c_size_t)]


P = C.c_void_p
PP = C.POINTER(C.c_void_p)
I32 = C.c_int32
I64 = C.c_int64
ST = C.c_int

SIGNATURES = {
    "qrvie_status_string": (C.c_char_p, [ST]),
    "qrvie_ctx_create": (ST, [C.c_int, P, C.c_size_t, PP]),
    "qrvie_ctx_destroy": (None, [P]),
    "qrvie_last_error": (C.c_char_p, [P]),
    "qrvie_ctx_bytes_in_use": (C.c_size_t, [P]),
    "qrvie_ctx_peak_bytes": (C.c_size_t, [P, I32]),
    "qrvie_geom_create": (ST, [P, C.POINTER(ArrayDescC), PP]),
    "qrvie_geom_ndof": (I64, [P]),
    "qrvie_geom_nlevels": (I32, [P]),
    "qrvie_geom_order": (ST, [P, C.POINTER(I32)]),
    "qrvie_geom_cells": (ST, [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "qrvie_geom_blocks": (ST, [P, C.POINTER(I32)]),
    "qrvie_geom_destroy": (None, [P]),
    "qrvie_assemble": (ST, [P, P, I32, C.POINTER(I32), I32, C.POINTER(I32), P, I64]),
    "qrvie_op_footprint_estimate": (ST, [P, C.POINTER(CompressOpts), C.POINTER(C.c_size_t)]),
    "qrvie_op_create": (ST, [P, P, C.POINTER(CompressOpts), PP]),
    "qrvie_op_stats_get": (ST, [P, C.POINTER(OpStats)]),
    "qrvie_op_num_blocks": (I64, [P]),
    "qrvie_op_export_block": (ST, [P, I64, C.POINTER(BlockInfo), P, P]),
    "qrvie_op_export_self": (ST, [P, I32, P, P]),
    "qrvie_op_destroy": (None, [P]),
    "qrvie_apply": (ST, [P, P, I32, P, I64, P, I64]),
    "qrvie_apply_prec": (ST, [P, P, I32, I32, P, I64, P, I64]),
    "qrvie_apply_noalloc": (ST, [P, P, P, P]),
    "qrvie_op_profile_apply": (ST, [P, P, I32, I32, C.POINTER(C.c_double), C.POINTER(I64)]),
    "qrvie_op_profile_block": (ST, [P, P, I32, I32, C.POINTER(C.c_double), C.POINTER(I64)]),
    "qrvie_op_tune_block": (ST, [P, P, I32, I32, I32, C.POINTER(BlockTune)]),
    "qrvie_probe_read": (ST, [P, P, C.c_size_t, I32, C.POINTER(C.c_double)]),
    "qrvie_probe_mfma": (ST, [P, I32, C.POINTER(C.c_double)]),
    "qrvie_precondition": (ST, [P, P, I32, P, I64, P, I64]),
    "qrvie_rhs_plane_waves": (ST, [P, P, I32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(I32), P, I64]),
    "qrvie_solve": (ST, [P, P, I32, P, I64, P, I64, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
    "qrvie_solve_footprint_estimate": (ST, [P, P, I32, C.POINTER(SolveOpts), C.POINTER(C.c_size_t)]),
    "qrvie_server_create": (ST, [C.c_int, C.POINTER(ServerOptsC), PP]),
    "qrvie_server_submit": (ST, [P, C.POINTER(ArrayDescC), I32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(I32), C.c_double, C.POINTER(C.c_uint64)]),
    "qrvie_server_poll": (ST, [P, C.c_uint64, C.POINTER(I32)]),
    "qrvie_server_wait": (ST, [P, C.c_uint64, C.c_double, C.POINTER(I32)]),
    "qrvie_server_fetch": (ST, [P, C.c_uint64, P, I64, C.POINTER(SolveInfo)]),
    "qrvie_server_get_stats": (ST, [P, C.POINTER(ServerStatsC)]),
    "qrvie_server_request_times": (ST, [P, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]),
    "qrvie_server_last_error": (C.c_char_p, [P]),
    "qrvie_server_destroy": (None, [P]),
}

_lib = None


def _torch_runtime_first():
    """PyTorch ships its own HIP runtime next to the one this library links.  Both can serve
    one process, but only if torch's initialises first (otherwise torch reports no device),
    so a GPU-enabled torch is initialised before the library can make any HIP call."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load() -> C.CDLL:
    """Load libqrvie.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    _torch_runtime_first()
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_10586_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
