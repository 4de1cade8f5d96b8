"""qrvie: compressed volume-integral-equation solves on one MI355X.

Thin Python layer over the C ABI of libqrvie (include/qrvie.h).  PyTorch provides
device memory and the stream; every step of the solve runs in the library's HIP
kernels.  Importing this package does not touch the GPU; the library is loaded on
first use and a missing library raises (there is no CPU fallback).
"""
from ._lib import (PREC_BF16X2, PREC_C64, PREC_C64_F32, PREC_C64_ONLY, PREC_C128, SOLVE_BLOCK,  # noqa: F401
                   SOLVE_BLOCK_IR, SOLVE_FP64, SOLVE_MIXED_IR)
from .api import (Context, Geometry, Operator, QrvieError, assemble, rhs_plane_waves)  # noqa: F401

__all__ = ["Context", "Geometry", "Operator", "QrvieError", "assemble", "rhs_plane_waves",
           "PREC_C128", "PREC_C64", "PREC_C64_ONLY", "PREC_C64_F32", "PREC_BF16X2", "SOLVE_FP64", "SOLVE_MIXED_IR", "SOLVE_BLOCK",
           "SOLVE_BLOCK_IR"]
