"""MI355X (gfx950) hot path of localized-collision Projective Dynamics.

The compute lives in libpdschur.so (hand-written HIP kernels behind a C ABI,
declared in include/pdschur.h).  This package is a thin ctypes binding with
the same entry-point names; PyTorch is only used for device memory and the
current HIP stream.  Importing the package does not load the library; the
first call does, and fails loudly if it has not been built.
"""
from ._lib import (MLP, DenseCholesky, chol_factor_noalloc, PD_CHOL_NOALLOC_MAX_N, PDContext, PDError, load_library, library_path, PD_FP64, PD_FP32_IR,
                   PD_BF16_IR, PD_ERR_IR_STALLED, PD_ERR_NOT_SPD, nd_analyse)

__all__ = ["MLP", "DenseCholesky", "chol_factor_noalloc", "PD_CHOL_NOALLOC_MAX_N", "PDContext", "PDError", "load_library", "library_path", "PD_FP64",
           "PD_FP32_IR", "PD_BF16_IR", "PD_ERR_IR_STALLED", "PD_ERR_NOT_SPD", "nd_analyse"]
