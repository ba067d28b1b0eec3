"""MI355X (gfx950) plane-wave block-LOBPCG eigensolver.

The computation lives in libpwlobpcg.so (HIP kernels behind the C ABI of
include/pwlobpcg.h); this package is its thin ctypes binding.  Importing it
does not load the library; `Context` does, and fails loudly if it is missing.
"""
from ._binding import (Context, PWError, PWStats, EXPORTS, apply_H_batch, fft_sizes, library_path,
                       load_library, PW_OK, PW_ERR_ARG, PW_ERR_STATE, PW_ERR_NOMEM,
                       PW_ERR_DEVICE, PW_ERR_NOT_CONVERGED, PW_ERR_NUMERIC, PW_PREC_FP64,
                       PW_PREC_MIXED, PW_PREC_MIXED_BF16, PW_PREC_MIXED_BF16_GRAM,
                       PW_PREC_MIXED_FP32_RR)
from .solver import PlaneWaveProblem, solve_batch

__all__ = ["Context", "PWError", "PWStats", "EXPORTS", "fft_sizes", "library_path",
           "load_library", "PlaneWaveProblem", "PW_OK", "PW_ERR_ARG", "PW_ERR_STATE",
           "PW_ERR_NOMEM", "PW_ERR_DEVICE", "PW_ERR_NOT_CONVERGED", "PW_ERR_NUMERIC",
           "PW_PREC_FP64", "PW_PREC_MIXED", "PW_PREC_MIXED_BF16", "PW_PREC_MIXED_BF16_GRAM",
           "PW_PREC_MIXED_FP32_RR",
           "solve_batch", "apply_H_batch"]
