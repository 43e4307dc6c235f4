"""CQRRPT on MI355X (gfx950): randomized pivoted CholeskyQR for tall matrices.

The computation runs in the HIP library ``libcqrrpt.so`` (C ABI in
``include/cqrrpt.h``); this package is its Python binding.
"""

from ._binding import (CQRRPT_FP64, CQRRPT_MIXED, CQRRPT_MIXED_CHECKED, CQRRPT_MIXED_FP32_CHOLQR2, CqrrptError, CqrrptInfo, Factorization,
                       Server, colmajor, empty_colmajor, factor, factor_implicit, factor_noalloc_into,
                       factor_sync, factor_dense, SKETCH_GAUSSIAN, SKETCH_SRHT, NOALLOC_SCRATCH_BYTES, lib, probe_copy, probe_mfma, qrcp,
                       saso_sample, sketch, sketched_cholqr, stage_timing, stage_times, workspace_bytes, STAGES)

__all__ = [
    "CQRRPT_FP64", "CQRRPT_MIXED", "CQRRPT_MIXED_CHECKED", "CQRRPT_MIXED_FP32_CHOLQR2", "CqrrptError", "CqrrptInfo", "Factorization", "Server",
    "colmajor",
    "empty_colmajor", "factor", "factor_implicit", "factor_noalloc_into", "factor_sync",
    "factor_dense", "SKETCH_GAUSSIAN", "SKETCH_SRHT",
    "NOALLOC_SCRATCH_BYTES", "lib", "probe_copy", "probe_mfma", "qrcp", "saso_sample", "sketch", "sketched_cholqr",
    "workspace_bytes", "stage_timing", "stage_times", "STAGES",
]
