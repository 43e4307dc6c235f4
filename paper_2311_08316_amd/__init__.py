"""CQRRPT on MI355X (gfx950): randomized pivoted CholeskyQR for tall matrices.

The computation runs in the HIP library ``libcqrrpt.so`` (C ABI in
``include/cqrrpt.h``); this package is its Python binding.
"""

from ._binding import (CQRRPT_FP64, CQRRPT_MIXED, CQRRPT_MIXED_CHECKED,
                       CQRRPT_MIXED_FP32_CHOLQR2, NOALLOC_SCRATCH_BYTES, SKETCH_GAUSSIAN,
                       SKETCH_SRHT, STAGES, CqrrptError, CqrrptInfo, Factorization, Server,
                       colmajor, empty_colmajor, empty_colmajor_ld, factor, factor_dense,
                       factor_hqrrp, factor_implicit, factor_noalloc_into, factor_sync, hqrrp,
                       lib, padded_ld, probe_copy, probe_mfma, qrcp, saso_sample, sketch,
                       sketched_cholqr, stage_timing, stage_times, workspace_bytes)

__all__ = [
    "CQRRPT_FP64", "CQRRPT_MIXED", "CQRRPT_MIXED_CHECKED", "CQRRPT_MIXED_FP32_CHOLQR2",
    "NOALLOC_SCRATCH_BYTES", "SKETCH_GAUSSIAN", "SKETCH_SRHT", "STAGES", "CqrrptError",
    "CqrrptInfo", "Factorization", "Server", "colmajor", "empty_colmajor", "empty_colmajor_ld",
    "factor", "factor_dense", "factor_hqrrp", "factor_implicit", "factor_noalloc_into",
    "factor_sync", "hqrrp", "lib", "padded_ld", "probe_copy", "probe_mfma", "qrcp",
    "saso_sample", "sketch", "sketched_cholqr", "stage_timing", "stage_times", "workspace_bytes",
]
