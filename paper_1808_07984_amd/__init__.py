"""Strassen-fused GEMM for AMD MI355X (gfx950).

One- and two-level Strassen matrix multiplication fused into a blocked MFMA
GEMM (Huang, Yu, van de Geijn, "Implementing Strassen's Algorithm with CUTLASS
on NVIDIA Volta GPUs", FLAME Working Note #88), re-designed for CDNA4: operand
sums are formed while tiles are staged into LDS, products run on the matrix
cores, and each product is scattered with its signs into the C blocks in the
kernel epilogue.  No workspace, no device allocation (the hybrid two-level
and the formed one-level schedules take caller workspace).

    import paper_1808_07984_amd as sg
    sg.gemm(A, B, C, alpha=1.0, beta=1.0, levels=1)      # torch tensors
    sg.strassen_gemm(m, n, k, pA, lda, pB, ldb, pC, ldc, alpha, beta, levels)
    sg.gemm_formed(A, B, C, mode="bf16x3")   # one level, sums formed first (levels=2: two)

The C ABI (include/strassen.h) lives in _build/libstrassen.so; this package
binds it with ctypes.  Importing fails if the library is not built.
"""
from ._binding import (  # noqa: F401
    LIB_PATH,
    STRASSEN_BF16,
    STRASSEN_F16,
    STRASSEN_F32,
    STRASSEN_MAX_LEVELS,
    STRASSEN_MODE_BF16X3,
    STRASSEN_MODE_PLAIN,
    STRASSEN_SCHEDULE_BATCHED,
    STRASSEN_SCHEDULE_CONCURRENT,
    STRASSEN_SCHEDULE_STREAMS,
    STRASSEN_TILE_128,
    STRASSEN_TILE_256,
    STRASSEN_TILE_AUTO,
    StrassenError,
    strassen_build_id,
    strassen_error_string,
    strassen_gemm,
    strassen_gemm_ex,
    strassen_gemm_formed,
    strassen_gemm_formed_ex,
    strassen_gemm_formed_noalloc,
    STRASSEN_NOALLOC_SCRATCH_BYTES,
    STRASSEN_ERROR_SCRATCH_LIMIT,
    strassen_formed_workspace_size,
    strassen_formed_workspace_size_ex,
    strassen_gemm_hybrid,
    strassen_hybrid_workspace_size,
    strassen_plan_info,
    strassen_plan_instances,
    strassen_profile_start,
    strassen_profile_stop,
    strassen_probe_mfma,
    strassen_set_schedule,
    strassen_set_stream,
    strassen_set_tile,
)
from .api import gemm, gemm_formed, gemm_hybrid, plan_info  # noqa: F401
from .autograd import StrassenMatmul, strassen_matmul  # noqa: F401
