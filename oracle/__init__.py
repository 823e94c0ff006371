"""CPU oracle for batched small-matrix GEMM (and, in oracle.blas, batched GEMV
and TRSM) -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package.  The product path (paper_1304_7053_amd) never imports it.
"""
from .oracle import (  # noqa: F401
    TYPE_CODES, gemm, gemm_strided, gemm_general, bound_strided, bound_general,
    set_threads, max_threads, encode_e4m3, round_bf16, decode, quant_e4m3, gemm_split3_general,
)
