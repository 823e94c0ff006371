"""Parity of every kernel path the launcher can select, not only the default
one: the team kernel for sizes <= 8 wherever it applies, the MFMA tile
kernels for those sizes (with the LDS-staged kernel for packed strided
batches, the prefetching (pipelined) direct kernel, the extreme tile unrolls
-- one tile per group, and the largest unroll the size class allows -- a
persistent grid of one work-group per CU walking many work units, and one of
32 work-groups per CU, more than can be resident).  Each path reruns the parity cases
of the default path (same oracle, same 4 max(k,1) u acceptance test), and the
kernel name the library reports confirms which kernel ran."""
import numpy as np
import pytest

import test_gpu_parity as P
from paper_1304_7053_amd import sbg
from gpu_util import say

pytestmark = pytest.mark.gpu

PATHS = {
    "team": dict(path=2),
    "staged": dict(staged=1, pipeline=0, path=1),
    "pipelined": dict(staged=0, pipeline=1, path=1),
    "unroll1": dict(staged=0, pipeline=0, tile_bytes=256, tile_bytes16=256, path=1),
    "unrollmax": dict(staged=0, pipeline=0, tile_bytes=1 << 20, tile_bytes16=1 << 20, path=1),
    "onewg": dict(staged=0, pipeline=0, wg_per_cu=1, xcd_chunk=1, path=1),
    "oversub": dict(staged=0, pipeline=0, wg_per_cu=32, path=1),
}


def _kernel(dtype, s, batch):
    t = {np.float32: "s", np.float64: "d", np.complex64: "c", np.complex128: "z"}[np.dtype(dtype).type]
    return sbg.describe_strided(t, "N", "N", s, s, s, s, s * s, s, s * s, s, s * s, batch)


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("dtype", P.ALL, ids=lambda d: np.dtype(d).name)
def test_path_parity(gpu_lib, path, dtype):
    with sbg.tuned(**PATHS[path]):
        name = _kernel(dtype, 8, 100_000)
        say(f"path {path} {np.dtype(dtype).name}: {name}")
        if path == "team":
            assert "gemm_team_kernel" in name
        elif path == "staged":
            assert "gemm_staged_kernel" in name
        else:
            assert "gemm_mfma_kernel" in name
            pipe_flag = name[: name.index(">(")].split(",")[-1].strip()
            assert pipe_flag == ("true" if path == "pipelined" else "false")
        P.test_square_sizes_all_op_pairs(gpu_lib, dtype)
        P.test_rectangular_random_shapes(gpu_lib, dtype)
        P.test_padded_layout_gaps_untouched(gpu_lib, dtype)
        P.test_alpha_zero_and_beta_zero_special_cases(gpu_lib, dtype)
        P.test_shared_operand_and_k_zero(gpu_lib, dtype)
        P.test_device_scalar_mode(gpu_lib, dtype)


@pytest.mark.parametrize("path", ["team", "staged", "pipelined", "oversub"])
@pytest.mark.parametrize("dtype", P.REAL, ids=lambda d: np.dtype(d).name)
def test_path_full_size(gpu_lib, path, dtype):
    """The N = 100,000 size sweep through the alternative paths."""
    with sbg.tuned(**PATHS[path]):
        P.test_full_size_square_sweep(gpu_lib, dtype)


@pytest.mark.parametrize("path", ["team", "staged", "pipelined"])
def test_path_integer_bit_exact(gpu_lib, path):
    with sbg.tuned(**PATHS[path]):
        for dtype in P.ALL:
            P.test_integer_data_bit_exact(gpu_lib, dtype, "strided")


@pytest.mark.parametrize("path", ["staged", "pipelined"])
def test_path_narrow_inputs(gpu_lib, path):
    """bf16 / f16 inputs and the three-term bf16 split through the alternative
    paths (the fp8 path carries per-matrix scales and always runs direct)."""
    import test_gpu_precision as Q
    with sbg.tuned(**PATHS[path]):
        for fmt in ("bf16", "f16"):
            Q.test_half_inputs_strided(gpu_lib, fmt, "uniform")
        Q.test_bf16x3_strided(gpu_lib, "logu")
