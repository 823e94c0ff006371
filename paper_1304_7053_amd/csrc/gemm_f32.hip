// Kernel instances for element type float (all size classes, both batch forms).
#include "gemm_mfma.h"
#include "gemm_staged.h"

SBG_INSTANTIATE_GEMM(float)
