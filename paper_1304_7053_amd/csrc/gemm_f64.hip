// Kernel instances for element type double (all size classes, both batch forms).
#include "gemm_mfma.h"

SBG_INSTANTIATE_GEMM(double)
