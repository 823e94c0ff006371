// Kernel instances for element type double (all size classes, both batch forms).
#include "gemm_vbatched.h"
#include "gemm_vbteam.h"
#include "gemm_staged.h"
#include "gemm_blocked.h"
#include "gemm_team.h"
#include "trsm.h"

SBG_INSTANTIATE_GEMM(double)
SBG_INSTANTIATE_TRSM(double)
