// Layer-GEMM kernel instantiations for FP8.
#include "gemm_dispatch.h"

template drc_status run_gemm<P_FP8>(int, bool, LayerArgs&, int, int, hipStream_t);
