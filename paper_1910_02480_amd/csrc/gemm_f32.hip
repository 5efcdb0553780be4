// Layer-GEMM kernel instantiations for F32.
#include "gemm_dispatch.h"

template drc_status run_gemm<P_F32>(int, bool, LayerArgs&, int, int, hipStream_t);
