// Layer-GEMM kernel instantiations for BF16.
#include "gemm_dispatch.h"

template drc_status run_gemm<P_BF16>(int, bool, LayerArgs&, int, int, hipStream_t);
