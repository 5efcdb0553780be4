// Compile-time dispatch of the layer-GEMM kernel instantiations. Each
// precision's instantiations are compiled in their own translation unit
// (gemm_f32.hip, gemm_bf16.hip, gemm_fp8.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "drc_cae.h"
#include "common.h"
#include "conv_layer.h"
#include "internal.h"

using namespace drc;

// ------------------------------------------------------------------ GEMM dispatch
// Compile-time facts of one layer-GEMM instantiation: K step, packed row
// length, LDS bytes for the weight pack and whether it is staged in LDS.
template <int P, int MODE, int CIN, int COUTP>
struct GemmCfg {
    static constexpr int KS = (P == P_F32) ? 16 : (P == P_BF16 ? 32 : 128);
    static constexpr int ES = (P == P_F32) ? 4 : (P == P_BF16 ? 2 : 1);
    static constexpr int KSTRIDE = (((MODE == M_TCONV ? 4 : 9) * CIN) + KS - 1) / KS * KS;
    static constexpr int LDS = COUTP * wlds_row_bytes(KSTRIDE, ES);
    static constexpr bool WLDS = LDS <= 80 * 1024;
};

template <int P, int MODE, int CIN, int C0, int COUTP, int NPW, bool RAW, bool OF32>
static drc_status launch_one(const LayerArgs& a, dim3 grid, hipStream_t s) {
    typedef GemmCfg<P, MODE, CIN, COUTP> C;
    auto kern = conv_layer_kernel<P, MODE, CIN, C0, COUTP, NPW, RAW, OF32, C::WLDS>;
    const int lds = C::WLDS ? C::LDS : 0;
    if (lds > 64 * 1024) {
        static bool attr_set = false;
        if (!attr_set) {
            if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds) !=
                hipSuccess)
                return drc_fail(DRC_ERR_HIP, "gemm: cannot raise the LDS limit to %d bytes", lds);
            attr_set = true;
        }
    }
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, a);
    return check_launch("gemm");
}

// Numbers the work items of every class and launches the persistent grid.
template <int P, int MODE, int CIN, int C0, int COUTP, bool RAW, bool OF32>
static drc_status launch_gemm(LayerArgs& a, int npw, int num_cu, hipStream_t s) {
    typedef GemmCfg<P, MODE, CIN, COUTP> C;
    if (a.kstride != C::KSTRIDE) return drc_fail(DRC_ERR_STATE, "gemm: weight pack stride mismatch");
    long items = 0;
    for (int c = 0; c < a.nclass; ++c) {
        ClassGeom& G = a.cls[c];
        const long npix = (long)G.nmaps * G.Hg * G.Wg;
        if (G.tile_px <= 0) G.tile_px = 64 * npw;
        G.item0 = items;
        G.items = (npix + G.tile_px - 1) / G.tile_px;
        items += G.items;
    }
    a.total_items = items;
    if (items == 0) return DRC_OK;
    const int nphase = MODE == M_TCONV ? 4 : 1;
    const int per_cu = C::WLDS ? std::max(1, std::min(4, (160 * 1024) / C::LDS)) : 4;
    const long want = ((long)num_cu * per_cu + nphase - 1) / nphase;
    dim3 grid((unsigned)std::min(items, want), nphase);
    constexpr int MT = COUTP / 16;
    switch (npw) {
        case 1:
            if constexpr (MT * 1 <= 16) return launch_one<P, MODE, CIN, C0, COUTP, 1, RAW, OF32>(a, grid, s);
            break;
        case 2:
            if constexpr (MT * 2 <= 16) return launch_one<P, MODE, CIN, C0, COUTP, 2, RAW, OF32>(a, grid, s);
            break;
        case 4:
            if constexpr (MT * 4 <= 16) return launch_one<P, MODE, CIN, C0, COUTP, 4, RAW, OF32>(a, grid, s);
            break;
        case 8:
            if constexpr (MT * 8 <= 16) return launch_one<P, MODE, CIN, C0, COUTP, 8, RAW, OF32>(a, grid, s);
            break;
    }
    return drc_fail(DRC_ERR_UNSUPPORTED, "gemm: tile npw=%d not built", npw);
}

template <int P>
drc_status run_gemm(int layer, bool bwd, LayerArgs& a, int npw, int num_cu, hipStream_t s) {
    if (!bwd) {
        switch (layer) {
            case 0: return launch_gemm<P, M_CONV, 8, 8, 32, true, false>(a, npw, num_cu, s);
            case 1: return launch_gemm<P, M_CONV, 32, 32, 64, false, false>(a, npw, num_cu, s);
            case 2: return launch_gemm<P, M_CONV, 64, 64, 128, false, false>(a, npw, num_cu, s);
            case 3: return launch_gemm<P, M_TCONV, 128, 128, 64, false, false>(a, npw, num_cu, s);
            case 4: return launch_gemm<P, M_TCONV, 128, 64, 32, false, false>(a, npw, num_cu, s);
            case 5: return launch_gemm<P, M_TCONV, 64, 32, 16, false, true>(a, npw, num_cu, s);
        }
    } else {
        if constexpr (P == P_FP8) {
            return drc_fail(DRC_ERR_UNSUPPORTED, "backward: FP8 is inference only");
        } else {
            constexpr int D1C = (P == P_F32) ? 4 : 8;
            switch (layer) {
                case 5: return launch_gemm<P, M_CONV, D1C, D1C, 64, true, false>(a, npw, num_cu, s);
                case 4: return launch_gemm<P, M_CONV, 32, 32, 128, false, false>(a, npw, num_cu, s);
                case 3: return launch_gemm<P, M_CONV, 64, 64, 128, false, false>(a, npw, num_cu, s);
                case 2: return launch_gemm<P, M_TCONV, 128, 128, 64, false, false>(a, npw, num_cu, s);
                case 1: return launch_gemm<P, M_TCONV, 64, 64, 32, false, false>(a, npw, num_cu, s);
                case 0: return launch_gemm<P, M_TCONV, 32, 32, 16, false, true>(a, npw, num_cu, s);
            }
        }
    }
    return drc_fail(DRC_ERR_INVALID_ARG, "gemm: layer %d", layer);
}


