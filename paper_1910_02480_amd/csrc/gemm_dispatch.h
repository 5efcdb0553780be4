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

// Compile-time facts of one layer-GEMM instantiation: K step, packed row
// length, weight rows, LDS bytes for the weight pack and whether it is
// staged in LDS. MODE: M_CONV, M_TCONV_PAIRS or M_TCONV_MERGED; ROWS: output
// channels (merged: per phase).
template <int P, int MODE, int CIN, int ROWS>
struct GemmCfg {
    static constexpr int KS = (P == P_F32) ? 16 : (P == P_BF16 ? 32 : 128);
    static constexpr int ES = (P == P_F32) ? 4 : (P == P_BF16 ? 2 : 1);
    static constexpr int RUP = (ROWS + 15) / 16 * 16;
    static constexpr int MROWS = (4 * ROWS + 15) / 16 * 16;
    static constexpr int KSTRIDE = MODE == M_CONV ? (9 * CIN + KS - 1) / KS * KS
                                 : MODE == M_TCONV_PAIRS ? (CIN + KS - 1) / KS * KS
                                                         : (4 * CIN + KS - 1) / KS * KS;
    static constexpr int WROWS = MODE == M_CONV ? RUP : (MODE == M_TCONV_PAIRS ? 9 * RUP : MROWS);
    static constexpr int LDS = WROWS * wlds_row_bytes(KSTRIDE, ES);
    static constexpr bool WLDS = LDS <= 160 * 1024;
    // weights read from L2: split the row blocks over up to 4 waves for reuse
    static constexpr int RB = MODE == M_TCONV_MERGED ? MROWS / 16 : RUP / 16;
    static constexpr int WM = (WLDS || MODE == M_TCONV_MERGED) ? 1 : (RB % 4 == 0 ? 4 : (RB % 2 == 0 ? 2 : 1));
    // accumulator blocks per wave and 16-pixel block
    static constexpr int MT = MODE == M_TCONV_PAIRS ? 4 * RB / WM : RB / WM;
};

template <typename K>
static drc_status launch_kernel(K kern, const LayerArgs& a, dim3 grid, int lds, hipStream_t s) {
    if (lds > 64 * 1024) {
        // raising the limit is idempotent; done before the first launch of each instantiation
        if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
            return drc_fail(DRC_ERR_HIP, "gemm: cannot raise the LDS limit to %d bytes", lds);
    }
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, a);
    return check_launch("gemm");
}

template <int P, int MODE, int CIN, int C0, int ROWS, int NPW, bool RAW, bool OF32>
static drc_status launch_one(const LayerArgs& a, dim3 grid, hipStream_t s) {
    typedef GemmCfg<P, MODE, CIN, ROWS> C;
    const int lds = C::WLDS ? C::LDS : 0;
    if constexpr (MODE == M_CONV)
        return launch_kernel(conv_layer_kernel<P, MODE, CIN, C0, C::RUP, NPW, RAW, OF32, C::WLDS, C::WM>, a, grid, lds, s);
    else if constexpr (MODE == M_TCONV_PAIRS)
        return launch_kernel(tconv_pairs_kernel<P, CIN, C0, C::RUP, NPW, OF32, C::WLDS, C::WM>, a, grid, lds, s);
    else
        return launch_kernel(tconv_merged_kernel<P, CIN, C0, ROWS, C::MROWS, NPW, OF32, C::WLDS>, a, grid, lds, s);
}

// Largest tile (pixel blocks of 16 per wave) built for an accumulator of MT blocks.
__host__ __device__ constexpr bool npw_ok(int mt, int npw) { return mt * npw <= 16; }

// Numbers the work items of every class and launches the persistent grid.
template <int P, int MODE, int CIN, int C0, int ROWS, bool RAW, bool OF32>
static drc_status launch_gemm(LayerArgs& a, int npw, int num_cu, hipStream_t s) {
    typedef GemmCfg<P, MODE, CIN, ROWS> C;
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
    const int per_cu = C::WLDS ? std::max(1, std::min(4, (160 * 1024) / C::LDS)) : 4;
    dim3 grid((unsigned)std::min(items, (long)num_cu * per_cu), 1);
    switch (npw) {
        case 1:
            if constexpr (npw_ok(C::MT, 1)) return launch_one<P, MODE, CIN, C0, ROWS, 1, RAW, OF32>(a, grid, s);
            break;
        case 2:
            if constexpr (npw_ok(C::MT, 2)) return launch_one<P, MODE, CIN, C0, ROWS, 2, RAW, OF32>(a, grid, s);
            break;
        case 4:
            if constexpr (npw_ok(C::MT, 4)) return launch_one<P, MODE, CIN, C0, ROWS, 4, RAW, OF32>(a, grid, s);
            break;
        case 8:
            if constexpr (npw_ok(C::MT, 8)) return launch_one<P, MODE, CIN, C0, ROWS, 8, RAW, OF32>(a, grid, s);
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
            case 3: return launch_gemm<P, M_TCONV_PAIRS, 128, 128, 64, false, false>(a, npw, num_cu, s);
            case 4: return launch_gemm<P, M_TCONV_PAIRS, 128, 64, 32, false, false>(a, npw, num_cu, s);
            case 5: return launch_gemm<P, M_TCONV_MERGED, 64, 32, 3, false, true>(a, npw, num_cu, s);
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
                case 2: return launch_gemm<P, M_TCONV_PAIRS, 128, 128, 64, false, false>(a, npw, num_cu, s);
                case 1: return launch_gemm<P, M_TCONV_PAIRS, 64, 64, 32, false, false>(a, npw, num_cu, s);
                case 0: return launch_gemm<P, M_TCONV_MERGED, 32, 32, 7, false, true>(a, npw, num_cu, s);
            }
        }
    }
    return drc_fail(DRC_ERR_INVALID_ARG, "gemm: layer %d", layer);
}
