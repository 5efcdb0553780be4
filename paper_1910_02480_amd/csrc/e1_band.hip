// E1 of the layer path in BF16 (Sec. 4.3: the first stride-2 3x3
// convolution, 7 input channels -> 32): the float32 input is staged in LDS.
//
// The generic layer kernel gathers the float32 input per lane and tap (7
// scattered 4-byte loads per pixel and tap), which made E1 the slowest layer
// of the layer path (about 1 TB/s at 128x128). Here a workgroup takes a band
// of BR = 256 / Wout output rows of one map: it loads the 2 BR + 1 input rows
// the band reads as whole 16-byte chunks (a map's rows are contiguous),
// writes them to LDS as BF16 with 8 channels per pixel (channel 7 = 0), and
// runs the MFMAs from there; the next band's chunks are loaded during this
// band's MFMAs. Operands, K order (k = tap * 8 + channel, lane group g taking
// tap 4 ks + g), rounding and epilogue are the generic kernel's, so the
// results are bitwise equal to it.
#include <hip/hip_runtime.h>

#include "drc_cae.h"
#include "conv_layer.h"
#include "internal.h"

namespace drc {
namespace {

constexpr int kThreads = 256;
constexpr int kBandPx = 256;     // output pixels per band (16 blocks of 16, 4 per wave)
constexpr int kChunks = 8;       // staged 16-byte chunks per thread (input rows of a band)
constexpr int kKSteps = 3;       // K = 9 taps x 8 channels, padded to 96
constexpr int kMaxRowPx = 1152;  // staged pixels: (2 BR + 1) Win = 2 * kBandPx * 2 + Win <= 1152 for Win <= 128

struct BandGeom {
    int bands_per_map, br;  // bands of a map, output rows per band
    long band0;             // first band of the class
};

struct E1Args {
    LayerArgs a;
    BandGeom bg[kMaxClasses];
    long total;
};

__global__ __launch_bounds__(kThreads) void e1_band_kernel(const E1Args e) {
    extern __shared__ __align__(16) char smem[];
    const LayerArgs& a = e.a;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    uint16_t* xs = (uint16_t*)smem;                // [pixel][8] bf16
    const int zoff = kMaxRowPx * 16;               // 16 zero bytes: taps left of the map
    // channel 7 of every staged pixel and the zero block stay zero: the
    // staging writes channels 0..6 only
    for (int i = tid; i < kMaxRowPx + 1; i += kThreads) *(uint4*)(smem + 16 * i) = make_uint4(0, 0, 0, 0);

    // A fragments of both 16-row blocks, every K step, from the row-major pack
    uint4 A[kKSteps][2];
#pragma unroll
    for (int ks = 0; ks < kKSteps; ++ks)
#pragma unroll
        for (int m = 0; m < 2; ++m)
            A[ks][m] = *(const uint4*)((const uint16_t*)a.wpack + (size_t)(16 * m + r16) * a.kstride + 32 * ks + 8 * g);

    auto class_of = [&](long item) {
        int c = 0;
#pragma unroll
        for (int k = 1; k < kMaxClasses; ++k)
            if (k < a.nclass && item >= e.bg[k].band0) c = k;
        return c;
    };
    // loads the 16-byte chunks of band `item` (input rows 2 oy0 - 1 .. 2 oy0 + 2 BR - 1);
    // every lane loads (rows above the map read the map's first chunk and are zeroed)
    float4 vf[kChunks];
    auto load_band = [&](long item) {
        const int c = class_of(item);
        const ClassGeom& G = a.cls[c];
        const long b = item - e.bg[c].band0;
        const int n = (int)(b / e.bg[c].bands_per_map), oy0 = (int)(b % e.bg[c].bands_per_map) * e.bg[c].br;
        const float* xm = (const float*)G.s0.p + (G.in_off ? G.in_off[n] : (long)n * G.Hin * G.Win * 7);
        const int rowf = G.Win * 7, nf4 = (2 * e.bg[c].br + 1) * rowf / 4;
        const long base = (long)(2 * oy0 - 1) * rowf;
#pragma unroll
        for (int k = 0; k < kChunks; ++k) {
            const int i = tid + kThreads * k;
            const int qi = 2 * oy0 - 1 + (4 * i) / rowf;
            const bool ok = i < nf4 && qi >= 0;
            const float4 v = *(const float4*)(xm + (ok ? base + 4L * i : 0L));
            vf[k] = ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };

    if (blockIdx.x < e.total) load_band(blockIdx.x);
    for (long item = blockIdx.x; item < e.total; item += gridDim.x) {
        const int c = class_of(item);
        const ClassGeom& G = a.cls[c];
        const int br = e.bg[c].br;
        const long b = item - e.bg[c].band0;
        const int n = (int)(b / e.bg[c].bands_per_map), oy0 = (int)(b % e.bg[c].bands_per_map) * br;
        const int Win = G.Win, Wout = G.Wout;
        const int nf4 = (2 * br + 1) * Win * 7 / 4;
        __syncthreads();  // the previous band's LDS reads are done
#pragma unroll
        for (int k = 0; k < kChunks; ++k) {
            const int i = tid + kThreads * k;
            if (i >= nf4) continue;
            // float j of chunk i is channel (4 i + j) % 7 of staged pixel (4 i + j) / 7
            const float f[4] = {vf[k].x, vf[k].y, vf[k].z, vf[k].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int q = 4 * i + j, pix = q / 7;
                xs[pix * 8 + (q - pix * 7)] = to_store<P_BF16>(f[j], 1.0f);
            }
        }
        __syncthreads();
        if (item + gridDim.x < e.total) load_band(item + gridDim.x);

        float bias[2][4];
        const int nb = G.seg0.c + G.seg1.c;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ch = 16 * m + 4 * g + r;
                bias[m][r] = (a.bias && ch < nb) ? a.bias[ch] : 0.0f;
            }
        f4 acc[2][4];
        int oyl[4], ox[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int q = (wave * 4 + p) * 16 + r16;  // output pixel of the band
            oyl[p] = q / Wout;
            ox[p] = q - oyl[p] * Wout;
#pragma unroll
            for (int m = 0; m < 2; ++m) acc[m][p] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int ks = 0; ks < kKSteps; ++ks) {
            const int t = 4 * ks + g, kh = t / 3, kw = t - 3 * (t / 3);
            uint4 bv[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                // staged row 0 is input row 2 oy0 - 1; rows past the map bottom are never read
                const bool ok = t < 9 && (kw > 0 || ox[p] > 0);
                const int off = ok ? ((2 * oyl[p] + kh) * Win + 2 * ox[p] + kw - 1) * 16 : zoff;
                bv[p] = *(const uint4*)(smem + off);
            }
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    acc[m][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A[ks][m]),
                                                                      __builtin_bit_cast(bf16x8, bv[p]), acc[m][p],
                                                                      0, 0, 0);
        }
        // epilogue: lane holds channels 16 m + 4 g .. + 3 of its pixel
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const long opix = ((long)n * G.Hout + oy0 + oyl[p]) * Wout + ox[p];
            const long doff0 = opix * G.seg0.ld, doff1 = opix * G.seg1.ld;
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int ch = 16 * m + 4 * g;
                float val[4] = {acc[m][p].x * a.acc_scale + bias[m][0], acc[m][p].y * a.acc_scale + bias[m][1],
                                acc[m][p].z * a.acc_scale + bias[m][2], acc[m][p].w * a.acc_scale + bias[m][3]};
                if (ch < G.seg0.c)
                    store_seg<P_BF16, false>(G.seg0, doff0, opix, ch, val);
                else if (ch - G.seg0.c < G.seg1.c)
                    store_seg<P_BF16, false>(G.seg1, doff1, opix, ch - G.seg0.c, val);
            }
        }
    }
}

}  // namespace

bool e1_band_fits(int Hin, int Win) {
    if (Win != 32 && Win != 64 && Win != 128) return false;
    const int Wout = Win / 2, br = kBandPx / Wout;
    return Hin % 2 == 0 && (Hin / 2) % br == 0 && (2 * br + 1) * Win <= kMaxRowPx &&
           (2 * br + 1) * Win * 7 / 4 <= kThreads * kChunks;
}

drc_status e1_band_forward(const LayerArgs& a, int num_cu, hipStream_t s) {
    E1Args e;
    e.a = a;
    long total = 0;
    for (int c = 0; c < a.nclass; ++c) {
        const ClassGeom& G = a.cls[c];
        if (!e1_band_fits(G.Hin, G.Win) || G.Hout * 2 != G.Hin || G.Wout * 2 != G.Win || a.raw_c != 7 ||
            G.s0.ld != 7 || a.kstride < 32 * kKSteps)
            return drc_fail(DRC_ERR_STATE, "e1 band: class %d (%dx%d) does not fit", c, G.Hin, G.Win);
        e.bg[c].br = kBandPx / G.Wout;
        e.bg[c].bands_per_map = G.Hout / e.bg[c].br;
        e.bg[c].band0 = total;
        total += (long)G.nmaps * e.bg[c].bands_per_map;
    }
    e.total = total;
    if (total == 0) return DRC_OK;
    const int lds = (kMaxRowPx + 1) * 16;
    const long grid = std::min(total, (long)num_cu * 2);  // two resident workgroups per CU (184 registers)
    hipLaunchKernelGGL(e1_band_kernel, dim3((unsigned)grid), dim3(kThreads), lds, s, e);
    return check_launch("e1 band");
}

}  // namespace drc
