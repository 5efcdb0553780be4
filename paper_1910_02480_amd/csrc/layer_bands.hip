// Layer-path kernels whose input rows are staged in LDS by bands,
// for the first and the last layer of the autoencoder (Sec. 4.3), the two
// whose generic kernels were the slowest of the layer path.
//
// E1 (stride-2 3x3 convolution, 7 input channels -> 32): the generic
// kernel gathers the float32 input per lane and tap (7 scattered 4-byte
// loads per pixel and tap; about 1 TB/s at 128x128). Here a workgroup takes
// a band of BR = 256 / Wout output rows of one map: it loads the 2 BR + 1
// input rows the band reads as whole 16-byte chunks (a map's rows are
// contiguous), writes them to LDS in the compute type (BF16, or FP8 e4m3
// with the input's scale) with 8 channels per pixel (channel 7 = 0), and
// runs the MFMAs from there.
//
// D1 (stride-2 3x3 transposed convolution [u2 | h1] -> 3 channels, float32
// out, the four output phases merged into one 16-row block; BF16 or FP8): the generic
// kernel reads each input pixel from L2 once per GEMM pixel that has it as
// a neighbour (4 times). Here a workgroup stages BR = 256 / Win input rows
// plus the row below them (64 channels, 16-byte chunks) and gathers the
// neighbours from LDS.
//
// In both, the next band's chunks are loaded during this band's MFMAs, and
// operands, K order, rounding and epilogue are the generic kernels', so the
// results are bitwise equal to them.
#include <hip/hip_runtime.h>

#include "drc_cae.h"
#include "conv_layer.h"
#include "internal.h"

namespace drc {
namespace {

constexpr int kThreads = 256;
constexpr int kBandPx = 256;     // output pixels per band (16 blocks of 16, 4 per wave)
constexpr int kChunks = 8;       // E1: staged 16-byte chunks per thread (input rows of a band)
constexpr int kKSteps = 3;       // E1: K = 9 taps x 8 channels, padded to 96
constexpr int kMaxRowPx = 1152;  // E1: staged pixels, (2 BR + 1) Win = 2 * kBandPx * 2 + Win <= 1152 for Win <= 128
constexpr int kD1Chunks = 10;    // D1: staged 16-byte chunks per thread, (BR + 1) Win * 8 <= 2560
constexpr int kD1MaxPx = 320;    // D1: staged pixels, (BR + 1) Win = kBandPx + Win <= 320 for Win <= 64
constexpr int kD1YOff = kD1MaxPx * 144 + 32;  // D1: the band's output (2 BR rows x 2 Win x 3 floats = 12 KB),
                                              // after the staged pixels (at most 144 bytes each) and the zero block

struct BandGeom {
    int bands_per_map, br;  // bands of a map, output rows per band
    long band0;             // first band of the class
};

struct E1Args {
    LayerArgs a;
    BandGeom bg[kMaxClasses];
    long total;
};

// P = P_BF16: 3 K steps of 32 (lane group g takes tap 4 ks + g); P_FP8: one
// K step of 128 (lane group g takes taps 4 g .. 4 g + 3, 8 bytes each).
template <int P>
__global__ __launch_bounds__(kThreads) void e1_band_kernel(const E1Args e) {
    typedef typename Traits<P>::T T;
    typedef typename Traits<P>::V V;
    constexpr int PXB = 8 * (int)sizeof(T);        // staged bytes per pixel
    constexpr int KST = P == P_FP8 ? 1 : kKSteps;  // K steps
    extern __shared__ __align__(16) char smem[];
    const LayerArgs& a = e.a;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    T* xs = (T*)smem;                              // [pixel][8]
    const int zoff = kMaxRowPx * PXB;              // 16 zero bytes: taps left of the map
    // channel 7 of every staged pixel and the zero block stay zero: the
    // staging writes channels 0..6 only
    for (int i = tid; i < kMaxRowPx * PXB / 16 + 1; i += kThreads) *(uint4*)(smem + 16 * i) = make_uint4(0, 0, 0, 0);

    // A fragments of both 16-row blocks, every K step, from the row-major pack
    V A[KST][2];
#pragma unroll
    for (int ks = 0; ks < KST; ++ks)
#pragma unroll
        for (int m = 0; m < 2; ++m)
            A[ks][m] = *(const V*)((const T*)a.wpack + (size_t)(16 * m + r16) * a.kstride +
                                   ks * Traits<P>::KS + g * Traits<P>::VW);

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
                xs[pix * 8 + (q - pix * 7)] = to_store<P>(f[j], a.raw_qscale);
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
        // staged row 0 is input row 2 oy0 - 1; rows past the map bottom are never read
        auto tap_off = [&](int t, int p) {
            const int kh = t / 3, kw = t - 3 * (t / 3);
            const bool ok = t < 9 && (kw > 0 || ox[p] > 0);
            return ok ? ((2 * oyl[p] + kh) * Win + 2 * ox[p] + kw - 1) * PXB : zoff;
        };
#pragma unroll
        for (int ks = 0; ks < KST; ++ks) {
            V bv[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                if constexpr (P == P_FP8) {
                    uint2 h[4];
#pragma unroll
                    for (int s = 0; s < 4; ++s) h[s] = *(const uint2*)(smem + tap_off(4 * g + s, p));
                    bv[p] = __builtin_bit_cast(V, h);
                } else {
                    bv[p] = *(const V*)(smem + tap_off(4 * ks + g, p));
                }
            }
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int p = 0; p < 4; ++p) Traits<P>::mma(acc[m][p], A[ks][m], bv[p]);
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
                    store_seg<P, false>(G.seg0, doff0, opix, ch, val);
                else if (ch - G.seg0.c < G.seg1.c)
                    store_seg<P, false>(G.seg1, doff1, opix, ch - G.seg0.c, val);
            }
        }
    }
}


// D1: rows r = phase * 3 + co of the 16-row block (12 used), K = (neighbour,
// channel) in steps of 32 (8 steps); lane group g of step ks takes neighbour
// ks / 2, channels 32 (ks % 2) + 8 g .. + 8 (u2 below 32, h1 above).
// P = P_BF16: 8 K steps of 32 (above); P_FP8: 2 K steps of 128, lane group g
// of step ks taking neighbour 2 ks + g / 2, channels 32 (g % 2) .. + 32.
template <int P>
__global__ __launch_bounds__(kThreads) void d1_band_kernel(const E1Args e) {
    typedef typename Traits<P>::T T;
    typedef typename Traits<P>::V V;
    constexpr int ES = (int)sizeof(T);
    constexpr int PIXB = 64 * ES + 16;     // staged bytes per pixel (64 channels + 16 against bank conflicts)
    constexpr int CPS = 2 * ES;            // 16-byte chunks per source (32 channels)
    constexpr int CPP = 2 * CPS;           // chunks per pixel
    constexpr int KST = 256 / Traits<P>::KS;
    extern __shared__ __align__(16) char smem[];
    const LayerArgs& a = e.a;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int zoff = kD1MaxPx * PIXB;  // 32 zero bytes: neighbours right of the map
    if (tid < 2) *(uint4*)(smem + zoff + 16 * tid) = make_uint4(0, 0, 0, 0);

    V A[KST];
#pragma unroll
    for (int ks = 0; ks < KST; ++ks)
        A[ks] = *(const V*)((const T*)a.wpack + (size_t)r16 * a.kstride + ks * Traits<P>::KS + g * Traits<P>::VW);
    float bias[4];
    int rph[4], rco[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = g * 4 + r;
        rph[r] = row / 3;
        rco[r] = row - (row / 3) * 3;
        bias[r] = (a.bias && row < 12) ? a.bias[rco[r]] : 0.0f;
    }

    auto class_of = [&](long item) {
        int c = 0;
#pragma unroll
        for (int k = 1; k < kMaxClasses; ++k)
            if (k < a.nclass && item >= e.bg[k].band0) c = k;
        return c;
    };
    // chunks of band `item`: input rows a0 .. a0 + BR (the last one only when
    // inside the map), pixel by pixel 4 chunks of u2 then 4 of h1; every lane
    // loads (rows below the map read the map's first chunk and are zeroed)
    typedef uint4 Piece[kD1Chunks];
    auto load_band = [&](long item, Piece& vq) {
        const int c = class_of(item);
        const ClassGeom& G = a.cls[c];
        const long b = item - e.bg[c].band0;
        const int n = (int)(b / e.bg[c].bands_per_map), a0 = (int)(b % e.bg[c].bands_per_map) * e.bg[c].br;
        const int nch = (e.bg[c].br + 1) * G.Win * CPP;
        const long pix0 = ((long)n * G.Hin + a0) * G.Win;
#pragma unroll
        for (int k = 0; k < kD1Chunks; ++k) {
            const int i = tid + kThreads * k;
            const int px = i / CPP, part = i % CPP;
            const bool ok = i < nch && a0 + px / G.Win < G.Hin;
            const long pix = ok ? pix0 + px : 0;
            const T* src = part < CPS ? (const T*)G.s0.p + pix * G.s0.ld + (16 / ES) * part
                                      : (const T*)G.s1.p + pix * G.s1.ld + (16 / ES) * (part - CPS);
            const uint4 v = *(const uint4*)src;
            vq[k] = ok ? v : make_uint4(0, 0, 0, 0);
        }
    };

    // BF16: two bands in flight per workgroup, band item + 2 G (G =
    // gridDim.x) loaded while band item is computed and stored and band
    // item + G waiting in the other set of registers; FP8 (whose registers
    // would then drop it to one workgroup per CU): one band ahead
    constexpr bool kTwo = P != P_FP8;
    const long step = (kTwo ? 2L : 1L) * gridDim.x;
    auto run_band = [&](long item, Piece& vq) {
        const int c = class_of(item);
        const ClassGeom& G = a.cls[c];
        const int br = e.bg[c].br;
        const long b = item - e.bg[c].band0;
        const int n = (int)(b / e.bg[c].bands_per_map), a0 = (int)(b % e.bg[c].bands_per_map) * br;
        const int Win = G.Win;
        const int nch = (br + 1) * Win * CPP;
        __syncthreads();  // the previous band's LDS reads are done
#pragma unroll
        for (int k = 0; k < kD1Chunks; ++k) {
            const int i = tid + kThreads * k;
            if (i < nch) *(uint4*)(smem + (i / CPP) * PIXB + (i % CPP) * 16) = vq[k];
        }
        __syncthreads();
        if (item + step < e.total) load_band(item + step, vq);

        f4 acc[4];
        int al[4], bj[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int q = (wave * 4 + p) * 16 + r16;  // GEMM pixel of the band
            al[p] = q / Win;
            bj[p] = q - al[p] * Win;
            acc[p] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int ks = 0; ks < KST; ++ks) {
            // neighbour and byte offset of this lane's K elements within the staged pixel
            const int nb = P == P_FP8 ? 2 * ks + (g >> 1) : ks >> 1, di = nb >> 1, dj = nb & 1;
            const int cb = P == P_FP8 ? 32 * (g & 1) : (4 * (ks & 1) + g) * 16;
            V bv[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                // the row below the band is staged (zero below the map)
                const bool ok = !dj || bj[p] + 1 < Win;
                const int off = ok ? ((al[p] + di) * Win + bj[p] + dj) * PIXB + cb : zoff;
                bv[p] = *(const V*)(smem + off);
            }
#pragma unroll
            for (int p = 0; p < 4; ++p) Traits<P>::mma(acc[p], A[ks], bv[p]);
        }
        // epilogue: lane holds rows 4 g .. 4 g + 3 = (phase, channel) of its
        // GEMM pixel; the band's 2 BR output rows (contiguous in y) are
        // assembled in LDS and written with 16-byte stores
        float* ys = (float*)(smem + kD1YOff);
        const int Wout = G.Wout;
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (g * 4 + r >= 12) continue;
                const int ph = rph[r], co = rco[r];
                float v = acc[p][r] * a.acc_scale + bias[r];
                if (G.seg0.relu) v = relu(v);
                ys[((2 * al[p] + (ph >> 1)) * Wout + 2 * bj[p] + (ph & 1)) * 3 + co] = v;
            }
        __syncthreads();
        const long ybase = (G.out_off ? G.out_off[n] : (long)n * G.Hout * Wout * 3) + (long)2 * a0 * Wout * 3;
        float* yd = (float*)G.seg0.dst + ybase;
        const int nf = 2 * br * Wout * 3;  // floats of the band, a multiple of 4
        if (((uintptr_t)yd & 15) == 0) {
            for (int i = tid; i < nf / 4; i += kThreads) ((float4*)yd)[i] = ((const float4*)ys)[i];
        } else {
            for (int i = tid; i < nf; i += kThreads) yd[i] = ys[i];
        }
    };
    Piece va, vb;
    if (blockIdx.x < e.total) load_band(blockIdx.x, va);
    if (kTwo && blockIdx.x + (long)gridDim.x < e.total) load_band(blockIdx.x + (long)gridDim.x, vb);
    for (long item = blockIdx.x; item < e.total; item += step) {
        run_band(item, va);
        if (kTwo && item + gridDim.x < e.total) run_band(item + gridDim.x, vb);
    }
}

}  // namespace

bool e1_band_fits(int Hin, int Win) {
    if (Win != 32 && Win != 64 && Win != 128) return false;
    const int Wout = Win / 2, br = kBandPx / Wout;
    return Hin % 2 == 0 && (Hin / 2) % br == 0 && (2 * br + 1) * Win <= kMaxRowPx &&
           (2 * br + 1) * Win * 7 / 4 <= kThreads * kChunks;
}

drc_status e1_band_forward(const LayerArgs& a, int prec, int num_cu, hipStream_t s) {
    E1Args e;
    e.a = a;
    long total = 0;
    for (int c = 0; c < a.nclass; ++c) {
        const ClassGeom& G = a.cls[c];
        if (!e1_band_fits(G.Hin, G.Win) || G.Hout * 2 != G.Hin || G.Wout * 2 != G.Win || a.raw_c != 7 ||
            G.s0.ld != 7 || a.kstride < (prec == P_FP8 ? 128 : 32 * kKSteps) || (prec != P_BF16 && prec != P_FP8))
            return drc_fail(DRC_ERR_STATE, "e1 band: class %d (%dx%d) does not fit", c, G.Hin, G.Win);
        e.bg[c].br = kBandPx / G.Wout;
        e.bg[c].bands_per_map = G.Hout / e.bg[c].br;
        e.bg[c].band0 = total;
        total += (long)G.nmaps * e.bg[c].bands_per_map;
    }
    e.total = total;
    if (total == 0) return DRC_OK;
    const long grid = std::min(total, (long)num_cu * 2);  // two resident workgroups per CU (184 registers)
    if (prec == P_FP8)
        hipLaunchKernelGGL(e1_band_kernel<P_FP8>, dim3((unsigned)grid), dim3(kThreads), kMaxRowPx * 8 + 16, s, e);
    else
        hipLaunchKernelGGL(e1_band_kernel<P_BF16>, dim3((unsigned)grid), dim3(kThreads), kMaxRowPx * 16 + 16, s, e);
    return check_launch("e1 band");
}

bool d1_band_fits(int Hin, int Win) {
    if (Win != 16 && Win != 32 && Win != 64) return false;
    const int br = kBandPx / Win;
    return Hin % br == 0 && (br + 1) * Win <= kD1MaxPx && (br + 1) * Win * 8 <= kThreads * kD1Chunks;
}

drc_status d1_band_forward(const LayerArgs& a, int prec, int num_cu, int per_cu, hipStream_t s) {
    E1Args e;
    e.a = a;
    long total = 0;
    for (int c = 0; c < a.nclass; ++c) {
        const ClassGeom& G = a.cls[c];
        if (!d1_band_fits(G.Hin, G.Win) || G.Hout != 2 * G.Hin || G.Wout != 2 * G.Win || G.s0.c != 32 ||
            G.s1.c != 32 || G.s0.ld % 16 || G.s1.ld % 16 || G.seg0.c != 3 || G.seg0.ld != 3 || a.kstride < 256 ||
            a.raw_c || (prec != P_BF16 && prec != P_FP8))
            return drc_fail(DRC_ERR_STATE, "d1 band: class %d (%dx%d) does not fit", c, G.Hin, G.Win);
        e.bg[c].br = kBandPx / G.Win;
        e.bg[c].bands_per_map = G.Hin / e.bg[c].br;
        e.bg[c].band0 = total;
        total += (long)G.nmaps * e.bg[c].bands_per_map;
    }
    e.total = total;
    if (total == 0) return DRC_OK;
    // per_cu persistent workgroups per CU (two resident at a time): alone,
    // two; beside another stream's launches, more and shorter band lists, so
    // that workgroups that start late finish with the rest
    const long grid = std::min(total, (long)num_cu * std::max(1, per_cu));
    if (prec == P_FP8)
        hipLaunchKernelGGL(d1_band_kernel<P_FP8>, dim3((unsigned)grid), dim3(kThreads), kD1YOff + 12 * kBandPx * 4, s,
                           e);
    else
        hipLaunchKernelGGL(d1_band_kernel<P_BF16>, dim3((unsigned)grid), dim3(kThreads), kD1YOff + 12 * kBandPx * 4, s,
                           e);
    return check_launch("d1 band");
}

}  // namespace drc
