// Implicit-GEMM kernel for the two layer types of the radiance-cache
// autoencoder (Sec. 4.3): the stride-2 3x3 convolution of the encoder and
// the stride-2 3x3 transposed convolution of the decoder.
//
// GEMM view (A = packed weights, B = gathered activations):
//   D[co][pix] = sum_{tap, ci} Wp[co][tap*CIN_EFF + ci] * X[in(pix, tap)][ci]
// * conv (M_CONV): pix = output pixel (n,p,q), taps (kh,kw) in 3x3, input
//   pixel (2p+kh-1, 2q+kw-1).
// * transposed conv (M_TCONV): the output is split by parity into four
//   phases (py,px) (grid.y). Phase pixel (a,b) is output (2a+py, 2b+px);
//   row taps are {kh=1 -> i=a} for py=0 and {kh=0 -> i=a+1, kh=2 -> i=a}
//   for py=1, columns likewise, so the phases use 1, 2, 2 and 4 taps.
// The data gradient of a convolution is a transposed convolution with the
// channel-transposed weight and vice versa, so the same kernel runs the
// backward data pass with a transposed weight pack and a different
// epilogue.
//
// Execution: persistent workgroups of 4 waves. A workgroup stages its
// phase's packed weights in LDS once (when they fit, WLDS) and then walks
// work items (tiles of GEMM pixels) with a grid stride. Each wave owns all
// COUT_PAD rows and NPW blocks of 16 consecutive GEMM pixels; the gather of
// the next K step's activations is issued before the MFMAs of the current
// one. The GEMM row (output channel) dimension sits on the MFMA A side, so
// each lane ends with four consecutive channels of one pixel and stores
// them as one vector.
//
// One launch may cover up to four resolution classes (maps of different
// sizes): each class has its own geometry, tensors and tile size, and work
// items are numbered class after class.
#pragma once
#include "common.h"

namespace drc {

enum Mode : int { M_CONV = 0, M_TCONV = 1 };

// One source of input channels; a channel concatenation is two sources.
struct Src {
    const void* p;
    int c;   // channels taken from this source
    int ld;  // elements between consecutive pixels
};

// One output segment: a contiguous range of GEMM rows with its own tensor.
struct Seg {
    void* dst;
    int c;            // channels in this segment (0 = unused)
    int ld;           // elements between consecutive pixels of dst
    const void* add;  // optional tensor (compute type) added before activation
    int lda;
    const void* mask; // optional tensor (compute type): value kept where mask > 0
    int ldm;
    int relu;         // 1: v < 0 -> 0
    float qscale;     // FP8 stores: values are stored multiplied by qscale
};

// Geometry and tensors of one resolution class inside a launch.
struct ClassGeom {
    int nmaps;
    int Hin, Win;       // input spatial size
    int Hout, Wout;     // output spatial size
    int Hg, Wg;         // GEMM pixel grid per map (conv: output; tconv: input = phase grid)
    int tile_px;        // GEMM pixels per work item
    long item0;         // first work item of the class
    long items;         // work items of the class
    Src s0, s1;
    const long* in_off;  // raw float input: element offset of each map (null: packed)
    Seg seg0, seg1;
    const long* out_off; // float32 output: element offset of each map (null: packed)
};

constexpr int kMaxClasses = 4;

struct LayerArgs {
    int nclass;
    ClassGeom cls[kMaxClasses];
    long total_items;
    int raw_c;         // > 0: s0 is float32 with raw_c real channels (converted on load)
    float raw_qscale;  // FP8: scale applied to raw float input before the cast
    const void* wpack; // [phase][COUT_PAD][kstride] in the compute type
    int kstride;
    const float* bias; // per output channel, or null
    float acc_scale;   // multiplies the accumulator (FP8 dequantisation, gradient scale)
};

template <int MODE>
__device__ __forceinline__ int num_taps(int py, int px) {
    return MODE == M_CONV ? 9 : (py ? 2 : 1) * (px ? 2 : 1);
}

// Input offset (di, dj) of tap t relative to the pixel's base position.
template <int MODE>
__device__ __forceinline__ void tap_offset(int t, int py, int px, int& di, int& dj) {
    if (MODE == M_CONV) {
        const int kh = t / 3;
        di = kh - 1;
        dj = t - 3 * kh - 1;
    } else {
        const int tr = px ? (t >> 1) : t;
        const int tc = px ? (t & 1) : 0;
        di = (py && tr == 0) ? 1 : 0;
        dj = (px && tc == 0) ? 1 : 0;
    }
}

template <typename T>
__device__ __forceinline__ float to_float(T v);
template <> __device__ __forceinline__ float to_float<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_float<uint16_t>(uint16_t v) { return bf16_to_f32(v); }
template <> __device__ __forceinline__ float to_float<uint8_t>(uint8_t v) { return e4m3_to_f32(v); }

// Per-lane description of one GEMM pixel: map, base input row/column, and
// the element offset of its map's first raw input pixel.
struct PixRef {
    int n, bi, bj;
    long rawbase;
    bool v;
};

// Gather the lane's VW consecutive K elements of one GEMM column (pixel).
template <int P, int MODE, int CIN_EFF, bool RAW>
__device__ __forceinline__ typename Traits<P>::V load_cols(const ClassGeom& G, int raw_c, float raw_qscale,
                                                           int kk, const PixRef& r, int py, int px,
                                                           int ntaps) {
    typedef Traits<P> TR;
    typedef typename TR::T T;
    typedef typename TR::V V;
    constexpr int VW = TR::VW;
    constexpr int SUB = VW < CIN_EFF ? VW : CIN_EFF;
    constexpr int NSUB = VW / SUB;
    V v = vzero<V>();
    if (!r.v) return v;
    if constexpr (!RAW && NSUB == 1) {
        const int t = kk / CIN_EFF;
        const int c = kk % CIN_EFF;
        if (t >= ntaps) return v;
        int di, dj;
        tap_offset<MODE>(t, py, px, di, dj);
        const int i = r.bi + di, j = r.bj + dj;
        if ((unsigned)i >= (unsigned)G.Hin || (unsigned)j >= (unsigned)G.Win) return v;
        const long pix = ((long)r.n * G.Hin + i) * G.Win + j;
        const T* src = (c < G.s0.c) ? (const T*)G.s0.p + pix * G.s0.ld + c
                                    : (const T*)G.s1.p + pix * G.s1.ld + (c - G.s0.c);
        return *(const V*)src;
    } else {
        T tmp[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) tmp[e] = T(0);
#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
            const int k = kk + s * SUB;
            const int t = k / CIN_EFF;
            const int c = k % CIN_EFF;
            if (t >= ntaps) continue;
            int di, dj;
            tap_offset<MODE>(t, py, px, di, dj);
            const int i = r.bi + di, j = r.bj + dj;
            if ((unsigned)i >= (unsigned)G.Hin || (unsigned)j >= (unsigned)G.Win) continue;
            if constexpr (RAW) {
                const float* src = (const float*)G.s0.p + r.rawbase + ((long)i * G.Win + j) * G.s0.ld;
#pragma unroll
                for (int e = 0; e < SUB; ++e)
                    if (c + e < raw_c) tmp[s * SUB + e] = TR::from_f32(src[c + e], raw_qscale);
            } else {
                const long pix = ((long)r.n * G.Hin + i) * G.Win + j;
                const T* src = (c < G.s0.c) ? (const T*)G.s0.p + pix * G.s0.ld + c
                                            : (const T*)G.s1.p + pix * G.s1.ld + (c - G.s0.c);
#pragma unroll
                for (int e = 0; e < SUB; ++e) tmp[s * SUB + e] = src[e];
            }
        }
        __builtin_memcpy(&v, tmp, sizeof(V));
        return v;
    }
}

// Stores channels [lc, lc+4) of one pixel: dst at element doff + c, add and
// mask tensors at pixel opix of their own layout.
template <int P, bool OUT_F32>
__device__ __forceinline__ void store_seg(const Seg& s, long doff, long opix, int lc,
                                          const float (&val)[4]) {
    typedef typename Traits<P>::T T;
    if constexpr (!OUT_F32) {
        // fast path: a whole 4-channel group with no add/mask tensors
        if (lc + 4 <= s.c && !s.add && !s.mask) {
            T o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float v = val[e];
                if (s.relu) v = (v < 0.0f) ? 0.0f : v;
                o[e] = Traits<P>::from_f32(v, s.qscale);
            }
            T* d = (T*)s.dst + doff + lc;
            if constexpr (sizeof(T) == 4) {
                *(float4*)d = make_float4(o[0], o[1], o[2], o[3]);
            } else if constexpr (sizeof(T) == 2) {
                uint2 w;
                w.x = (uint32_t)o[0] | ((uint32_t)o[1] << 16);
                w.y = (uint32_t)o[2] | ((uint32_t)o[3] << 16);
                *(uint2*)d = w;
            } else {
                *(uint32_t*)d = (uint32_t)o[0] | ((uint32_t)o[1] << 8) | ((uint32_t)o[2] << 16) |
                                ((uint32_t)o[3] << 24);
            }
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int c = lc + e;
        if (c >= s.c) break;
        float v = val[e];
        if (s.add) v += to_float<T>(((const T*)s.add)[opix * s.lda + c]);
        if (s.relu) v = (v < 0.0f) ? 0.0f : v;
        if (s.mask && !(to_float<T>(((const T*)s.mask)[opix * s.ldm + c]) > 0.0f)) v = 0.0f;
        if constexpr (OUT_F32)
            ((float*)s.dst)[doff + c] = v;
        else
            ((T*)s.dst)[doff + c] = Traits<P>::from_f32(v, s.qscale);
    }
}

// LDS bytes a WLDS kernel needs for its weight pack (row stride padded by
// 16 bytes so that the 16 rows read by one MFMA fragment hit distinct banks).
__host__ __device__ constexpr int wlds_row_bytes(int kstride, int esize) { return kstride * esize + 16; }

template <int P, int MODE, int CIN_EFF, int COUT_PAD, int NPW, bool RAW, bool OUT_F32, bool WLDS>
__global__ __launch_bounds__(256) void conv_layer_kernel(const LayerArgs a) {
    typedef Traits<P> TR;
    typedef typename TR::T T;
    typedef typename TR::V V;
    constexpr int KS = TR::KS, VW = TR::VW;
    constexpr int MT = COUT_PAD / 16;
    constexpr int ES = (int)sizeof(T);
    static_assert(COUT_PAD % 16 == 0, "rows come in blocks of 16");
    extern __shared__ __align__(16) char smem[];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int phase = (MODE == M_TCONV) ? (int)blockIdx.y : 0;
    const int py = phase >> 1, px = phase & 1;
    const int ntaps = num_taps<MODE>(py, px);
    const int ksteps = (ntaps * CIN_EFF + KS - 1) / KS;
    const int klen = ksteps * KS;  // K elements this phase uses

    const T* wglob = (const T*)a.wpack + (size_t)phase * COUT_PAD * a.kstride;
    const int rowb = wlds_row_bytes(a.kstride, ES);
    if constexpr (WLDS) {
        // stage rows [0, COUT_PAD) x [0, klen) of this phase's pack, 16 bytes per thread step
        const int chunks_per_row = klen * ES / 16;
        for (int e = threadIdx.x; e < COUT_PAD * chunks_per_row; e += 256) {
            const int row = e / chunks_per_row, ch = e - row * chunks_per_row;
            *(uint4*)(smem + row * rowb + ch * 16) =
                *(const uint4*)((const char*)(wglob + (size_t)row * a.kstride) + ch * 16);
        }
        __syncthreads();
    }

    for (long item = blockIdx.x; item < a.total_items; item += gridDim.x) {
        int c = 0;
#pragma unroll
        for (int k = 1; k < kMaxClasses; ++k)
            if (k < a.nclass && item >= a.cls[k].item0) c = k;
        const ClassGeom& G = a.cls[c];
        const long npix = (long)G.nmaps * G.Hg * G.Wg;
        const long t0 = (item - G.item0) * G.tile_px;
        const long t1 = min(npix, t0 + G.tile_px);
        const long hw = (long)G.Hg * G.Wg;

        for (long pix0 = t0 + (long)wave * (NPW * 16); pix0 < t1; pix0 += 4L * NPW * 16) {
            PixRef pr[NPW];
#pragma unroll
            for (int p = 0; p < NPW; ++p) {
                long pix = pix0 + p * 16 + r16;
                pr[p].v = pix < t1;
                if (!pr[p].v) pix = t0;
                const int n = (int)(pix / hw);
                const int rem = (int)(pix - (long)n * hw);
                const int P_ = rem / G.Wg, Q_ = rem - P_ * G.Wg;
                pr[p].n = n;
                pr[p].bi = (MODE == M_CONV) ? 2 * P_ : P_;
                pr[p].bj = (MODE == M_CONV) ? 2 * Q_ : Q_;
                if constexpr (RAW)
                    pr[p].rawbase = G.in_off ? G.in_off[n] : (long)n * G.Hin * G.Win * G.s0.ld;
                else
                    pr[p].rawbase = 0;
            }

            f4 acc[MT][NPW];
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int p = 0; p < NPW; ++p) acc[m][p] = f4{0.f, 0.f, 0.f, 0.f};

            V bcur[NPW];
#pragma unroll
            for (int p = 0; p < NPW; ++p)
                bcur[p] = load_cols<P, MODE, CIN_EFF, RAW>(G, a.raw_c, a.raw_qscale, g * VW, pr[p], py, px,
                                                           ntaps);
            for (int ks = 0; ks < ksteps; ++ks) {
                V bnext[NPW];
                if (ks + 1 < ksteps) {
#pragma unroll
                    for (int p = 0; p < NPW; ++p)
                        bnext[p] = load_cols<P, MODE, CIN_EFF, RAW>(G, a.raw_c, a.raw_qscale,
                                                                    (ks + 1) * KS + g * VW, pr[p], py, px,
                                                                    ntaps);
                }
                V av[MT];
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    if constexpr (WLDS)
                        av[m] = *(const V*)(smem + (m * 16 + r16) * rowb + (ks * KS + g * VW) * ES);
                    else
                        av[m] = *(const V*)(wglob + (size_t)(m * 16 + r16) * a.kstride + ks * KS + g * VW);
                }
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int p = 0; p < NPW; ++p) TR::mma(acc[m][p], av[m], bcur[p]);
                if (ks + 1 < ksteps) {
#pragma unroll
                    for (int p = 0; p < NPW; ++p) bcur[p] = bnext[p];
                }
            }

            // Epilogue: lane holds rows 4g..4g+3 of each 16-row block for pixel r16.
#pragma unroll
            for (int p = 0; p < NPW; ++p) {
                if (!pr[p].v) continue;
                int oi, oj;
                if (MODE == M_CONV) {
                    oi = pr[p].bi >> 1;
                    oj = pr[p].bj >> 1;
                } else {
                    oi = 2 * pr[p].bi + py;
                    oj = 2 * pr[p].bj + px;
                }
                const long opix_local = (long)oi * G.Wout + oj;
                const long opix = (long)pr[p].n * G.Hout * G.Wout + opix_local;
                long doff0 = opix * G.seg0.ld;
                if constexpr (OUT_F32)
                    if (G.out_off) doff0 = G.out_off[pr[p].n] + opix_local * G.seg0.ld;
                const long doff1 = opix * G.seg1.ld;
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    const int ch = m * 16 + g * 4;
                    float val[4] = {acc[m][p].x * a.acc_scale, acc[m][p].y * a.acc_scale,
                                    acc[m][p].z * a.acc_scale, acc[m][p].w * a.acc_scale};
                    if (a.bias) {
                        const int nb = G.seg0.c + G.seg1.c;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (ch + e < nb) val[e] += a.bias[ch + e];
                    }
                    if (ch < G.seg0.c)
                        store_seg<P, OUT_F32>(G.seg0, doff0, opix, ch, val);
                    else if (ch - G.seg0.c < G.seg1.c)
                        store_seg<P, OUT_F32>(G.seg1, doff1, opix, ch - G.seg0.c, val);
                }
            }
        }
    }
}

}  // namespace drc
