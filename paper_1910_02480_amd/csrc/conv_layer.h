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
// Layout: NHWC activations; the GEMM row (output channel) dimension sits on
// the MFMA A side, so each lane ends with four consecutive channels of one
// pixel and stores them as one vector. A workgroup is 4 waves; each wave
// owns all COUT_PAD rows and NPW blocks of 16 consecutive GEMM pixels.
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

struct LayerArgs {
    Src s0, s1;
    int raw_c;         // > 0: s0 is float32 with raw_c real channels (converted on load)
    float raw_qscale;  // FP8: scale applied to raw float input before the cast
    int nmaps;
    int Hin, Win;      // input spatial size
    int Hout, Wout;    // output spatial size
    int Hg, Wg;        // GEMM pixel grid per map (conv: output; tconv: input = phase grid)
    const void* wpack; // [phase][COUT_PAD][kstride] in the compute type
    int kstride;
    const float* bias; // per output channel, or null
    float acc_scale;   // multiplies the accumulator (FP8 dequantisation, gradient scale)
    Seg seg0, seg1;
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

// Gather the lane's VW consecutive K elements of one GEMM column (pixel).
template <int P, int MODE, int CIN_EFF, bool RAW>
__device__ __forceinline__ typename Traits<P>::V load_cols(const LayerArgs& a, int kk, int n, int bi,
                                                           int bj, bool pv, int py, int px, int ntaps) {
    typedef Traits<P> TR;
    typedef typename TR::T T;
    typedef typename TR::V V;
    constexpr int VW = TR::VW;
    constexpr int SUB = VW < CIN_EFF ? VW : CIN_EFF;
    constexpr int NSUB = VW / SUB;
    V v = vzero<V>();
    if (!pv) return v;
    if constexpr (!RAW && NSUB == 1) {
        const int t = kk / CIN_EFF;
        const int c = kk % CIN_EFF;
        if (t >= ntaps) return v;
        int di, dj;
        tap_offset<MODE>(t, py, px, di, dj);
        const int i = bi + di, j = bj + dj;
        if ((unsigned)i >= (unsigned)a.Hin || (unsigned)j >= (unsigned)a.Win) return v;
        const long pix = ((long)n * a.Hin + i) * a.Win + j;
        const T* src = (c < a.s0.c) ? (const T*)a.s0.p + pix * a.s0.ld + c
                                    : (const T*)a.s1.p + pix * a.s1.ld + (c - a.s0.c);
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
            const int i = bi + di, j = bj + dj;
            if ((unsigned)i >= (unsigned)a.Hin || (unsigned)j >= (unsigned)a.Win) continue;
            const long pix = ((long)n * a.Hin + i) * a.Win + j;
            if constexpr (RAW) {
                const float* src = (const float*)a.s0.p + pix * a.s0.ld;
#pragma unroll
                for (int e = 0; e < SUB; ++e)
                    if (c + e < a.raw_c) tmp[s * SUB + e] = TR::from_f32(src[c + e], a.raw_qscale);
            } else {
                const T* src = (c < a.s0.c) ? (const T*)a.s0.p + pix * a.s0.ld + c
                                            : (const T*)a.s1.p + pix * a.s1.ld + (c - a.s0.c);
#pragma unroll
                for (int e = 0; e < SUB; ++e) tmp[s * SUB + e] = src[e];
            }
        }
        __builtin_memcpy(&v, tmp, sizeof(V));
        return v;
    }
}

template <int P, bool OUT_F32>
__device__ __forceinline__ void store_seg(const Seg& s, long opix, int lc, const float (&val)[4]) {
    typedef typename Traits<P>::T T;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int c = lc + e;
        if (c >= s.c) break;
        float v = val[e];
        if (s.add) v += to_float<T>(((const T*)s.add)[opix * s.lda + c]);
        if (s.relu) v = (v < 0.0f) ? 0.0f : v;
        if (s.mask && !(to_float<T>(((const T*)s.mask)[opix * s.ldm + c]) > 0.0f)) v = 0.0f;
        if constexpr (OUT_F32)
            ((float*)s.dst)[opix * s.ld + c] = v;
        else
            ((T*)s.dst)[opix * s.ld + c] = Traits<P>::from_f32(v, s.qscale);
    }
}

// Consecutive workgroups land on different XCDs (round robin over 8). Remap
// so that each XCD works on a contiguous range of pixel tiles (shared input
// halos stay in that XCD's L2).
__device__ __forceinline__ int xcd_swizzle(int bid, int nblk) {
    const int per = nblk / 8;
    if (per == 0 || bid >= per * 8) return bid;
    return (bid & 7) * per + (bid >> 3);
}

template <int P, int MODE, int CIN_EFF, int COUT_PAD, int NPW, bool RAW, bool OUT_F32>
__global__ __launch_bounds__(256) void conv_layer_kernel(LayerArgs a) {
    typedef Traits<P> TR;
    typedef typename TR::T T;
    typedef typename TR::V V;
    constexpr int KS = TR::KS, VW = TR::VW;
    constexpr int MT = COUT_PAD / 16;
    static_assert(COUT_PAD % 16 == 0, "rows come in blocks of 16");

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int phase = (MODE == M_TCONV) ? (int)blockIdx.y : 0;
    const int py = phase >> 1, px = phase & 1;
    const int ntaps = num_taps<MODE>(py, px);
    const int ksteps = (ntaps * CIN_EFF + KS - 1) / KS;

    const long npix = (long)a.nmaps * a.Hg * a.Wg;
    const int blk = xcd_swizzle((int)blockIdx.x, (int)gridDim.x);
    const long pix0 = ((long)blk * 4 + wave) * (NPW * 16);
    if (pix0 >= npix) return;

    int pn[NPW], pbi[NPW], pbj[NPW];
    bool pv[NPW];
#pragma unroll
    for (int p = 0; p < NPW; ++p) {
        long pix = pix0 + p * 16 + r16;
        pv[p] = pix < npix;
        if (!pv[p]) pix = 0;
        const long hw = (long)a.Hg * a.Wg;
        const int n = (int)(pix / hw);
        const int rem = (int)(pix - (long)n * hw);
        const int P_ = rem / a.Wg, Q_ = rem - (rem / a.Wg) * a.Wg;
        pn[p] = n;
        pbi[p] = (MODE == M_CONV) ? 2 * P_ : P_;
        pbj[p] = (MODE == M_CONV) ? 2 * Q_ : Q_;
    }

    f4 acc[MT][NPW];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int p = 0; p < NPW; ++p) acc[m][p] = f4{0.f, 0.f, 0.f, 0.f};

    const T* wbase = (const T*)a.wpack + (size_t)phase * COUT_PAD * a.kstride + g * VW;
    for (int ks = 0; ks < ksteps; ++ks) {
        const int kk = ks * KS + g * VW;
        V av[MT], bv[NPW];
#pragma unroll
        for (int m = 0; m < MT; ++m)
            av[m] = *(const V*)(wbase + (size_t)(m * 16 + r16) * a.kstride + ks * KS);
#pragma unroll
        for (int p = 0; p < NPW; ++p)
            bv[p] = load_cols<P, MODE, CIN_EFF, RAW>(a, kk, pn[p], pbi[p], pbj[p], pv[p], py, px, ntaps);
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int p = 0; p < NPW; ++p) TR::mma(acc[m][p], av[m], bv[p]);
    }

    // Epilogue: lane holds rows 4g..4g+3 of each 16-row block for pixel r16.
#pragma unroll
    for (int p = 0; p < NPW; ++p) {
        if (!pv[p]) continue;
        int oi, oj;
        if (MODE == M_CONV) {
            oi = pbi[p] >> 1;
            oj = pbj[p] >> 1;
        } else {
            oi = 2 * pbi[p] + py;
            oj = 2 * pbj[p] + px;
        }
        const long opix = ((long)pn[p] * a.Hout + oi) * a.Wout + oj;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int c = m * 16 + g * 4;
            float val[4] = {acc[m][p].x * a.acc_scale, acc[m][p].y * a.acc_scale,
                            acc[m][p].z * a.acc_scale, acc[m][p].w * a.acc_scale};
            if (a.bias) {
                const int nb = a.seg0.c + a.seg1.c;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (c + e < nb) val[e] += a.bias[c + e];
            }
            if (c < a.seg0.c)
                store_seg<P, OUT_F32>(a.seg0, opix, c, val);
            else if (c - a.seg0.c < a.seg1.c)
                store_seg<P, OUT_F32>(a.seg1, opix, c - a.seg0.c, val);
        }
    }
}

}  // namespace drc
