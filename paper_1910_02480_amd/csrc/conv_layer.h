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

template <typename T>
__device__ __forceinline__ float to_float(T v);
template <> __device__ __forceinline__ float to_float<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_float<uint16_t>(uint16_t v) { return bf16_to_f32(v); }
template <> __device__ __forceinline__ float to_float<uint8_t>(uint8_t v) { return e4m3_to_f32(v); }

// Tap t's input offset (di, dj) relative to a GEMM pixel's base position;
// all arguments are compile-time constants after unrolling.
template <int MODE, int PHASE>
__host__ __device__ constexpr int tap_di(int t) {
    return MODE == M_CONV ? t / 3 - 1 : (((PHASE >> 1) && ((PHASE & 1) ? (t >> 1) : t) == 0) ? 1 : 0);
}
template <int MODE, int PHASE>
__host__ __device__ constexpr int tap_dj(int t) {
    return MODE == M_CONV ? t % 3 - 1 : (((PHASE & 1) && (t & 1) == 0) ? 1 : 0);
}
template <int MODE, int PHASE>
__host__ __device__ constexpr int ntaps_of() {
    return MODE == M_CONV ? 9 : ((PHASE >> 1) ? 2 : 1) * ((PHASE & 1) ? 2 : 1);
}

// Per-lane state of one GEMM pixel: element offsets of its base input
// position in each source, border flags, and its output position.
struct PixState {
    long off0, off1;  // element offsets of (n, bi, bj) in s0 / s1 (raw: in the float input)
    long opix;        // output pixel index (n, oi, oj) in the packed output
    long oloc;        // output pixel index inside its map (oi * Wout + oj)
    int n;
    bool v, up, down, left, right;
};

// float -> storage type with hardware RNE for bfloat16.
template <int P>
__device__ __forceinline__ typename Traits<P>::T to_store(float v, float qs) {
    if constexpr (P == P_BF16) {
        const __bf16 b = (__bf16)v;
        return __builtin_bit_cast(uint16_t, b);
    } else {
        return Traits<P>::from_f32(v, qs);
    }
}

// Loads 4 consecutive elements of type T at p (4-element aligned) as floats.
template <typename T>
__device__ __forceinline__ void load4(const T* p, float (&o)[4]) {
    if constexpr (sizeof(T) == 4) {
        const float4 v = *(const float4*)p;
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    } else if constexpr (sizeof(T) == 2) {
        const uint2 v = *(const uint2*)p;
        o[0] = bf16_to_f32((uint16_t)(v.x & 0xffffu));
        o[1] = bf16_to_f32((uint16_t)(v.x >> 16));
        o[2] = bf16_to_f32((uint16_t)(v.y & 0xffffu));
        o[3] = bf16_to_f32((uint16_t)(v.y >> 16));
    } else {
        const uint32_t v = *(const uint32_t*)p;
#pragma unroll
        for (int e = 0; e < 4; ++e) o[e] = e4m3_to_f32((uint8_t)(v >> (8 * e)));
    }
}

// Stores channels [lc, lc+4) of one pixel: dst at element doff + c, add and
// mask tensors at pixel opix of their own layout.
template <int P, bool OUT_F32>
__device__ __forceinline__ void store_seg(const Seg& s, long doff, long opix, int lc,
                                          const float (&val)[4]) {
    typedef typename Traits<P>::T T;
    float v[4] = {val[0], val[1], val[2], val[3]};
    if (lc + 4 <= s.c) {
        if (s.add) {
            float ad[4];
            load4<T>((const T*)s.add + opix * s.lda + lc, ad);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] += ad[e];
        }
        if (s.relu) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (v[e] < 0.0f) ? 0.0f : v[e];
        }
        if (s.mask) {
            float mk[4];
            load4<T>((const T*)s.mask + opix * s.ldm + lc, mk);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (mk[e] > 0.0f) ? v[e] : 0.0f;
        }
        if constexpr (OUT_F32) {
            *(float4*)((float*)s.dst + doff + lc) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
            T o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = to_store<P>(v[e], s.qscale);
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
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int c = lc + e;
        if (c >= s.c) break;
        float x = v[e];
        if (s.add) x += to_float<T>(((const T*)s.add)[opix * s.lda + c]);
        if (s.relu) x = (x < 0.0f) ? 0.0f : x;
        if (s.mask && !(to_float<T>(((const T*)s.mask)[opix * s.ldm + c]) > 0.0f)) x = 0.0f;
        if constexpr (OUT_F32)
            ((float*)s.dst)[doff + c] = x;
        else
            ((T*)s.dst)[doff + c] = to_store<P>(x, s.qscale);
    }
}

// LDS bytes a WLDS kernel needs for its weight pack (row stride padded by
// 16 bytes so that the 16 rows read by one MFMA fragment hit distinct banks).
__host__ __device__ constexpr int wlds_row_bytes(int kstride, int esize) { return kstride * esize + 16; }

// Gathers the lane's VW K elements [kk, kk+VW) of one GEMM pixel.
// C0: channels of source 0 (the rest come from source 1).
template <int P, int MODE, int PHASE, int CIN, int C0, bool RAW>
__device__ __forceinline__ typename Traits<P>::V gather(const ClassGeom& G, int raw_c, float raw_qscale,
                                                        const PixState& ps, int kk, long rowd0, long rowd1) {
    typedef Traits<P> TR;
    typedef typename TR::T T;
    typedef typename TR::V V;
    constexpr int VW = TR::VW;
    constexpr int NT = ntaps_of<MODE, PHASE>();
    constexpr int SUB = VW < CIN ? VW : CIN;
    constexpr int NSUB = VW / SUB;
    V v = vzero<V>();
    if (!ps.v) return v;
    T tmp[VW];
    if constexpr (NSUB > 1 || RAW) {
#pragma unroll
        for (int e = 0; e < VW; ++e) tmp[e] = T(0);
    }
#pragma unroll
    for (int s = 0; s < NSUB; ++s) {
        const int k = kk + s * SUB;
        const int t = k / CIN, c = k % CIN;
        if (t >= NT) continue;
        // tap offsets: constant-folded when t is a compile-time constant
        int di = 0, dj = 0;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
            if (t == tt) {
                di = tap_di<MODE, PHASE>(tt);
                dj = tap_dj<MODE, PHASE>(tt);
            }
        const bool ok = (di < 0 ? ps.up : (di > 0 ? ps.down : true)) && (dj < 0 ? ps.left : (dj > 0 ? ps.right : true));
        if (!ok) continue;
        if constexpr (RAW) {
            const float* src = (const float*)G.s0.p + ps.off0 + di * rowd0 + dj * G.s0.ld;
#pragma unroll
            for (int e = 0; e < SUB; ++e)
                if (c + e < raw_c) tmp[s * SUB + e] = TR::from_f32(src[c + e], raw_qscale);
        } else {
            const T* src = (c < C0) ? (const T*)G.s0.p + ps.off0 + di * rowd0 + dj * G.s0.ld + c
                                    : (const T*)G.s1.p + ps.off1 + di * rowd1 + dj * G.s1.ld + (c - C0);
            if constexpr (NSUB == 1) {
                return *(const V*)src;
            } else {
#pragma unroll
                for (int e = 0; e < SUB; ++e) tmp[s * SUB + e] = src[e];
            }
        }
    }
    if constexpr (NSUB > 1 || RAW) __builtin_memcpy(&v, tmp, sizeof(V));
    return v;
}

// One phase's worth of the persistent layer kernel (PHASE = 0 for conv).
template <int P, int MODE, int PHASE, int CIN, int C0, int COUT_PAD, int NPW, bool RAW, bool OUT_F32, bool WLDS>
__device__ __forceinline__ void conv_layer_phase(const LayerArgs& a, const char* smem, int rowb) {
    typedef Traits<P> TR;
    typedef typename TR::T T;
    typedef typename TR::V V;
    constexpr int KS = TR::KS, VW = TR::VW;
    constexpr int MT = COUT_PAD / 16;
    constexpr int ES = (int)sizeof(T);
    constexpr int NT = ntaps_of<MODE, PHASE>();
    constexpr int KSTEPS = (NT * CIN + KS - 1) / KS;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const T* wglob = (const T*)a.wpack + (size_t)PHASE * COUT_PAD * a.kstride;

    // biases of this lane's output channels, loaded once
    float bias[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[m][e] = 0.0f;

    for (long item = blockIdx.x; item < a.total_items; item += gridDim.x) {
        int c = 0;
#pragma unroll
        for (int k = 1; k < kMaxClasses; ++k)
            if (k < a.nclass && item >= a.cls[k].item0) c = k;
        const ClassGeom& G = a.cls[c];
        if (a.bias) {
            const int nb = G.seg0.c + G.seg1.c;
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int ch = m * 16 + g * 4 + e;
                    bias[m][e] = ch < nb ? a.bias[ch] : 0.0f;
                }
        }
        const int hw = G.Hg * G.Wg;
        const long npix = (long)G.nmaps * hw;
        const long t0 = (item - G.item0) * G.tile_px;
        const long t1 = min(npix, t0 + G.tile_px);
        const long rowd0 = (long)G.Win * G.s0.ld, rowd1 = (long)G.Win * G.s1.ld;

        for (long pix0 = t0 + (long)wave * (NPW * 16); pix0 < t1; pix0 += 4L * NPW * 16) {
            PixState ps[NPW];
#pragma unroll
            for (int p = 0; p < NPW; ++p) {
                long pix = pix0 + p * 16 + r16;
                ps[p].v = pix < t1;
                if (!ps[p].v) pix = t0;
                const int n = (int)(pix / hw);
                const int rem = (int)(pix - (long)n * hw);
                const int P_ = rem / G.Wg, Q_ = rem - P_ * G.Wg;
                const int bi = (MODE == M_CONV) ? 2 * P_ : P_;
                const int bj = (MODE == M_CONV) ? 2 * Q_ : Q_;
                ps[p].n = n;
                ps[p].up = bi > 0;
                ps[p].left = bj > 0;
                ps[p].down = bi + 1 < G.Hin;
                ps[p].right = bj + 1 < G.Win;
                const long ploc = (long)bi * G.Win + bj;
                if constexpr (RAW) {
                    const long base = G.in_off ? G.in_off[n] : (long)n * G.Hin * G.Win * G.s0.ld;
                    ps[p].off0 = base + ploc * G.s0.ld;
                    ps[p].off1 = 0;
                } else {
                    const long pl = (long)n * G.Hin * G.Win + ploc;
                    ps[p].off0 = pl * G.s0.ld;
                    ps[p].off1 = pl * G.s1.ld;
                }
                const int oi = (MODE == M_CONV) ? P_ : 2 * P_ + (PHASE >> 1);
                const int oj = (MODE == M_CONV) ? Q_ : 2 * Q_ + (PHASE & 1);
                ps[p].oloc = (long)oi * G.Wout + oj;
                ps[p].opix = (long)n * G.Hout * G.Wout + ps[p].oloc;
            }

            f4 acc[MT][NPW];
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int p = 0; p < NPW; ++p) acc[m][p] = f4{0.f, 0.f, 0.f, 0.f};

            V bv[2][NPW];
#pragma unroll
            for (int p = 0; p < NPW; ++p)
                bv[0][p] = gather<P, MODE, PHASE, CIN, C0, RAW>(G, a.raw_c, a.raw_qscale, ps[p], g * VW, rowd0, rowd1);
#pragma unroll
            for (int ks = 0; ks < KSTEPS; ++ks) {
                const int cur = ks & 1;
                if (ks + 1 < KSTEPS) {
#pragma unroll
                    for (int p = 0; p < NPW; ++p)
                        bv[cur ^ 1][p] = gather<P, MODE, PHASE, CIN, C0, RAW>(G, a.raw_c, a.raw_qscale, ps[p],
                                                                               (ks + 1) * KS + g * VW, rowd0, rowd1);
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
                    for (int p = 0; p < NPW; ++p) TR::mma(acc[m][p], av[m], bv[cur][p]);
            }

            // Epilogue: lane holds rows 4g..4g+3 of each 16-row block for pixel r16.
#pragma unroll
            for (int p = 0; p < NPW; ++p) {
                if (!ps[p].v) continue;
                long doff0 = ps[p].opix * G.seg0.ld;
                if constexpr (OUT_F32)
                    if (G.out_off) doff0 = G.out_off[ps[p].n] + ps[p].oloc * G.seg0.ld;
                const long doff1 = ps[p].opix * G.seg1.ld;
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    const int ch = m * 16 + g * 4;
                    float val[4] = {acc[m][p].x * a.acc_scale + bias[m][0], acc[m][p].y * a.acc_scale + bias[m][1],
                                    acc[m][p].z * a.acc_scale + bias[m][2], acc[m][p].w * a.acc_scale + bias[m][3]};
                    if (ch < G.seg0.c)
                        store_seg<P, OUT_F32>(G.seg0, doff0, ps[p].opix, ch, val);
                    else if (ch - G.seg0.c < G.seg1.c)
                        store_seg<P, OUT_F32>(G.seg1, doff1, ps[p].opix, ch - G.seg0.c, val);
                }
            }
        }
    }
}

// Persistent layer kernel. For transposed convolutions grid.y selects the
// output phase, each compiled with its own tap table.
template <int P, int MODE, int CIN, int C0, int COUT_PAD, int NPW, bool RAW, bool OUT_F32, bool WLDS>
__global__ __launch_bounds__(256) void conv_layer_kernel(const LayerArgs a) {
    typedef typename Traits<P>::T T;
    constexpr int ES = (int)sizeof(T);
    constexpr int KS = Traits<P>::KS;
    extern __shared__ __align__(16) char smem[];
    const int phase = (MODE == M_TCONV) ? (int)blockIdx.y : 0;
    const int ntaps = MODE == M_CONV ? 9 : ((phase >> 1) ? 2 : 1) * ((phase & 1) ? 2 : 1);
    const int klen = (ntaps * CIN + KS - 1) / KS * KS;
    const int rowb = wlds_row_bytes(a.kstride, ES);
    if constexpr (WLDS) {
        // stage rows [0, COUT_PAD) x [0, klen) of this phase's pack, 16 bytes per thread step
        const T* wglob = (const T*)a.wpack + (size_t)phase * COUT_PAD * a.kstride;
        const int chunks_per_row = klen * ES / 16;
        for (int e = threadIdx.x; e < COUT_PAD * chunks_per_row; e += 256) {
            const int row = e / chunks_per_row, ch = e - row * chunks_per_row;
            *(uint4*)(smem + row * rowb + ch * 16) =
                *(const uint4*)((const char*)(wglob + (size_t)row * a.kstride) + ch * 16);
        }
        __syncthreads();
    }
    if constexpr (MODE == M_CONV) {
        conv_layer_phase<P, MODE, 0, CIN, C0, COUT_PAD, NPW, RAW, OUT_F32, WLDS>(a, smem, rowb);
    } else {
        switch (phase) {
            case 0: conv_layer_phase<P, MODE, 0, CIN, C0, COUT_PAD, NPW, RAW, OUT_F32, WLDS>(a, smem, rowb); break;
            case 1: conv_layer_phase<P, MODE, 1, CIN, C0, COUT_PAD, NPW, RAW, OUT_F32, WLDS>(a, smem, rowb); break;
            case 2: conv_layer_phase<P, MODE, 2, CIN, C0, COUT_PAD, NPW, RAW, OUT_F32, WLDS>(a, smem, rowb); break;
            default: conv_layer_phase<P, MODE, 3, CIN, C0, COUT_PAD, NPW, RAW, OUT_F32, WLDS>(a, smem, rowb); break;
        }
    }
}

}  // namespace drc
