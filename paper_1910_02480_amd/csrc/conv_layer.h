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

enum Mode : int {
    M_CONV = 0,          // stride-2 convolution, taps in 3x3 order
    M_TCONV = 1,         // transposed convolution (one output phase per GEMM; packs only)
    M_TCONV_PAIRS = 2,   // transposed convolution, all phases: 9 (phase, neighbour) weight blocks
    M_TCONV_MERGED = 3   // transposed convolution, all phases: rows = (phase, channel), K = (neighbour, channel)
};

// The 9 (output phase, input neighbour) pairs of a stride-2 transposed 3x3
// convolution. Phase p = 2 py + px is output (2a+py, 2b+px); neighbour
// nb = 2 di + dj is input (a+di, b+dj). Row tap kh = 1 for py = 0, and for
// py = 1 kh = 0 with di = 1 or kh = 2 with di = 0; columns likewise.
__host__ __device__ constexpr int pair_phase(int q) { return q == 0 ? 0 : (q <= 2 ? 1 : (q <= 4 ? 2 : 3)); }
__host__ __device__ constexpr int pair_nb(int q) {
    return q == 0 ? 0 : (q == 1 ? 0 : (q == 2 ? 1 : (q == 3 ? 0 : (q == 4 ? 2 : q - 5))));
}
__host__ __device__ constexpr bool phase_uses(int ph, int nb) {
    return ((ph >> 1) || !(nb >> 1)) && ((ph & 1) || !(nb & 1));
}
__host__ __device__ constexpr int tap_kh(int ph, int nb) { return (ph >> 1) ? ((nb >> 1) ? 0 : 2) : 1; }
__host__ __device__ constexpr int tap_kw(int ph, int nb) { return (ph & 1) ? ((nb & 1) ? 0 : 2) : 1; }

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
    int circ;            // 1: the width is periodic (circular padding), 0: zero padding
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
    int jl, jr;       // column steps to the left / right neighbour (+-1, or across the seam when circular)
    bool v, up, down, left, right;
};

// Column step of tap offset dj in {-1, 0, 1}.
__device__ __forceinline__ int col_step(const PixState& ps, int dj) { return dj < 0 ? ps.jl : (dj > 0 ? ps.jr : 0); }

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
        if constexpr (P == P_FP8 && !OUT_F32) {
            // the ReLU is folded into the store's clamp
            if (s.mask) {
                float mk[4];
                load4<T>((const T*)s.mask + opix * s.ldm + lc, mk);
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = (mk[e] > 0.0f) ? v[e] : 0.0f;
            }
            *(uint32_t*)((T*)s.dst + doff + lc) = e4m3_act4(v[0], v[1], v[2], v[3], s.qscale, s.relu);
            return;
        }
        if (s.relu) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = relu(v[e]);
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
            T* d = (T*)s.dst + doff + lc;
            if constexpr (sizeof(T) == 2) {
                *(uint2*)d = make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
                return;
            }
            T o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = to_store<P>(v[e], s.qscale);
            if constexpr (sizeof(T) == 4) {
                *(float4*)d = make_float4(o[0], o[1], o[2], o[3]);
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
        if constexpr (P == P_FP8 && !OUT_F32) {
            if (s.mask && !(to_float<T>(((const T*)s.mask)[opix * s.ldm + c]) > 0.0f)) x = 0.0f;
            ((T*)s.dst)[doff + c] = e4m3_act(x, s.qscale, s.relu);
            continue;
        }
        if (s.relu) x = relu(x);
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

// Input neighbour nb (= 2 di + dj) of a transposed-convolution GEMM pixel
// (a, b): the lane's VW channels [c, c+VW) of input pixel (a+di, b+dj).
template <int P, int C0>
__device__ __forceinline__ typename Traits<P>::V gather_nb(const ClassGeom& G, const PixState& ps, int nb, int c,
                                                           long rowd0, long rowd1) {
    typedef typename Traits<P>::T T;
    typedef typename Traits<P>::V V;
    const int di = nb >> 1, dj = nb & 1;
    if (!ps.v || (di && !ps.down) || (dj && !ps.right)) return vzero<V>();
    const int cj = dj ? ps.jr : 0;
    const T* src = (c < C0) ? (const T*)G.s0.p + ps.off0 + di * rowd0 + cj * G.s0.ld + c
                            : (const T*)G.s1.p + ps.off1 + di * rowd1 + cj * G.s1.ld + (c - C0);
    return *(const V*)src;
}

// Per-pixel setup shared by the kernels: map, base input position, border
// flags, input offsets and the output pixel of the GEMM pixel.
template <int MODE, bool RAW>
__device__ __forceinline__ void pix_setup(const ClassGeom& G, long pix, long t0, long t1, PixState& ps) {
    ps.v = pix < t1;
    if (!ps.v) pix = t0;
    const int hw = G.Hg * G.Wg;
    const int n = (int)(pix / hw);
    const int rem = (int)(pix - (long)n * hw);
    const int P_ = rem / G.Wg, Q_ = rem - P_ * G.Wg;
    const int bi = (MODE == M_CONV) ? 2 * P_ : P_;
    const int bj = (MODE == M_CONV) ? 2 * Q_ : Q_;
    ps.n = n;
    ps.up = bi > 0;
    ps.left = bj > 0 || G.circ;
    ps.down = bi + 1 < G.Hin;
    ps.right = bj + 1 < G.Win || G.circ;
    ps.jl = bj > 0 ? -1 : G.Win - 1;
    ps.jr = bj + 1 < G.Win ? 1 : 1 - G.Win;
    const long ploc = (long)bi * G.Win + bj;
    if constexpr (RAW) {
        const long base = G.in_off ? G.in_off[n] : (long)n * G.Hin * G.Win * G.s0.ld;
        ps.off0 = base + ploc * G.s0.ld;
        ps.off1 = 0;
    } else {
        const long pl = (long)n * G.Hin * G.Win + ploc;
        ps.off0 = pl * G.s0.ld;
        ps.off1 = pl * G.s1.ld;
    }
    // conv: output (P_, Q_); transposed conv: phase-0 output (2a, 2b)
    const int oi = (MODE == M_CONV) ? P_ : 2 * P_;
    const int oj = (MODE == M_CONV) ? Q_ : 2 * Q_;
    ps.oloc = (long)oi * G.Wout + oj;
    ps.opix = (long)n * G.Hout * G.Wout + ps.oloc;
}

// Finds the resolution class of a work item and its pixel range.
__device__ __forceinline__ const ClassGeom& item_class(const LayerArgs& a, long item, long& t0, long& t1) {
    int c = 0;
#pragma unroll
    for (int k = 1; k < kMaxClasses; ++k)
        if (k < a.nclass && item >= a.cls[k].item0) c = k;
    const ClassGeom& G = a.cls[c];
    const long npix = (long)G.nmaps * G.Hg * G.Wg;
    t0 = (item - G.item0) * G.tile_px;
    t1 = min(npix, t0 + G.tile_px);
    return G;
}

// Stages rows x klen of a weight pack into LDS (16 bytes per thread step).
template <int ES>
__device__ __forceinline__ void stage_weights(char* smem, const void* w, int rows, int kstride, int klen, int rowb) {
    const int chunks_per_row = klen * ES / 16;
    for (int e = threadIdx.x; e < rows * chunks_per_row; e += 256) {
        const int row = e / chunks_per_row, ch = e - row * chunks_per_row;
        *(uint4*)(smem + row * rowb + ch * 16) =
            *(const uint4*)((const char*)w + (size_t)row * kstride * ES + ch * 16);
    }
    __syncthreads();
}

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
    if constexpr (RAW && NSUB == 1) {
        // float32 source: no per-lane branch around the loads (a branch makes
        // the compiler wait for every load in flight). A tap outside the map,
        // a K position past the last tap, or a pixel past the end reads the
        // pixel's own (valid) position and is then zeroed.
        const int t = kk / CIN, c = kk % CIN;
        int di = 0, dj = 0;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
            if (t == tt) {
                di = tap_di<MODE, PHASE>(tt);
                dj = tap_dj<MODE, PHASE>(tt);
            }
        const bool ok = ps.v && t < NT && (di < 0 ? ps.up : (di > 0 ? ps.down : true)) &&
                        (dj < 0 ? ps.left : (dj > 0 ? ps.right : true));
        const float* src = (const float*)G.s0.p + ps.off0 + (ok ? di * rowd0 + col_step(ps, dj) * G.s0.ld : 0);
        float f[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) f[e] = src[min(c + e, raw_c - 1)];  // stays inside the pixel
        T tmp[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) tmp[e] = ok && c + e < raw_c ? to_store<P>(f[e], raw_qscale) : T(0);
        __builtin_memcpy(&v, tmp, sizeof(V));
        return v;
    }
    if constexpr (!RAW && NSUB == 1) {
        // one 16-byte (or 32-byte) load per lane, likewise without a branch:
        // a tap outside the map or past the last tap, or a pixel past the end,
        // reads the pixel's own position and the value is then zeroed
        const int t = kk / CIN, c = kk % CIN;
        int di = 0, dj = 0;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
            if (t == tt) {
                di = tap_di<MODE, PHASE>(tt);
                dj = tap_dj<MODE, PHASE>(tt);
            }
        const bool ok = ps.v && t < NT && (di < 0 ? ps.up : (di > 0 ? ps.down : true)) &&
                        (dj < 0 ? ps.left : (dj > 0 ? ps.right : true));
        const T* src;
        if constexpr (C0 >= CIN) {
            src = (const T*)G.s0.p + ps.off0 + (ok ? di * rowd0 + col_step(ps, dj) * G.s0.ld : 0) + c;
        } else {
            src = (c < C0) ? (const T*)G.s0.p + ps.off0 + (ok ? di * rowd0 + col_step(ps, dj) * G.s0.ld : 0) + c
                           : (const T*)G.s1.p + ps.off1 + (ok ? di * rowd1 + col_step(ps, dj) * G.s1.ld : 0) + (c - C0);
        }
        const V val = *(const V*)src;
        return ok ? val : v;
    }
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
            const float* src = (const float*)G.s0.p + ps.off0 + di * rowd0 + col_step(ps, dj) * G.s0.ld;
#pragma unroll
            for (int e = 0; e < SUB; ++e)
                if (c + e < raw_c) tmp[s * SUB + e] = to_store<P>(src[c + e], raw_qscale);
        } else {
            const T* src = (c < C0) ? (const T*)G.s0.p + ps.off0 + di * rowd0 + col_step(ps, dj) * G.s0.ld + c
                                    : (const T*)G.s1.p + ps.off1 + di * rowd1 + col_step(ps, dj) * G.s1.ld + (c - C0);
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
template <int P, int MODE, int PHASE, int CIN, int C0, int COUT_PAD, int NPW, bool RAW, bool OUT_F32, bool WLDS,
          int WM>
__device__ __forceinline__ void conv_layer_phase(const LayerArgs& a, const char* smem, int rowb) {
    typedef Traits<P> TR;
    typedef typename TR::T T;
    typedef typename TR::V V;
    constexpr int KS = TR::KS, VW = TR::VW;
    // WM waves share a pixel tile, each owning every WM-th block of 16 rows
    constexpr int MT = COUT_PAD / 16 / WM;
    constexpr int WP = 4 / WM;
    static_assert(COUT_PAD / 16 % WM == 0, "row blocks split evenly over waves");
    constexpr int ES = (int)sizeof(T);
    constexpr int NT = ntaps_of<MODE, PHASE>();
    constexpr int KSTEPS = (NT * CIN + KS - 1) / KS;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int wm = wave % WM, wp = wave / WM;
    const T* wglob = (const T*)a.wpack + (size_t)PHASE * COUT_PAD * a.kstride;

    // biases of this lane's output channels, loaded once
    float bias[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[m][e] = 0.0f;

    for (long item = blockIdx.x; item < a.total_items; item += gridDim.x) {
        long t0, t1;
        const ClassGeom& G = item_class(a, item, t0, t1);
        if (a.bias) {
            const int nb = G.seg0.c + G.seg1.c;
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int ch = (wm + WM * m) * 16 + g * 4 + e;
                    bias[m][e] = ch < nb ? a.bias[ch] : 0.0f;
                }
        }
        const long rowd0 = (long)G.Win * G.s0.ld, rowd1 = (long)G.Win * G.s1.ld;

        for (long pix0 = t0 + (long)wp * (NPW * 16); pix0 < t1; pix0 += (long)WP * NPW * 16) {
            PixState ps[NPW];
#pragma unroll
            for (int p = 0; p < NPW; ++p) pix_setup<MODE, RAW>(G, pix0 + p * 16 + r16, t0, t1, ps[p]);

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
                    const int row = (wm + WM * m) * 16 + r16;
                    if constexpr (WLDS)
                        av[m] = *(const V*)(smem + row * rowb + (ks * KS + g * VW) * ES);
                    else
                        av[m] = *(const V*)(wglob + (size_t)row * a.kstride + ks * KS + g * VW);
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
                    const int ch = (wm + WM * m) * 16 + g * 4;
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

// Persistent stride-2 convolution kernel.
template <int P, int MODE, int CIN, int C0, int COUT_PAD, int NPW, bool RAW, bool OUT_F32, bool WLDS, int WM>
__global__ __launch_bounds__(256) void conv_layer_kernel(const LayerArgs a) {
    static_assert(MODE == M_CONV, "transposed convolutions use tconv_pairs_kernel / tconv_merged_kernel");
    typedef typename Traits<P>::T T;
    constexpr int ES = (int)sizeof(T);
    constexpr int KS = Traits<P>::KS;
    extern __shared__ __align__(16) char smem[];
    const int rowb = wlds_row_bytes(a.kstride, ES);
    if constexpr (WLDS) stage_weights<ES>(smem, a.wpack, COUT_PAD, a.kstride, (9 * CIN + KS - 1) / KS * KS, rowb);
    conv_layer_phase<P, MODE, 0, CIN, C0, COUT_PAD, NPW, RAW, OUT_F32, WLDS, WM>(a, smem, rowb);
}

// Persistent stride-2 transposed convolution over all four output phases.
// Each GEMM pixel (a, b) gathers its 4 input neighbours once per K step and
// feeds them to the 9 (phase, neighbour) weight blocks; weight pack
// [pair q][COUT_PAD][kstride].
template <int P, int CIN, int C0, int COUT_PAD, int NPW, bool OUT_F32, bool WLDS, int WM>
__global__ __launch_bounds__(256) void tconv_pairs_kernel(const LayerArgs a) {
    typedef Traits<P> TR;
    typedef typename TR::T T;
    typedef typename TR::V V;
    constexpr int KS = TR::KS, VW = TR::VW;
    constexpr int ES = (int)sizeof(T);
    // WM waves share a pixel tile, each owning every WM-th block of 16 rows
    constexpr int MT = COUT_PAD / 16 / WM;
    constexpr int WP = 4 / WM;
    static_assert(COUT_PAD / 16 % WM == 0, "row blocks split evenly over waves");
    static_assert(CIN % KS == 0, "one neighbour per K step");
    constexpr int KSN = CIN / KS;
    extern __shared__ __align__(16) char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int wm = wave % WM, wp = wave / WM;
    const int rowb = wlds_row_bytes(a.kstride, ES);
    if constexpr (WLDS) stage_weights<ES>(smem, a.wpack, 9 * COUT_PAD, a.kstride, CIN, rowb);
    const T* wglob = (const T*)a.wpack;

    float bias[MT][4];
    for (long item = blockIdx.x; item < a.total_items; item += gridDim.x) {
        long t0, t1;
        const ClassGeom& G = item_class(a, item, t0, t1);
        const int nb_out = G.seg0.c + G.seg1.c;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ch = (wm + WM * m) * 16 + g * 4 + e;
                bias[m][e] = (a.bias && ch < nb_out) ? a.bias[ch] : 0.0f;
            }
        const long rowd0 = (long)G.Win * G.s0.ld, rowd1 = (long)G.Win * G.s1.ld;
        for (long pix0 = t0 + (long)wp * (NPW * 16); pix0 < t1; pix0 += (long)WP * NPW * 16) {
            PixState ps[NPW];
#pragma unroll
            for (int p = 0; p < NPW; ++p) pix_setup<M_TCONV, false>(G, pix0 + p * 16 + r16, t0, t1, ps[p]);
            f4 acc[4][MT][NPW];
#pragma unroll
            for (int ph = 0; ph < 4; ++ph)
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int p = 0; p < NPW; ++p) acc[ph][m][p] = f4{0.f, 0.f, 0.f, 0.f};
            V bv[2][4][NPW];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                for (int p = 0; p < NPW; ++p) bv[0][nb][p] = gather_nb<P, C0>(G, ps[p], nb, g * VW, rowd0, rowd1);
#pragma unroll
            for (int ks = 0; ks < KSN; ++ks) {
                const int cur = ks & 1;
                if (ks + 1 < KSN) {
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                        for (int p = 0; p < NPW; ++p)
                            bv[cur ^ 1][nb][p] = gather_nb<P, C0>(G, ps[p], nb, (ks + 1) * KS + g * VW, rowd0, rowd1);
                }
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    const int ph = pair_phase(q), nb = pair_nb(q);
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        const int row = q * COUT_PAD + (wm + WM * m) * 16 + r16;
                        V av;
                        if constexpr (WLDS)
                            av = *(const V*)(smem + row * rowb + (ks * KS + g * VW) * ES);
                        else
                            av = *(const V*)(wglob + (size_t)row * a.kstride + ks * KS + g * VW);
#pragma unroll
                        for (int p = 0; p < NPW; ++p) TR::mma(acc[ph][m][p], av, bv[cur][nb][p]);
                    }
                }
            }
#pragma unroll
            for (int ph = 0; ph < 4; ++ph)
#pragma unroll
                for (int p = 0; p < NPW; ++p) {
                    if (!ps[p].v) continue;
                    const long dpix = (long)(ph >> 1) * G.Wout + (ph & 1);
                    const long opix = ps[p].opix + dpix;
                    long doff0 = opix * G.seg0.ld;
                    if constexpr (OUT_F32)
                        if (G.out_off) doff0 = G.out_off[ps[p].n] + (ps[p].oloc + dpix) * G.seg0.ld;
                    const long doff1 = opix * G.seg1.ld;
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
                        const int ch = (wm + WM * m) * 16 + g * 4;
                        float val[4] = {acc[ph][m][p].x * a.acc_scale + bias[m][0], acc[ph][m][p].y * a.acc_scale + bias[m][1],
                                        acc[ph][m][p].z * a.acc_scale + bias[m][2], acc[ph][m][p].w * a.acc_scale + bias[m][3]};
                        if (ch < G.seg0.c)
                            store_seg<P, OUT_F32>(G.seg0, doff0, opix, ch, val);
                        else if (ch - G.seg0.c < G.seg1.c)
                            store_seg<P, OUT_F32>(G.seg1, doff1, opix, ch - G.seg0.c, val);
                    }
                }
        }
    }
}

// Transposed convolution with few output channels (Cout < 16): the four
// phases share one block of rows r = phase * COUT + co, and K runs over
// (neighbour, channel): pack [R][kstride], zero where a phase does not use a
// neighbour. One gather per neighbour feeds all phases.
template <int P, int CIN, int C0, int COUT, int R, int NPW, bool OUT_F32, bool WLDS>
__global__ __launch_bounds__(256) void tconv_merged_kernel(const LayerArgs a) {
    typedef Traits<P> TR;
    typedef typename TR::T T;
    typedef typename TR::V V;
    constexpr int KS = TR::KS, VW = TR::VW;
    constexpr int ES = (int)sizeof(T);
    constexpr int MT = R / 16;
    constexpr int KSTEPS = (4 * CIN + KS - 1) / KS;
    static_assert(CIN % VW == 0, "a lane's K elements stay inside one neighbour");
    extern __shared__ __align__(16) char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int rowb = wlds_row_bytes(a.kstride, ES);
    if constexpr (WLDS) stage_weights<ES>(smem, a.wpack, R, a.kstride, KSTEPS * KS, rowb);
    const T* wglob = (const T*)a.wpack;

    float bias[MT][4];
    int rph[MT][4], rco[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = m * 16 + g * 4 + e;
            rph[m][e] = r / COUT;
            rco[m][e] = r - (r / COUT) * COUT;
            bias[m][e] = (a.bias && r < 4 * COUT) ? a.bias[rco[m][e]] : 0.0f;
        }
    for (long item = blockIdx.x; item < a.total_items; item += gridDim.x) {
        long t0, t1;
        const ClassGeom& G = item_class(a, item, t0, t1);
        const long rowd0 = (long)G.Win * G.s0.ld, rowd1 = (long)G.Win * G.s1.ld;
        for (long pix0 = t0 + (long)wave * (NPW * 16); pix0 < t1; pix0 += 4L * NPW * 16) {
            PixState ps[NPW];
#pragma unroll
            for (int p = 0; p < NPW; ++p) pix_setup<M_TCONV, false>(G, pix0 + p * 16 + r16, t0, t1, ps[p]);
            f4 acc[MT][NPW];
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int p = 0; p < NPW; ++p) acc[m][p] = f4{0.f, 0.f, 0.f, 0.f};
            V bv[2][NPW];
#pragma unroll
            for (int p = 0; p < NPW; ++p) {
                const int k = g * VW;
                bv[0][p] = k < 4 * CIN ? gather_nb<P, C0>(G, ps[p], k / CIN, k % CIN, rowd0, rowd1) : vzero<V>();
            }
#pragma unroll
            for (int ks = 0; ks < KSTEPS; ++ks) {
                const int cur = ks & 1;
                if (ks + 1 < KSTEPS) {
                    const int k = (ks + 1) * KS + g * VW;
#pragma unroll
                    for (int p = 0; p < NPW; ++p)
                        bv[cur ^ 1][p] = k < 4 * CIN ? gather_nb<P, C0>(G, ps[p], k / CIN, k % CIN, rowd0, rowd1)
                                                     : vzero<V>();
                }
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    V av;
                    if constexpr (WLDS)
                        av = *(const V*)(smem + (m * 16 + r16) * rowb + (ks * KS + g * VW) * ES);
                    else
                        av = *(const V*)(wglob + (size_t)(m * 16 + r16) * a.kstride + ks * KS + g * VW);
#pragma unroll
                    for (int p = 0; p < NPW; ++p) TR::mma(acc[m][p], av, bv[cur][p]);
                }
            }
#pragma unroll
            for (int p = 0; p < NPW; ++p) {
                if (!ps[p].v) continue;
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (m * 16 + g * 4 + e >= 4 * COUT) continue;
                        const int ph = rph[m][e], co = rco[m][e];
                        const long dpix = (long)(ph >> 1) * G.Wout + (ph & 1);
                        const long opix = ps[p].opix + dpix;
                        long doff = opix * G.seg0.ld;
                        if constexpr (OUT_F32)
                            if (G.out_off) doff = G.out_off[ps[p].n] + (ps[p].oloc + dpix) * G.seg0.ld;
                        float v = acc[m][p][e] * a.acc_scale + bias[m][e];
                        if constexpr (P == P_FP8 && !OUT_F32) {
                            ((T*)G.seg0.dst)[doff + co] = e4m3_act(v, G.seg0.qscale, G.seg0.relu);
                            continue;
                        }
                        if (G.seg0.relu) v = relu(v);
                        if constexpr (OUT_F32)
                            ((float*)G.seg0.dst)[doff + co] = v;
                        else
                            ((T*)G.seg0.dst)[doff + co] = to_store<P>(v, G.seg0.qscale);
                    }
            }
        }
    }
}

}  // namespace drc
