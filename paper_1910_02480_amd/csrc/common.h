// Device-side building blocks shared by every kernel of the library:
// storage types per precision, round-to-nearest-even casts, and one MFMA
// "K step" per precision for gfx950 (CDNA4, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace drc {

enum Prec : int { P_F32 = 0, P_BF16 = 1, P_FP8 = 2 };

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i8v __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- casts
// float -> bfloat16, round to nearest even (the hardware conversion,
// v_cvt_pk_bf16_f32; a NaN stays a NaN).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
// Two floats -> two bfloat16 (RNE) in one word, a first: one v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef __bf16 b2v __attribute__((ext_vector_type(2)));
    const f2v f = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, b2v));
}
// ReLU as the IEEE 754-2019 maximum(v, +0) (one v_maximum3_f32): a NaN
// stays NaN, -0 becomes +0. Every ReLU of the library uses it.
__device__ __forceinline__ float relu(float v) { return __builtin_elementwise_maximum(v, 0.0f); }
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}

// float -> OCP FP8 E4M3 ("e4m3fn": bias 7, no infinities, 0x7f = NaN),
// round to nearest even, saturating at +-448 (infinities saturate too).
// The value is clamped to +-448 (med3) and converted by the hardware's
// round-to-nearest-even e4m3 conversion (v_cvt_pk_fp8_f32); on gfx950 that
// gives the same byte as the definition above for every finite input
// (checked over all floats of magnitude 2^-27 .. 2^14 with 2^19 mantissa
// steps per binade, covering every rounding boundary and tie, and the
// subnormal grid); NaN is mapped to 0x7f with its sign by the select.
__device__ __forceinline__ uint8_t f32_to_e4m3(float f) {
    const uint8_t nan = (uint8_t)(((__float_as_uint(f) >> 24) & 0x80u) | 0x7fu);
    const float c = __builtin_amdgcn_fmed3f(f, -448.0f, 448.0f);
    const uint8_t v = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(c, c, 0, false) & 0xff);
    return f != f ? nan : v;
}

// The FP8 store of an activation: e4m3(v * q) (q > 0, the output tensor's
// scale), after a ReLU when `relu`. The ReLU is the lower bound of the clamp
// (med3(v q, 0, 448)); without it the clamp is [-448, 448]. A NaN keeps its
// encoding (0x7f with its sign). Every FP8 activation store of the library
// goes through these two, so both give the same byte for the same value.
__device__ __forceinline__ uint8_t e4m3_act(float v, float q, bool relu) {
    const float u = v * q;
    const float c = __builtin_amdgcn_fmed3f(u, relu ? 0.0f : -448.0f, 448.0f);
    const uint8_t b = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(c, c, 0, false) & 0xff);
    return u != u ? (uint8_t)(((__float_as_uint(u) >> 24) & 0x80u) | 0x7fu) : b;
}
// Four values, bytes in order in one word: two conversions of two values
// each; a NaN among them (its sum is NaN) takes the per-value encoder.
__device__ __forceinline__ uint32_t e4m3_act4(float v0, float v1, float v2, float v3, float q, bool relu) {
    const float u0 = v0 * q, u1 = v1 * q, u2 = v2 * q, u3 = v3 * q;
    const float s = (u0 + u1) + (u2 + u3);
    if (__builtin_expect(s != s, 0))
        return (uint32_t)e4m3_act(v0, q, relu) | ((uint32_t)e4m3_act(v1, q, relu) << 8) |
               ((uint32_t)e4m3_act(v2, q, relu) << 16) | ((uint32_t)e4m3_act(v3, q, relu) << 24);
    const float lo = relu ? 0.0f : -448.0f;
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_fmed3f(u0, lo, 448.0f),
                                            __builtin_amdgcn_fmed3f(u1, lo, 448.0f), 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_fmed3f(u2, lo, 448.0f),
                                        __builtin_amdgcn_fmed3f(u3, lo, 448.0f), w, true);
    return (uint32_t)w;
}
__device__ __forceinline__ float e4m3_to_f32(uint8_t v) {
    const uint32_t s = (v & 0x80u) << 24;
    const uint32_t e = (v >> 3) & 0xfu, m = v & 7u;
    if (e == 15 && m == 7) return __uint_as_float(0x7fc00000u | s);
    float a = e ? __uint_as_float(((e + 120u) << 23) | (m << 20)) : (float)m * 0.001953125f;
    return __uint_as_float(__float_as_uint(a) | s);
}

// ---------------------------------------------------------------- precision traits
// Storage of one activation / weight element, and the MFMA K step.
// Lane l of a wave supplies, for one K step, VW consecutive K elements of
// row (l % 16) of the A operand and of column (l % 16) of the B operand,
// namely K positions [VW * (l / 16), VW * (l / 16) + VW). The K order inside
// a step is private to the kernel: A and B only have to agree.
template <int P> struct Traits;

template <> struct Traits<P_F32> {
    typedef float T;
    static constexpr int KS = 16;   // K per step: 4 x v_mfma_f32_16x16x4_f32
    static constexpr int VW = 4;
    typedef f4 V;                   // 16 bytes per lane
    __device__ static __forceinline__ void mma(f4& acc, const V& a, const V& b) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
    }
    __device__ static __forceinline__ T from_f32(float v, float) { return v; }
    __device__ static __forceinline__ float to_f32(T v) { return v; }
};

template <> struct Traits<P_BF16> {
    typedef uint16_t T;
    static constexpr int KS = 32;   // v_mfma_f32_16x16x32_bf16
    static constexpr int VW = 8;
    typedef uint4 V;                // 16 bytes per lane
    __device__ static __forceinline__ void mma(f4& acc, const V& a, const V& b) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                      __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
    }
    __device__ static __forceinline__ T from_f32(float v, float) { return f32_to_bf16(v); }
    __device__ static __forceinline__ float to_f32(T v) { return bf16_to_f32(v); }
};

template <> struct Traits<P_FP8> {
    typedef uint8_t T;
    static constexpr int KS = 128;  // v_mfma_scale_f32_16x16x128_f8f6f4, both operands e4m3
    static constexpr int VW = 32;
    typedef i8v V;                  // 32 bytes per lane
    __device__ static __forceinline__ void mma(f4& acc, const V& a, const V& b) {
        // formats 0/0 = e4m3 for A and B; E8M0 block scales 127 = 1.0
        acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc, 0, 0, 0, 127, 0, 127);
    }
    // fp8 values are stored pre-multiplied by the tensor's scale s
    __device__ static __forceinline__ T from_f32(float v, float s) { return f32_to_e4m3(v * s); }
    __device__ static __forceinline__ float to_f32(T v) { return e4m3_to_f32(v); }
};

template <typename V> __device__ __forceinline__ V vzero() {
    V v;
    __builtin_memset(&v, 0, sizeof(V));
    return v;
}

// ---------------------------------------------------------------- training augmentation
// A symmetry of the hemispherical lat-long map (Sec. 5: the loader rotates
// and flips the training maps; read as rotations about the normal by whole
// columns and mirror images through a plane containing it). Map m is turned
// by k = roll[m] mod W columns and mirrored when flip[m] != 0: augmented
// column u holds source column (u - k) mod W, or (k - 1 - u) mod W when
// mirrored, with the normal's (Nx, Ny) reflected (Ny -> -Ny) when mirrored
// and then rotated by 2 pi k / W; the other channels and the target keep
// their values. Every reader of augmented maps (the augmentation kernel and
// the loaders that apply it on the fly) uses these helpers, so they agree
// bit for bit.
struct AugMap {
    int k;
    bool flip;
    float cs, sn;
};
__device__ __forceinline__ AugMap aug_map(const int32_t* roll, const int32_t* flip, long m, int W) {
    AugMap a;
    int k = roll[m] % W;
    if (k < 0) k += W;
    a.k = k;
    a.flip = flip[m] != 0;
    sincosf(6.28318530717958648f * (float)k / (float)W, &a.sn, &a.cs);
    return a;
}
// Source column of augmented column u (0 <= u < W).
__device__ __forceinline__ int aug_src_col(const AugMap& a, int u, int W) {
    int s = a.flip ? a.k - 1 - u : u - a.k;  // in (-2W, W)
    if (s < 0) s += W;
    if (s < 0) s += W;
    return s;
}
// Source column for channels that only move (the target map): no rotation.
__device__ __forceinline__ int aug_src_col(const int32_t* roll, const int32_t* flip, long m, int u, int W) {
    AugMap a;
    int k = roll[m] % W;
    if (k < 0) k += W;
    a.k = k;
    a.flip = flip[m] != 0;
    return aug_src_col(a, u, W);
}
// Channels 3 and 4 (Nx, Ny) of a moved pixel, in place.
__device__ __forceinline__ void aug_normal(const AugMap& a, float& nx, float& ny) {
    const float x = nx, y = a.flip ? -ny : ny;
    nx = fmaf(a.cs, x, -(a.sn * y));
    ny = fmaf(a.sn, x, a.cs * y);
}

}  // namespace drc
