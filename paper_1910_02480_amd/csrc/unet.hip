// The paper's own network (Sec. 4.3 and Sec. 5), inference form: a
// U-Net-like autoencoder with two 3x3 convolutions per stage (batch norm and
// LeakyReLU), 2x2 max-pool, 2x2 bilinear upsampling with skip
// concatenation, and a 1x1 output convolution with ReLU; widths 64-128-256
// and a 256-channel bottleneck (the 20 MB model of Sec. 5).
//
// Kernels (BF16 activations NHWC, FP32 accumulation):
// * unet_conv_kernel: stride-1 convolution (3x3 or 1x1) as an implicit GEMM
//   on v_mfma_f32_16x16x32_bf16: rows = output channels (A = weights, packed
//   in MFMA fragment order so that a fragment is one 1 KB load), columns =
//   output pixels (B gathered straight from NHWC, 16 bytes = 8 channels of
//   one pixel per lane), K = (tap, input channel) in steps of 32. Each wave
//   owns MT row blocks x NPW pixel blocks; the next K step's fragments are
//   loaded before the current step's MFMAs. Epilogue: y = act(acc * scale +
//   shift) with batch norm and bias folded into scale / shift.
// * cast, 2x2 max-pool, and bilinear 2x upsampling fused with the skip
//   concatenation: HBM-bound element kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "drc_cae.h"
#include "common.h"
#include "internal.h"

using namespace drc;

namespace {

constexpr int kUnetLayers = 15;
constexpr float kSlope = 0.01f;
constexpr float kBnEps = 1e-5f;

// (cin, cout, taps, batch norm) in execution order
struct UnetLayer {
    int cin, cout, taps, bn;
};
constexpr UnetLayer kUnet[kUnetLayers] = {
    {7, 64, 9, 1},   {64, 64, 9, 1},   {64, 128, 9, 1},  {128, 128, 9, 1}, {128, 256, 9, 1},
    {256, 256, 9, 1}, {256, 256, 9, 1}, {256, 256, 9, 1}, {512, 256, 9, 1}, {256, 256, 9, 1},
    {384, 128, 9, 1}, {128, 128, 9, 1}, {192, 64, 9, 0},  {64, 64, 9, 0},   {64, 3, 1, 0},
};

__host__ __device__ constexpr int cin_pad(int l) { return l == 0 ? 8 : kUnet[l].cin; }
__host__ __device__ constexpr int kdim(int l) { return kUnet[l].taps * cin_pad(l); }
__host__ __device__ constexpr int kpad(int l) { return (kdim(l) + 31) / 32 * 32; }
__host__ __device__ constexpr int rows_pad(int l) { return (kUnet[l].cout + 15) / 16 * 16; }

long param_count_l(int l) {
    const UnetLayer& L = kUnet[l];
    return (long)L.cout * L.cin * L.taps + L.cout + (L.bn ? 4L * L.cout : 0);
}

// ------------------------------------------------------------------ packing
// Fragment (rb, ks) of layer l: 64 lanes x 8 bf16; lane 16 g + r holds
// W[16 rb + r][32 ks + 8 g .. + 8] with K index k = tap * cin_pad + c.
struct PackArgsU {
    const float* w;  // [cout][taps][cin] (3x3: [cout][3][3][cin])
    const float* b;
    const float* bn; // gamma, beta, mean, var (each [cout]) or null
    uint16_t* pack;
    float* scale;
    float* shift;
    int cin, cinp, cout, taps, ks, rb;
};

__global__ void unet_pack_kernel(PackArgsU a) {
    const long total = (long)a.rb * a.ks * 64 * 8;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int el = (int)(e & 7);
        const int lane = (int)((e >> 3) & 63);
        const long frag = e >> 9;
        const int ks = (int)(frag % a.ks), rb = (int)(frag / a.ks);
        const int co = 16 * rb + (lane & 15);
        const int k = 32 * ks + 8 * (lane >> 4) + el;
        const int t = k / a.cinp, c = k - (k / a.cinp) * a.cinp;
        float v = 0.0f;
        if (co < a.cout && t < a.taps && c < a.cin) v = a.w[((long)co * a.taps + t) * a.cin + c];
        a.pack[e] = f32_to_bf16(v);
    }
    for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < a.cout; c += (long)gridDim.x * blockDim.x) {
        float s = 1.0f, h = a.b[c];
        if (a.bn) {
            const float gamma = a.bn[c], beta = a.bn[a.cout + c], mean = a.bn[2 * a.cout + c],
                        var = a.bn[3 * a.cout + c];
            s = gamma / sqrtf(var + kBnEps);
            h = (a.b[c] - mean) * s + beta;
        }
        a.scale[c] = s;
        a.shift[c] = h;
    }
}

// ------------------------------------------------------------------ convolution
struct ConvArgsU {
    const uint16_t* in;   // [n, H, W, cinp] bf16
    const uint4* pack;    // fragment-ordered weights
    const float* scale;
    const float* shift;
    void* out;            // [n, H, W, cout] bf16, or float32 when out_f32
    const uint4* zero;    // 16 zero bytes: the load of a tap outside the map
    int n, H, W, cinp, cout, ks, act, out_f32;
};

// Output pixels of one pixel block per lane: element offset of the pixel in
// the input, and its (y, x).
struct PixU {
    long base;
    int y, x;
    bool v;
};

template <int MT, int NPW, int TAPS>
__global__ __launch_bounds__(256) void unet_conv_kernel(ConvArgsU a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const long npix = (long)a.n * a.H * a.W;
    const int rb0 = blockIdx.y * MT;
    const int nrb = (a.cout + 15) / 16;
    PixU px[NPW];
#pragma unroll
    for (int j = 0; j < NPW; ++j) {
        const long p = ((long)blockIdx.x * 4 * NPW + wave * NPW + j) * 16 + r16;
        px[j].v = p < npix;
        const long pp = px[j].v ? p : 0;
        const int x = (int)(pp % a.W);
        const long q = pp / a.W;
        px[j].x = x;
        px[j].y = (int)(q % a.H);
        px[j].base = pp * a.cinp;
    }
    f4 acc[MT][NPW];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NPW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    // K step ks covers tap t = (32 ks) / cinp and channels c .. c + 31 when
    // cinp is a multiple of 32; with cinp = 8, lane group g takes tap 4 ks + g.
    auto load_b = [&](int ks, uint4 (&bf)[NPW]) {
        int t, c;
        if (a.cinp % 32 == 0) {
            t = (32 * ks) / a.cinp;
            c = 32 * ks - t * a.cinp + 8 * g;
        } else {
            t = 4 * ks + g;
            c = 0;
        }
        const int dy = TAPS == 9 ? t / 3 - 1 : 0, dx = TAPS == 9 ? t % 3 - 1 : 0;
        // every lane loads (taps outside the map read the zero block): loads
        // under a per-lane condition would make the compiler wait for all
        // loads in flight before the MFMAs that follow
#pragma unroll
        for (int j = 0; j < NPW; ++j) {
            const int yy = px[j].y + dy, xx = px[j].x + dx;
            const bool ok = px[j].v && t < TAPS && (unsigned)yy < (unsigned)a.H && (unsigned)xx < (unsigned)a.W;
            const uint4* src = (const uint4*)(a.in + px[j].base + ((long)dy * a.W + dx) * a.cinp + c);
            bf[j] = *(ok ? src : a.zero);
        }
    };
    auto load_a = [&](int ks, uint4 (&af)[MT]) {
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const int rb = rb0 + i;
            af[i] = *(rb < nrb ? a.pack + ((long)rb * a.ks + ks) * 64 + lane : a.zero);
        }
    };
    uint4 af[MT], bf[NPW];
    load_a(0, af);
    load_b(0, bf);
    for (int ks = 0; ks < a.ks; ++ks) {
        // the next step's loads are unconditional (the last step reloads its
        // own fragments): a load under a condition would make the compiler
        // wait for every load in flight before the MFMAs
        const int kn = min(ks + 1, a.ks - 1);
        uint4 an[MT], bn[NPW];
        load_a(kn, an);
        load_b(kn, bn);
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NPW; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af[i]),
                                                                  __builtin_bit_cast(bf16x8, bf[j]), acc[i][j], 0,
                                                                  0, 0);
#pragma unroll
        for (int i = 0; i < MT; ++i) af[i] = an[i];
#pragma unroll
        for (int j = 0; j < NPW; ++j) bf[j] = bn[j];
    }
    // epilogue: lane holds channels 16 rb + 4 g .. + 3 of pixel 16 pb + r16
#pragma unroll
    for (int j = 0; j < NPW; ++j) {
        if (!px[j].v) continue;
        const long p = px[j].base / a.cinp;
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const int c0 = (rb0 + i) * 16 + 4 * g;
            if (c0 >= a.cout) continue;
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = min(c0 + r, a.cout - 1);
                float y = acc[i][j][r] * a.scale[c] + a.shift[c];
                y = a.act == 1 ? (y > 0.0f ? y : kSlope * y) : (a.act == 2 ? fmaxf(y, 0.0f) : y);
                v[r] = y;
            }
            if (a.out_f32) {
                float* o = (float*)a.out + p * a.cout;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (c0 + r < a.cout) o[c0 + r] = v[r];
            } else {
                const uint32_t lo = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
                const uint32_t hi = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
                *(uint2*)((uint16_t*)a.out + p * a.cout + c0) = make_uint2(lo, hi);
            }
        }
    }
}

// Operands of K step ks for unet_conv_lds_kernel: ACH weight chunks (16 bytes
// of fragment (rb0 + e / 64, ks), lane e % 64) and BCH activation chunks
// (pixel e / 4, channels 8 (e % 4) .. + 8 of the step's tap); taps outside
// the map are zero.
template <int ACH, int BCH>
__device__ __forceinline__ void unet_lds_load(const ConvArgsU& a, int ks, int rb0, const long (&bbase)[BCH],
                                              const int (&by)[BCH], const int (&bx)[BCH], const bool (&bok)[BCH],
                                              uint4 (&ra)[ACH], uint4 (&rb)[BCH]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < ACH; ++j) {
        const int e = tid + 256 * j;
        ra[j] = a.pack[((long)(rb0 + (e >> 6)) * a.ks + ks) * 64 + (e & 63)];
    }
    const int t = (32 * ks) / a.cinp, c = 32 * ks - t * a.cinp;
    const int dy = t / 3 - 1, dx = t % 3 - 1;
#pragma unroll
    for (int j = 0; j < BCH; ++j) {
        // one unconditional load per lane (a selected offset, the value zeroed
        // after): a load behind a selected pointer becomes two guarded loads
        const int yy = by[j] + dy, xx = bx[j] + dx;
        const bool ok = bok[j] && (unsigned)yy < (unsigned)a.H && (unsigned)xx < (unsigned)a.W;
        const long off = ok ? bbase[j] + ((long)dy * a.W + dx) * a.cinp + c : 0;
        const uint4 v = *(const uint4*)(a.in + off);
        rb[j] = ok ? v : make_uint4(0, 0, 0, 0);
    }
}

// Writes the staged operands to LDS buffer st: A fragments first (1 KB
// each, as packed), then B fragments (pixel block q / 16, lane 16 kc + q % 16).
template <int ACH, int BCH, int AF>
__device__ __forceinline__ void unet_lds_store(char* st, const uint4 (&ra)[ACH], const uint4 (&rb)[BCH]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < ACH; ++j) *(uint4*)(st + (tid + 256 * j) * 16) = ra[j];
#pragma unroll
    for (int j = 0; j < BCH; ++j) {
        const int e = tid + 256 * j, q = e >> 2, kc = e & 3;
        *(uint4*)(st + AF * 1024 + (q >> 4) * 1024 + (16 * kc + (q & 15)) * 16) = rb[j];
    }
}

// LDS-tiled variant for the 3x3 layers with cinp a multiple of 32 (all but
// the first): a workgroup computes BM output channels x BN pixels with 4
// waves of 64 x 64 (BM = 128: 2 x 2 waves, BN = 128; BM = 64: 1 x 4 waves,
// BN = 256). Per K step the workgroup stages the BM rows' weight fragments
// (1 KB each, as packed) and the BN pixels' 32 channels of the step's tap
// (16-byte gathers, in MFMA fragment order) in LDS once, so each fragment
// crosses the L1 once per workgroup instead of once per wave; the next
// step's operands are loaded into registers during the current step's
// MFMAs (double-buffered LDS, one barrier per step). Operands, K order and
// epilogue are those of unet_conv_kernel, so the outputs are bitwise equal.
template <int BM>
__global__ __launch_bounds__(256) void unet_conv_lds_kernel(ConvArgsU a) {
    constexpr int WR = BM / 64, WP = 4 / WR;  // waves along rows / pixels
    constexpr int BN = WP * 64;               // pixels per workgroup
    constexpr int AF = BM / 16, BF = BN / 16; // A / B fragments per K step
    constexpr int ACH = AF * 64 / 256, BCH = BF * 64 / 256;  // 16-byte chunks per thread
    constexpr int STAGE = (AF + BF) * 1024;   // bytes of one buffer
    static_assert(ACH >= 1 && BCH >= 1, "every thread stages whole chunks");
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int wr = wave / WP, wp = wave % WP;
    const long npix = (long)a.n * a.H * a.W;
    const long px0 = (long)blockIdx.x * BN;
    const int rb0 = blockIdx.y * AF;

    long bbase[BCH];
    int by[BCH], bx[BCH];
    bool bok[BCH];
#pragma unroll
    for (int j = 0; j < BCH; ++j) {
        const int e = tid + 256 * j;  // (pixel, chunk) index of the tile
        const long p = px0 + (e >> 2);
        bok[j] = p < npix;
        const long pp = bok[j] ? p : 0;
        bx[j] = (int)(pp % a.W);
        by[j] = (int)((pp / a.W) % a.H);
        bbase[j] = pp * a.cinp + 8 * (e & 3);
    }
    uint4 ra[ACH], rb[BCH];
    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    unet_lds_load<ACH, BCH>(a, 0, rb0, bbase, by, bx, bok, ra, rb);
    unet_lds_store<ACH, BCH, AF>(smem, ra, rb);
    __syncthreads();
    for (int ks = 0; ks < a.ks; ++ks) {
        const int cur = ks & 1;
        // unconditional (the last step reloads itself into the idle buffer): operands
        // loaded under a condition were kept in scratch memory by the compiler
        unet_lds_load<ACH, BCH>(a, min(ks + 1, a.ks - 1), rb0, bbase, by, bx, bok, ra, rb);
        const char* st = smem + cur * STAGE;
        uint4 af[4], bf[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) af[i] = *(const uint4*)(st + (wr * 4 + i) * 1024 + lane * 16);
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[j] = *(const uint4*)(st + AF * 1024 + (wp * 4 + j) * 1024 + lane * 16);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af[i]),
                                                                  __builtin_bit_cast(bf16x8, bf[j]), acc[i][j], 0,
                                                                  0, 0);
        unet_lds_store<ACH, BCH, AF>(smem + (cur ^ 1) * STAGE, ra, rb);
        __syncthreads();
    }
    // epilogue (as unet_conv_kernel): lane holds channels 16 rb + 4 g .. + 3 of pixel 16 pb + r16
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const long p = px0 + (wp * 4 + j) * 16 + r16;
        if (p >= npix) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c0 = (rb0 + wr * 4 + i) * 16 + 4 * g;
            if (c0 >= a.cout) continue;
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = min(c0 + r, a.cout - 1);
                float y = acc[i][j][r] * a.scale[c] + a.shift[c];
                y = a.act == 1 ? (y > 0.0f ? y : kSlope * y) : (a.act == 2 ? fmaxf(y, 0.0f) : y);
                v[r] = y;
            }
            const uint32_t lo = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
            const uint32_t hi = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
            *(uint2*)((uint16_t*)a.out + p * a.cout + c0) = make_uint2(lo, hi);
        }
    }
}

// ------------------------------------------------------------------ element kernels
// x float32 [n, H, W, 7] -> bf16 [n, H, W, 8] (zero 8th channel)
__global__ void unet_cast_kernel(const float* x, uint16_t* xb, long npix) {
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < npix; p += (long)gridDim.x * blockDim.x) {
        uint16_t h[8];
#pragma unroll
        for (int c = 0; c < 7; ++c) h[c] = f32_to_bf16(x[7 * p + c]);
        h[7] = 0;
        uint4 v;
        v.x = h[0] | ((uint32_t)h[1] << 16);
        v.y = h[2] | ((uint32_t)h[3] << 16);
        v.z = h[4] | ((uint32_t)h[5] << 16);
        v.w = h[6] | ((uint32_t)h[7] << 16);
        *(uint4*)(xb + 8 * p) = v;
    }
}

__device__ __forceinline__ void unpack8(const uint4& v, float (&f)[8]) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = bf16_to_f32((uint16_t)(w[i] & 0xffffu));
        f[2 * i + 1] = bf16_to_f32((uint16_t)(w[i] >> 16));
    }
}

__device__ __forceinline__ uint4 pack8(const float (&f)[8]) {
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = (uint32_t)f32_to_bf16(f[2 * i]) | ((uint32_t)f32_to_bf16(f[2 * i + 1]) << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// 2x2 max-pool, bf16 [n, H, W, C] -> [n, H/2, W/2, C]; one thread per
// (output pixel, 8 channels). The maximum of bf16 values is exact.
__global__ void unet_pool_kernel(const uint16_t* in, uint16_t* out, int n, int H, int W, int C) {
    const int Ho = H / 2, Wo = W / 2, CG = C / 8;
    const long total = (long)n * Ho * Wo * CG;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int cg = (int)(e % CG);
        const long p = e / CG;
        const int x = (int)(p % Wo);
        const long q = p / Wo;
        const int y = (int)(q % Ho);
        const long m = q / Ho;
        float best[8];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const long src = ((m * H + 2 * y + (d >> 1)) * W + 2 * x + (d & 1)) * C + 8 * cg;
            float f[8];
            unpack8(*(const uint4*)(in + src), f);
#pragma unroll
            for (int i = 0; i < 8; ++i) best[i] = d == 0 ? f[i] : fmaxf(best[i], f[i]);
        }
        *(uint4*)(out + p * C + 8 * cg) = pack8(best);
    }
}

// [upsample2(a) | skip]: a bf16 [n, h, w, Ca], skip bf16 [n, 2h, 2w, Cs] ->
// out bf16 [n, 2h, 2w, Ca + Cs]. Bilinear with half-pixel centres: output
// index i reads source coordinate max(0, (i + 1/2) / 2 - 1/2); one thread
// per (output pixel, 8 channels).
__global__ void unet_upcat_kernel(const uint16_t* a, const uint16_t* skip, uint16_t* out, int n, int h, int w,
                                  int Ca, int Cs) {
    const int H = 2 * h, W = 2 * w, C = Ca + Cs, CG = C / 8;
    const long total = (long)n * H * W * CG;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int cg = (int)(e % CG);
        const long p = e / CG;
        const int x = (int)(p % W);
        const long q = p / W;
        const int y = (int)(q % H);
        const long m = q / H;
        uint4 v;
        if (8 * cg < Ca) {
            const float sy = fmaxf(0.5f * (float)y - 0.25f, 0.0f), sx = fmaxf(0.5f * (float)x - 0.25f, 0.0f);
            const int y0 = min((int)sy, h - 1), x0 = min((int)sx, w - 1);
            const int y1 = min(y0 + 1, h - 1), x1 = min(x0 + 1, w - 1);
            const float fy = sy - (float)y0, fx = sx - (float)x0;
            float f00[8], f01[8], f10[8], f11[8], r[8];
            const long b = m * h;
            unpack8(*(const uint4*)(a + ((b + y0) * w + x0) * Ca + 8 * cg), f00);
            unpack8(*(const uint4*)(a + ((b + y0) * w + x1) * Ca + 8 * cg), f01);
            unpack8(*(const uint4*)(a + ((b + y1) * w + x0) * Ca + 8 * cg), f10);
            unpack8(*(const uint4*)(a + ((b + y1) * w + x1) * Ca + 8 * cg), f11);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float top = f00[i] * (1.0f - fx) + f01[i] * fx;
                const float bot = f10[i] * (1.0f - fx) + f11[i] * fx;
                r[i] = top * (1.0f - fy) + bot * fy;
            }
            v = pack8(r);
        } else {
            v = *(const uint4*)(skip + p * Cs + (8 * cg - Ca));
        }
        *(uint4*)(out + p * C + 8 * cg) = v;
    }
}

int grid_of(long work, int per_block) {
    const long g = (work + per_block - 1) / per_block;
    return (int)(g < 1 ? 1 : (g > 65535 ? 65535 : g));
}

// Activation buffers of a batch (element counts per map at resolution H x W).
struct UnetWs {
    size_t off[24];
    size_t bytes;
};

// buffers: 0 xb, 1 t1, 2 s1, 3 p1, 4 t2, 5 s2, 6 p2, 7 t3, 8 s3, 9 p3, 10 tm, 11 m,
// 12 c3, 13 t4, 14 d3, 15 c2, 16 t5, 17 d2, 18 c1, 19 t6, 20 d1
UnetWs unet_ws(int n, int H, int W) {
    const long P = (long)n * H * W;
    const long elems[21] = {P * 8,       P * 64,      P * 64,       P / 4 * 64,  P / 4 * 128, P / 4 * 128,
                            P / 16 * 128, P / 16 * 256, P / 16 * 256, P / 64 * 256, P / 64 * 256, P / 64 * 256,
                            P / 16 * 512, P / 16 * 256, P / 16 * 256, P / 4 * 384,  P / 4 * 128, P / 4 * 128,
                            P * 192,      P * 64,      P * 64};
    UnetWs w;
    size_t o = 0;
    for (int i = 0; i < 21; ++i) {
        w.off[i] = o;
        o += ((size_t)elems[i] * 2 + 255) / 256 * 256;
    }
    w.bytes = o;
    return w;
}

}  // namespace

struct drc_unet {
    int device;
    uint4* zero;  // 256 zero bytes
    uint16_t* pack[kUnetLayers];
    float* scale[kUnetLayers];
    float* shift[kUnetLayers];
    void* mem;
    int params_set;
};

#define TRYU(expr)                   \
    do {                             \
        drc_status s_ = (expr);      \
        if (s_ != DRC_OK) return s_; \
    } while (0)

extern "C" size_t drc_unet_num_params(void) {
    long t = 0;
    for (int l = 0; l < kUnetLayers; ++l) t += param_count_l(l);
    return (size_t)t;
}

extern "C" drc_status drc_unet_create(drc_unet** out) {
    if (!out) return drc_fail(DRC_ERR_INVALID_ARG, "unet_create: out is NULL");
    *out = nullptr;
    drc_unet* u = new (std::nothrow) drc_unet;
    if (!u) return drc_fail(DRC_ERR_HIP, "unet_create: host allocation failed");
    memset(u, 0, sizeof *u);
    if (hipGetDevice(&u->device) != hipSuccess) {
        delete u;
        return drc_fail(DRC_ERR_HIP, "unet_create: hipGetDevice failed");
    }
    size_t bytes = 0;
    size_t offs[kUnetLayers][3];
    for (int l = 0; l < kUnetLayers; ++l) {
        offs[l][0] = bytes;
        bytes += ((size_t)rows_pad(l) * kpad(l) * 2 + 255) / 256 * 256;
        offs[l][1] = bytes;
        bytes += ((size_t)kUnet[l].cout * 4 + 255) / 256 * 256;
        offs[l][2] = bytes;
        bytes += ((size_t)kUnet[l].cout * 4 + 255) / 256 * 256;
    }
    const size_t zoff = bytes;
    bytes += 256;
    if (hipMalloc(&u->mem, bytes) != hipSuccess) {
        delete u;
        return drc_fail(DRC_ERR_HIP, "unet_create: device allocation of %zu bytes failed", bytes);
    }
    u->zero = (uint4*)((char*)u->mem + zoff);
    if (hipMemset(u->zero, 0, 256) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(u->mem);
        delete u;
        return drc_fail(DRC_ERR_HIP, "unet_create: clearing the zero block failed");
    }
    for (int l = 0; l < kUnetLayers; ++l) {
        u->pack[l] = (uint16_t*)((char*)u->mem + offs[l][0]);
        u->scale[l] = (float*)((char*)u->mem + offs[l][1]);
        u->shift[l] = (float*)((char*)u->mem + offs[l][2]);
    }
    *out = u;
    return DRC_OK;
}

extern "C" void drc_unet_destroy(drc_unet* u) {
    if (!u) return;
    if (u->mem) (void)hipFree(u->mem);
    delete u;
}

extern "C" drc_status drc_unet_set_params(drc_unet* u, const float* d_params, void* stream) {
    if (!u) return drc_fail(DRC_ERR_INVALID_ARG, "unet_set_params: handle is NULL");
    TRYU(check_ptr("unet_set_params", "d_params", d_params, 4, false));
    const hipStream_t s = (hipStream_t)stream;
    long off = 0;
    for (int l = 0; l < kUnetLayers; ++l) {
        const UnetLayer& L = kUnet[l];
        PackArgsU a;
        a.w = d_params + off;
        a.b = a.w + (long)L.cout * L.cin * L.taps;
        a.bn = L.bn ? a.b + L.cout : nullptr;
        a.pack = u->pack[l];
        a.scale = u->scale[l];
        a.shift = u->shift[l];
        a.cin = L.cin;
        a.cinp = cin_pad(l);
        a.cout = L.cout;
        a.taps = L.taps;
        a.ks = kpad(l) / 32;
        a.rb = rows_pad(l) / 16;
        hipLaunchKernelGGL(unet_pack_kernel, dim3(grid_of((long)a.rb * a.ks * 512, 256)), dim3(256), 0, s, a);
        off += param_count_l(l);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return drc_fail(DRC_ERR_HIP, "unet_set_params: launch failed: %s", hipGetErrorString(e));
    u->params_set = 1;
    return DRC_OK;
}

static drc_status unet_shape(const char* who, int n, int H, int W) {
    if (n < 1) return drc_fail(DRC_ERR_SHAPE, "%s: n = %d (must be >= 1)", who, n);
    if (H < 8 || W < 8 || H % 8 || W % 8)
        return drc_fail(DRC_ERR_SHAPE, "%s: H = %d, W = %d (must be multiples of 8, >= 8)", who, H, W);
    if ((long)n * H * W > (1L << 31) / 64)
        return drc_fail(DRC_ERR_SHAPE, "%s: n*H*W = %ld too large", who, (long)n * H * W);
    return DRC_OK;
}

extern "C" drc_status drc_unet_workspace_size(int n, int H, int W, size_t* bytes) {
    if (!bytes) return drc_fail(DRC_ERR_INVALID_ARG, "unet_workspace_size: bytes is NULL");
    TRYU(unet_shape("unet_workspace_size", n, H, W));
    *bytes = unet_ws(n, H, W).bytes;
    return DRC_OK;
}

template <int MT, int NPW, int TAPS>
static void launch_conv(const ConvArgsU& c, hipStream_t s) {
    const long npix = (long)c.n * c.H * c.W;
    const dim3 grid((unsigned)((npix + 64 * NPW - 1) / (64 * NPW)), (unsigned)((c.cout + 16 * MT - 1) / (16 * MT)));
    hipLaunchKernelGGL((unet_conv_kernel<MT, NPW, TAPS>), grid, dim3(256), 0, s, c);
}

template <int BM>
static void launch_conv_lds(const ConvArgsU& c, hipStream_t s) {
    constexpr int BN = 4 / (BM / 64) * 64;
    const long npix = (long)c.n * c.H * c.W;
    const dim3 grid((unsigned)((npix + BN - 1) / BN), (unsigned)(c.cout / BM));
    const int lds = 2 * (BM / 16 + BN / 16) * 1024;
    hipLaunchKernelGGL((unet_conv_lds_kernel<BM>), grid, dim3(256), lds, s, c);
}

extern "C" drc_status drc_unet_forward(drc_unet* u, const float* d_x, float* d_y, int n, int H, int W,
                                       void* d_ws, size_t ws_bytes, void* stream) {
    if (!u) return drc_fail(DRC_ERR_INVALID_ARG, "unet_forward: handle is NULL");
    if (!u->params_set) return drc_fail(DRC_ERR_STATE, "unet_forward: call drc_unet_set_params first");
    TRYU(unet_shape("unet_forward", n, H, W));
    TRYU(check_ptr("unet_forward", "d_x", d_x, 4, false));
    TRYU(check_ptr("unet_forward", "d_y", d_y, 4, false));
    TRYU(check_ptr("unet_forward", "d_ws", d_ws, 256, false));
    const UnetWs ws = unet_ws(n, H, W);
    if (ws_bytes < ws.bytes)
        return drc_fail(DRC_ERR_WORKSPACE, "unet_forward: workspace %zu < %zu bytes", ws_bytes, ws.bytes);
    const hipStream_t s = (hipStream_t)stream;
    auto buf = [&](int i) { return (uint16_t*)((char*)d_ws + ws.off[i]); };
    const long P = (long)n * H * W;
    hipLaunchKernelGGL(unet_cast_kernel, dim3(grid_of(P, 256)), dim3(256), 0, s, d_x, buf(0), P);

    auto conv = [&](int l, const uint16_t* in, void* out, int h, int w) {
        ConvArgsU c;
        c.in = in;
        c.pack = (const uint4*)u->pack[l];
        c.scale = u->scale[l];
        c.shift = u->shift[l];
        c.out = out;
        c.zero = u->zero;
        c.n = n;
        c.H = h;
        c.W = w;
        c.cinp = cin_pad(l);
        c.cout = kUnet[l].cout;
        c.ks = kpad(l) / 32;
        c.act = l == kUnetLayers - 1 ? 2 : 1;
        c.out_f32 = l == kUnetLayers - 1;
        if (kUnet[l].taps == 1) launch_conv<1, 4, 1>(c, s);
        else if (c.cinp % 32 == 0 && c.cout % 128 == 0 && !c.out_f32) launch_conv_lds<128>(c, s);
        else if (c.cinp % 32 == 0 && c.cout % 64 == 0 && !c.out_f32) launch_conv_lds<64>(c, s);
        else launch_conv<4, 4, 9>(c, s);
    };
    auto pool = [&](const uint16_t* in, uint16_t* out, int h, int w, int C) {
        hipLaunchKernelGGL(unet_pool_kernel, dim3(grid_of((long)n * h * w / 4 * (C / 8), 256)), dim3(256), 0, s,
                           in, out, n, h, w, C);
    };
    auto upcat = [&](const uint16_t* a, const uint16_t* skip, uint16_t* out, int h, int w, int Ca, int Cs) {
        hipLaunchKernelGGL(unet_upcat_kernel, dim3(grid_of((long)n * 4 * h * w * ((Ca + Cs) / 8), 256)), dim3(256),
                           0, s, a, skip, out, n, h, w, Ca, Cs);
    };
    const int H2 = H / 2, W2 = W / 2, H4 = H / 4, W4 = W / 4, H8 = H / 8, W8 = W / 8;
    conv(0, buf(0), buf(1), H, W);
    conv(1, buf(1), buf(2), H, W);            // s1
    pool(buf(2), buf(3), H, W, 64);
    conv(2, buf(3), buf(4), H2, W2);
    conv(3, buf(4), buf(5), H2, W2);          // s2
    pool(buf(5), buf(6), H2, W2, 128);
    conv(4, buf(6), buf(7), H4, W4);
    conv(5, buf(7), buf(8), H4, W4);          // s3
    pool(buf(8), buf(9), H4, W4, 256);
    conv(6, buf(9), buf(10), H8, W8);
    conv(7, buf(10), buf(11), H8, W8);        // bottleneck
    upcat(buf(11), buf(8), buf(12), H8, W8, 256, 256);
    conv(8, buf(12), buf(13), H4, W4);
    conv(9, buf(13), buf(14), H4, W4);        // d3
    upcat(buf(14), buf(5), buf(15), H4, W4, 256, 128);
    conv(10, buf(15), buf(16), H2, W2);
    conv(11, buf(16), buf(17), H2, W2);       // d2
    upcat(buf(17), buf(2), buf(18), H2, W2, 128, 64);
    conv(12, buf(18), buf(19), H, W);
    conv(13, buf(19), buf(20), H, W);         // d1
    conv(14, buf(20), d_y, H, W);             // 1x1 + ReLU, float32
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return drc_fail(DRC_ERR_HIP, "unet_forward: launch failed: %s", hipGetErrorString(e));
    return DRC_OK;
}
