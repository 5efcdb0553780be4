// Whole-network BF16 forward of the autoencoder (Sec. 4.3, Fig. 3 layout as
// configured: 3x3 stride-2 encoder 7->32->64->128 with ReLU, mirrored
// stride-2 transposed-convolution decoder with skip concatenation, linear
// 3-channel output), one map per workgroup pass, every activation of the
// map resident in LDS.
//
// The layer path moves every activation through HBM (about 690 KB per 64x64
// map in BF16 with FP32 input and output); here a map costs its FP32 input
// (7 channels) and output (3 channels) plus one 64 KB round trip of h1
// through a per-workgroup slot that stays in the L2/last-level caches.
//
// LDS plan for an H x W map (bytes, BF16 NHWC, 16-byte channel chunks XOR-
// swizzled by column against bank conflicts):
//   R0 [0, 16HW)           h1 (E1 -> E2), then u2 (D2 -> D1)
//   R1 [16HW, 24HW)        h2 (E2 -> D2)
//   R2 [24HW, 32HW)        u3 (D3 -> D2)
//   R3 [32HW, 36HW)        h3 (E3 -> D3)
//   R1+R2                  x as BF16, 8 channels (staging -> E1), and h1
//                          again for D1 (reloaded from the workgroup's slot)
//   [36HW, 36HW + 256)     zeros, read by taps that fall outside the map
// 36 HW bytes + 256 in all: 144 KB at 64x64 (one workgroup per CU), 36 KB
// at 32x32.
//
// Every GEMM uses the same weight packs, K order and epilogue arithmetic as
// the layer kernels, so the two paths agree bit for bit.
#include <hip/hip_runtime.h>
#include <string.h>

#include "drc_cae.h"
#include "common.h"
#include "conv_layer.h"
#include "internal.h"

using namespace drc;

namespace {

constexpr int FT = 512;      // threads per workgroup
constexpr int FW = FT / 64;  // waves
constexpr int kZeroBytes = 256;  // zero block read by taps outside the map (any chunk XOR stays inside)

struct FusedArgs {
    const float* x;      // [.., H, W, 7] float32
    float* y;            // [.., H, W, 3] float32
    int nmaps;
    const long* x_off;   // element offset of each map (null: packed)
    const long* y_off;
    const uint16_t* w[6];  // forward packs in MFMA fragment order
    const float* b[6];
    char* scratch;       // one h1 slot of 16 H W bytes per workgroup (when h1 is not saved)
    char* save[5];       // optional: h1 h2 h3 u3 u2 of every map, plain NHWC BF16 (null = not kept)
    int final_relu;
};

__device__ __forceinline__ uint16_t bf16_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

// Byte offset of 16-byte chunk `chunk` of pixel (y, x) in an LDS tensor of C
// channels and row length WI. The chunk index is XORed with bits of the
// column x, so that the 16 lanes of an MFMA operand, which read the same
// chunk of pixels 1 or 2 columns apart, spread over the LDS banks; since the
// swizzle ignores the row, moving by whole rows is a constant byte offset.
template <int C>
__device__ __forceinline__ int swz(int x) {
    constexpr int CH = C / 8;
    if constexpr (CH == 1) return 0;
    else if constexpr (CH == 4) return (x >> 2) & 3;
    else if constexpr (CH == 8) return (x >> 1) & 7;
    else return x & 15;
}
template <int C, int WI>
__device__ __forceinline__ int loff(int y, int x, int chunk) {
    constexpr int CH = C / 8;
    return (y * WI + x) * (C * 2) + ((chunk ^ swz<C>(x)) & (CH - 1)) * 16;
}

// Stores channels [ch, ch+4) of pixel (y, x) (bias added, optional ReLU) as BF16.
template <int C, int WI>
__device__ __forceinline__ void lds_store4(char* smem, int region, int y, int x, int ch, const f4& acc,
                                           const float* bias, bool relu) {
    float v[4] = {acc.x + bias[0], acc.y + bias[1], acc.z + bias[2], acc.w + bias[3]};
    if (relu) {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (v[e] < 0.0f) ? 0.0f : v[e];
    }
    uint2 w;
    w.x = (uint32_t)bf16_bits(v[0]) | ((uint32_t)bf16_bits(v[1]) << 16);
    w.y = (uint32_t)bf16_bits(v[2]) | ((uint32_t)bf16_bits(v[3]) << 16);
    *(uint2*)(smem + region + loff<C, WI>(y, x, ch >> 3) + ((ch >> 2) & 1) * 8) = w;
}

__device__ __forceinline__ void mma(f4& acc, const uint4& a, const uint4& b) { Traits<P_BF16>::mma(acc, a, b); }

// Hides a value from the optimiser. Weight loads are then issued inside the
// layer instead of being hoisted out of the map loop (where they would pin
// hundreds of registers across every layer), and per-lane addresses are
// recomputed per layer rather than kept live. Only an integer goes through
// the asm statement, so pointers keep their global address space.
template <typename T>
__device__ __forceinline__ const T* opaque(const T* p) {
    int z = 0;
    asm volatile("" : "+s"(z));
    return p + z;
}
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

__device__ __forceinline__ uint4 lds16(const char* smem, int off) { return *(const uint4*)(smem + off); }

// x (float32, 7 channels) -> LDS region xs as BF16 with 8 channels (channel
// 7 = 0), 16 bytes per pixel. A thread converts 4 consecutive pixels (112
// bytes of input = 7 float4, read together) per pass.
template <int H, int W>
__device__ __forceinline__ void stage_x(char* smem, int xs, const float* xm) {
    constexpr int Q = H * W / 4;
    constexpr int IT = (Q + FT - 1) / FT;
    const int tid = opaque_tid();
    float4 v[IT][7];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int q = tid + it * FT;
        if (Q % FT == 0 || q < Q)
#pragma unroll
            for (int k = 0; k < 7; ++k) v[it][k] = ((const float4*)xm)[q * 7 + k];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int q = tid + it * FT;
        if (Q % FT == 0 || q < Q) {
            const float* f = (const float*)v[it];
#pragma unroll
            for (int px = 0; px < 4; ++px) {
                uint4 o;
                o.x = (uint32_t)bf16_bits(f[7 * px + 0]) | ((uint32_t)bf16_bits(f[7 * px + 1]) << 16);
                o.y = (uint32_t)bf16_bits(f[7 * px + 2]) | ((uint32_t)bf16_bits(f[7 * px + 3]) << 16);
                o.z = (uint32_t)bf16_bits(f[7 * px + 4]) | ((uint32_t)bf16_bits(f[7 * px + 5]) << 16);
                o.w = (uint32_t)bf16_bits(f[7 * px + 6]);
                *(uint4*)(smem + xs + (4 * q + px) * 16) = o;
            }
        }
    }
}

// Stride-2 3x3 convolution, LDS -> LDS, bias + ReLU (E1, E2, E3). Weights:
// the layer pack [COUT][KSTEPS*32] (k = tap * CIN + c) in fragment order. Wave w owns the row blocks of group
// w % TR for the whole layer and loads their weights (its A panel) into
// registers once; it then walks the pixel tiles w / TR, w / TR + FW / TR, ...
// (NPW blocks of 16 consecutive output pixels each). Taps that fall outside
// the map read the zero block at zoff.
template <int HI, int WI, int CIN, int COUT, int MT, int NPW>
__device__ __forceinline__ void conv_phase(char* smem, int in, int out, int zoff, const uint16_t* wp,
                                           const float* bias_g) {
    constexpr int HO = HI / 2, WO = WI / 2;
    constexpr int PB = HO * WO / 16, RB = COUT / 16;
    constexpr int KSTEPS = (9 * CIN + 31) / 32;
    constexpr int TR = RB / MT, TP = PB / NPW;
    constexpr int ROW = WI * CIN * 2;  // bytes per input row
    static_assert(RB % MT == 0 && PB % NPW == 0 && FW % TR == 0, "tiles cover the layer");
    const int tid = opaque_tid();
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int tr = (wave + blockIdx.x) % TR;  // rotated by workgroup: CUs start on different weights
    const uint16_t* w = opaque(wp);
    uint4 A[KSTEPS][MT];
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks)
#pragma unroll
        for (int m = 0; m < MT; ++m)
            A[ks][m] = *(const uint4*)(w + ((size_t)((tr * MT + m) * KSTEPS + ks) * 64 + lane) * 8);
    const float* bg = opaque(bias_g);
    float bias[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[m][e] = bg[(tr * MT + m) * 16 + g * 4 + e];
    // CIN == 8: the lane group g takes tap 4 ks + g of every K step
    int dk[KSTEPS];
    bool tv[KSTEPS], nt[KSTEPS], nl[KSTEPS];
    if constexpr (CIN == 8) {
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            const int t = ks * 4 + g, kh = t / 3, kw = t - (t / 3) * 3;
            tv[ks] = t < 9;
            nt[ks] = kh == 0;
            nl[ks] = kw == 0;
            dk[ks] = kh * ROW + kw * 16;
        }
    }
    for (int tp = wave / TR; tp < TP; tp += FW / TR) {
        int oy[NPW], ox[NPW];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = (tp * NPW + p) * 16 + r16;
            oy[p] = pix / WO;
            ox[p] = pix % WO;
        }
        // byte offsets of the 9 taps (CIN >= 32) or of the lane's tap per K step (CIN == 8)
        int off[NPW][CIN == 8 ? KSTEPS : 9];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const bool top = oy[p] > 0, left = ox[p] > 0;
            if constexpr (CIN == 8) {
                const int base = in + ((2 * oy[p] - 1) * WI + 2 * ox[p] - 1) * 16;
#pragma unroll
                for (int ks = 0; ks < KSTEPS; ++ks)
                    off[p][ks] = (tv[ks] && (top || !nt[ks]) && (left || !nl[ks])) ? base + dk[ks] : zoff;
            } else {
#pragma unroll
                for (int kw = 0; kw < 3; ++kw) {
                    const int b = in + loff<CIN, WI>(2 * oy[p] - 1, 2 * ox[p] + kw - 1, g);
#pragma unroll
                    for (int kh = 0; kh < 3; ++kh)
                        off[p][kh * 3 + kw] = ((kh == 0 && !top) || (kw == 0 && !left)) ? zoff : b + kh * ROW;
                }
            }
        }
        f4 acc[MT][NPW];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int p = 0; p < NPW; ++p) acc[m][p] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            uint4 b[NPW];
#pragma unroll
            for (int p = 0; p < NPW; ++p) {
                if constexpr (CIN == 8) {
                    b[p] = lds16(smem, off[p][ks]);
                } else {
                    // K step ks covers channels [(ks*32) % CIN, +32) of tap (ks*32) / CIN;
                    // chunk (c0 / 8 + g) ^ swz = (g ^ swz) ^ (c0 / 8): an XOR of the byte offset
                    const int t = ks * 32 / CIN, c0 = ks * 32 % CIN;
                    b[p] = lds16(smem, off[p][t] ^ (c0 / 8 * 16));
                }
            }
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int p = 0; p < NPW; ++p) mma(acc[m][p], A[ks][m], b[p]);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int ch = (tr * MT + m) * 16 + g * 4;
#pragma unroll
            for (int p = 0; p < NPW; ++p)
                lds_store4<COUT, WO>(smem, out, oy[p], ox[p], ch, acc[m][p], bias[m], true);
        }
    }
}

// Stride-2 3x3 transposed convolution over all four output phases, LDS ->
// LDS, bias + ReLU (D3, D2). Input = [in0 (C0 ch) | in1 (C1 ch)] at HI x WI;
// GEMM pixel (a, b) gathers its neighbours (a + di, b + dj) and feeds the
// (phase, neighbour) weight blocks (pack [q][COUT][C0 + C1], fragment
// order). The 9 blocks
// are split into two sets of whole phases, SET 0 = phases 0-2 (blocks
// 0-4) and SET 1 = phase 3 (blocks 5-8), so that a wave loads only the
// weights of its set and of its row blocks into registers (the weights are
// read from L2 and their bandwidth bounds these layers). Within a phase the
// accumulation order is the layer kernel's: K step, then block.
template <int HI, int WI, int C0, int C1, int COUT, int MT, int NPW, int SET>
__device__ __forceinline__ void pairs_set(char* smem, int in0, int in1, int out, int zoff, const uint16_t* wp,
                                          const float* bias_g, int tr, int tp0, int tp_step) {
    constexpr int CIN = C0 + C1, PB = HI * WI / 16, KSN = CIN / 32;
    constexpr int WO = 2 * WI;
    constexpr int TP = PB / NPW;
    constexpr int ROW = WI * C0 * 2;
    constexpr int NSRC = C1 > 0 ? 2 : 1;
    constexpr int Q0 = SET ? 5 : 0, NQ = SET ? 4 : 5;   // weight blocks of the set
    constexpr int PH0 = SET ? 3 : 0, NPH = SET ? 1 : 3; // its phases
    constexpr int NNB = SET ? 4 : 3;                    // neighbours it reads
    const int lane = opaque_tid() & 63;
    const int g = lane >> 4, r16 = lane & 15;
    const uint16_t* w = opaque(wp);
    uint4 A[KSN][NQ][MT];
#pragma unroll
    for (int ks = 0; ks < KSN; ++ks)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int m = 0; m < MT; ++m)
                A[ks][q][m] =
                    *(const uint4*)(w + ((size_t)(((Q0 + q) * (COUT / 16) + tr * MT + m) * KSN + ks) * 64 + lane) * 8);
    const float* bg = opaque(bias_g);
    float bias[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[m][e] = bg[(tr * MT + m) * 16 + g * 4 + e];
    for (int tp = tp0; tp < TP; tp += tp_step) {
        int ia[NPW], ib[NPW];
        int off[NPW][NSRC][4];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = (tp * NPW + p) * 16 + r16;
            ia[p] = pix / WI;
            ib[p] = pix % WI;
            const bool down = ia[p] + 1 < HI, right = ib[p] + 1 < WI;
#pragma unroll
            for (int s = 0; s < NSRC; ++s)
#pragma unroll
                for (int dj = 0; dj < 2; ++dj) {
                    const int b = (s ? in1 : in0) + loff<C0, WI>(ia[p], ib[p] + dj, g);
                    off[p][s][dj] = (dj && !right) ? zoff : b;
                    off[p][s][2 + dj] = ((dj && !right) || !down) ? zoff : b + ROW;
                }
        }
        f4 acc[NPH][MT][NPW];
#pragma unroll
        for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int p = 0; p < NPW; ++p) acc[ph][m][p] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KSN; ++ks) {
            const int s = ks * 32 >= C0 ? 1 : 0;
            const int c0 = ks * 32 - s * C0;  // first channel of the step within its source
            uint4 bv[NNB][NPW];
#pragma unroll
            for (int nb = 0; nb < NNB; ++nb)
#pragma unroll
                for (int p = 0; p < NPW; ++p) bv[nb][p] = lds16(smem, off[p][s][nb] ^ (c0 / 8 * 16));
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int ph = pair_phase(Q0 + q) - PH0, nb = pair_nb(Q0 + q);
#pragma unroll
                for (int m = 0; m < MT; ++m)
#pragma unroll
                    for (int p = 0; p < NPW; ++p) mma(acc[ph][m][p], A[ks][q][m], bv[nb][p]);
            }
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int ch = (tr * MT + m) * 16 + g * 4;
#pragma unroll
            for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
                for (int p = 0; p < NPW; ++p) {
                    const int P = PH0 + ph;
                    lds_store4<COUT, WO>(smem, out, 2 * ia[p] + (P >> 1), 2 * ib[p] + (P & 1), ch, acc[ph][m][p],
                                         bias[m], true);
                }
        }
    }
}

// Work split of a transposed-convolution layer: 2 * TR groups (row-block
// group x set), rotated by workgroup so that CUs start on different weights.
template <int HI, int WI, int C0, int C1, int COUT, int MT, int NPW>
__device__ __forceinline__ void pairs_phase(char* smem, int in0, int in1, int out, int zoff, const uint16_t* wp,
                                            const float* bias_g) {
    constexpr int PB = HI * WI / 16, RB = COUT / 16, TR = RB / MT, NG = 2 * TR;
    static_assert(RB % MT == 0 && PB % NPW == 0 && FW % NG == 0 && C0 % 32 == 0 && C1 % 32 == 0,
                  "tiles cover the layer");
    static_assert(C1 == 0 || C1 == C0, "both sources share one LDS layout");
    const int wave = opaque_tid() >> 6;
    const int gid = (wave + blockIdx.x) % NG;
    const int tr = gid >> 1, set = gid & 1;
    const int tp0 = wave / NG, step = FW / NG;
    if (set == 0)
        pairs_set<HI, WI, C0, C1, COUT, MT, NPW, 0>(smem, in0, in1, out, zoff, wp, bias_g, tr, tp0, step);
    else
        pairs_set<HI, WI, C0, C1, COUT, MT, NPW, 1>(smem, in0, in1, out, zoff, wp, bias_g, tr, tp0, step);
}

// D1: transposed convolution [u2 | h1] (32 + 32 channels at HI x WI) -> 3
// channels, linear, float32 to global. Merged rows r = phase * 3 + co (12 of
// 16 used), K = neighbour * 64 + c, pack [16][256] in fragment order.
template <int HI, int WI, int NPW>
__device__ __forceinline__ void d1_phase(char* smem, int u2, int h1, int zoff, float* ym, const uint16_t* wp,
                                         const float* bias_g, bool relu) {
    constexpr int PB = HI * WI / 16, WO = 2 * WI, TP = PB / NPW;
    constexpr int ROW = WI * 64;
    static_assert(PB % NPW == 0, "tiles cover the layer");
    const int tid = opaque_tid();
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    uint4 a[8];
    const uint16_t* w = opaque(wp);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) a[ks] = *(const uint4*)(w + ((size_t)ks * 64 + lane) * 8);
    const float* bg = opaque(bias_g);
    float bias[4];
    int rph[4], rco[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = g * 4 + e;
        rph[e] = r / 3;
        rco[e] = r - (r / 3) * 3;
        bias[e] = r < 12 ? bg[rco[e]] : 0.0f;
    }
    for (int tp = wave; tp < TP; tp += FW) {
        int ia[NPW], ib[NPW];
        int off[NPW][4];  // neighbours of the pixel in u2; h1 is at h1 - u2 further on
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = (tp * NPW + p) * 16 + r16;
            ia[p] = pix / WI;
            ib[p] = pix % WI;
            const bool down = ia[p] + 1 < HI, right = ib[p] + 1 < WI;
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
                const int b = loff<32, WI>(ia[p], ib[p] + dj, g);
                off[p][dj] = (dj && !right) ? -1 : b;
                off[p][2 + dj] = ((dj && !right) || !down) ? -1 : b + ROW;
            }
        }
        f4 acc[NPW];
#pragma unroll
        for (int p = 0; p < NPW; ++p) acc[p] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const int nb = ks >> 1;
            const int src = (ks & 1) ? h1 : u2;
#pragma unroll
            for (int p = 0; p < NPW; ++p) {
                const int o = off[p][nb];
                mma(acc[p], a[ks], lds16(smem, o < 0 ? zoff : src + o));
            }
        }
#pragma unroll
        for (int p = 0; p < NPW; ++p)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (g * 4 + e >= 12) continue;
                const int ph = rph[e];
                const int opix = (2 * ia[p] + (ph >> 1)) * WO + 2 * ib[p] + (ph & 1);
                float v = acc[p][e] + bias[e];
                if (relu) v = (v < 0.0f) ? 0.0f : v;
                ym[opix * 3 + rco[e]] = v;
            }
    }
}

// Copies an LDS tensor (C channels, HI x WI, column-swizzled chunks) to a
// plain NHWC tensor in global memory and back, 16 bytes per thread step:
// global chunks are consecutive, the LDS side undoes / applies the swizzle.
template <int C, int HI, int WI>
__device__ __forceinline__ void copy_out(char* dst, const char* smem, int region) {
    constexpr int CH = C / 8, N = HI * WI * CH;
    for (int i = threadIdx.x; i < N; i += FT) {
        const int pix = i / CH, j = i - pix * CH;
        ((uint4*)dst)[i] = *(const uint4*)(smem + region + loff<C, WI>(pix / WI, pix % WI, j));
    }
}
template <int C, int HI, int WI>
__device__ __forceinline__ void copy_in(char* smem, int region, const char* src) {
    constexpr int CH = C / 8, N = HI * WI * CH;
    for (int i = threadIdx.x; i < N; i += FT) {
        const int pix = i / CH, j = i - pix * CH;
        *(uint4*)(smem + region + loff<C, WI>(pix / WI, pix % WI, j)) = ((const uint4*)src)[i];
    }
}

// MID = false: the whole network, x -> y (h1 kept in a per-workgroup slot
// or in save[0]; every non-null save[k] receives that activation).
// MID = true: the recompute of a training backward, h2 (read from save[1])
// -> h3, u3, u2 (written to save[2..4]); E1, E2 and D1 are skipped.
template <int H, int W, bool MID>
__global__ __launch_bounds__(FT) void cae_fused_forward_kernel(const FusedArgs a) {
    extern __shared__ __align__(16) char smem[];
    constexpr int HW = H * W;
    constexpr int R0 = 0, R1 = 16 * HW, R2 = 24 * HW, R3 = 32 * HW, ZO = 36 * HW;
    // tiles: a wave owns one group of row blocks (MT blocks of 16) per layer and
    // walks pixel tiles of NPW blocks; chosen so that 8 waves have work and
    // few waves load the same weights
    constexpr int E1N = (HW / 64) >= 8 * 4 * 2 ? 4 : 2;     // E1: 2 row blocks (one group), PB = HW/64
    constexpr int E2N = (HW / 256) >= 8 ? 4 : 1;            // E2: 4 groups of 1, PB = HW/256
    constexpr int E3N = (HW / 1024) >= 4 ? 4 : 1;           // E3: 8 groups of 1, PB = HW/1024
    constexpr int D3N = (HW / 1024) >= 4 ? 2 : 1;           // D3: 4 groups x 2 sets, PB = HW/1024
    constexpr int D2N = (HW / 256) >= 16 ? 2 : 1;           // D2: 2 groups x 2 sets, PB = HW/256
    constexpr int D1N = (HW / 64) >= 8 * 4 ? 4 : 2;         // D1: PB = HW/64
    // per-map bytes of h1 h2 h3 u3 u2
    constexpr long B1 = 16L * HW, B2 = 8L * HW, B3 = 4L * HW, B4 = 8L * HW, B5 = 16L * HW;
    if (threadIdx.x < kZeroBytes / 16) *(uint4*)(smem + ZO + 16 * threadIdx.x) = uint4{0u, 0u, 0u, 0u};
    for (int m = blockIdx.x; m < a.nmaps; m += gridDim.x) {
        if constexpr (!MID) {
            const float* xm = a.x + (a.x_off ? a.x_off[m] : (long)m * HW * 7);
            float* ym = a.y + (a.y_off ? a.y_off[m] : (long)m * HW * 3);
            char* slot = a.save[0] ? a.save[0] + m * B1 : a.scratch + (size_t)blockIdx.x * B1;
            stage_x<H, W>(smem, R1, xm);
            __syncthreads();
            conv_phase<H, W, 8, 32, 2, E1N>(smem, R1, R0, ZO, a.w[0], a.b[0]);
            __syncthreads();
            copy_out<32, H / 2, W / 2>(slot, smem, R0);
            conv_phase<H / 2, W / 2, 32, 64, 1, E2N>(smem, R0, R1, ZO, a.w[1], a.b[1]);
            __syncthreads();
            if (a.save[1]) copy_out<64, H / 4, W / 4>(a.save[1] + m * B2, smem, R1);
            conv_phase<H / 4, W / 4, 64, 128, 1, E3N>(smem, R1, R3, ZO, a.w[2], a.b[2]);
            __syncthreads();
            if (a.save[2]) copy_out<128, H / 8, W / 8>(a.save[2] + m * B3, smem, R3);
            pairs_phase<H / 8, W / 8, 128, 0, 64, 1, D3N>(smem, R3, R3, R2, ZO, a.w[3], a.b[3]);
            __syncthreads();
            if (a.save[3]) copy_out<64, H / 4, W / 4>(a.save[3] + m * B4, smem, R2);
            pairs_phase<H / 4, W / 4, 64, 64, 32, 1, D2N>(smem, R2, R1, R0, ZO, a.w[4], a.b[4]);
            __syncthreads();
            if (a.save[4]) copy_out<32, H / 2, W / 2>(a.save[4] + m * B5, smem, R0);
            copy_in<32, H / 2, W / 2>(smem, R1, slot);
            __syncthreads();
            d1_phase<H / 2, W / 2, D1N>(smem, R0, R1, ZO, ym, a.w[5], a.b[5], a.final_relu != 0);
            __syncthreads();
        } else {
            copy_in<64, H / 4, W / 4>(smem, R1, a.save[1] + m * B2);
            __syncthreads();
            conv_phase<H / 4, W / 4, 64, 128, 1, E3N>(smem, R1, R3, ZO, a.w[2], a.b[2]);
            __syncthreads();
            copy_out<128, H / 8, W / 8>(a.save[2] + m * B3, smem, R3);
            pairs_phase<H / 8, W / 8, 128, 0, 64, 1, D3N>(smem, R3, R3, R2, ZO, a.w[3], a.b[3]);
            __syncthreads();
            copy_out<64, H / 4, W / 4>(a.save[3] + m * B4, smem, R2);
            pairs_phase<H / 4, W / 4, 64, 64, 32, 1, D2N>(smem, R2, R1, R0, ZO, a.w[4], a.b[4]);
            __syncthreads();
            copy_out<32, H / 2, W / 2>(a.save[4] + m * B5, smem, R0);
            __syncthreads();
        }
    }
}

template <int H, int W, bool MID>
drc_status launch_fused(const FusedArgs& a, int grid, hipStream_t s) {
    const int lds = 36 * H * W + kZeroBytes;
    auto kern = cae_fused_forward_kernel<H, W, MID>;
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
            return drc_fail(DRC_ERR_HIP, "fused forward: cannot raise the LDS limit to %d bytes", lds);
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(FT), lds, s, a);
    return check_launch("fused forward");
}

FusedArgs fused_args(const drc_cae* h, int n) {
    FusedArgs a;
    memset(&a, 0, sizeof a);
    a.nmaps = n;
    for (int l = 0; l < 6; ++l) {
        a.w[l] = (const uint16_t*)h->wfrag[l];
        a.b[l] = h->bias + bias_slot(l);
    }
    a.final_relu = h->desc.final_relu;
    return a;
}

}  // namespace

// Map sizes the fused kernel is built for.
bool fused_forward_size(int H, int W) { return (H == 64 && W == 64) || (H == 32 && W == 32); }

// Workgroups of one fused launch over n maps of H x W.
int fused_forward_grid(const drc_cae* h, int n, int H, int W) {
    const int per_cu = (H * W >= 4096) ? 1 : 2;
    return std::max(1, std::min(n, h->num_cu * per_cu));
}

// Scratch bytes of one fused launch (one h1 slot per workgroup) when h1 is not saved.
size_t fused_forward_scratch(const drc_cae* h, int n, int H, int W) {
    return (size_t)fused_forward_grid(h, n, H, W) * 16 * H * W;
}

drc_status fused_forward(drc_cae* h, const float* x, float* y, int n, int H, int W, const long* x_off,
                         const long* y_off, void* scratch, size_t scratch_bytes, hipStream_t s,
                         char* const* save) {
    if (h->prec != P_BF16 || !fused_forward_size(H, W))
        return drc_fail(DRC_ERR_UNSUPPORTED, "fused forward: BF16 maps of 32x32 or 64x64 only");
    if (n < 1) return DRC_OK;
    FusedArgs a = fused_args(h, n);
    if (save)
        for (int k = 0; k < 5; ++k) a.save[k] = save[k];
    if (!a.save[0] && scratch_bytes < fused_forward_scratch(h, n, H, W))
        return drc_fail(DRC_ERR_WORKSPACE, "fused forward: scratch %zu < %zu bytes", scratch_bytes,
                        fused_forward_scratch(h, n, H, W));
    a.x = x;
    a.y = y;
    a.x_off = x_off;
    a.y_off = y_off;
    a.scratch = (char*)scratch;
    const int grid = fused_forward_grid(h, n, H, W);
    const long tok = prof_begin(h, PROF_FUSED, s);
    drc_status st = (H == 64) ? launch_fused<64, 64, false>(a, grid, s) : launch_fused<32, 32, false>(a, grid, s);
    prof_end(h, tok, s);
    return st;
}

drc_status fused_recompute(drc_cae* h, int n, int H, int W, const void* h2, void* h3, void* u3, void* u2,
                           hipStream_t s) {
    if (h->prec != P_BF16 || !fused_forward_size(H, W))
        return drc_fail(DRC_ERR_UNSUPPORTED, "fused recompute: BF16 maps of 32x32 or 64x64 only");
    if (n < 1) return DRC_OK;
    FusedArgs a = fused_args(h, n);
    a.save[1] = (char*)h2;
    a.save[2] = (char*)h3;
    a.save[3] = (char*)u3;
    a.save[4] = (char*)u2;
    const int grid = fused_forward_grid(h, n, H, W);
    const long tok = prof_begin(h, PROF_FUSED, s);
    drc_status st = (H == 64) ? launch_fused<64, 64, true>(a, grid, s) : launch_fused<32, 32, true>(a, grid, s);
    prof_end(h, tok, s);
    return st;
}
