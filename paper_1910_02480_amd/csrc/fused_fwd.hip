// Whole-network BF16 forward of the autoencoder (Sec. 4.3, Fig. 3 layout as
// configured: 3x3 stride-2 encoder 7->32->64->128 with ReLU, mirrored
// stride-2 transposed-convolution decoder with skip concatenation, linear
// 3-channel output), one map per workgroup pass, every activation of the
// map resident in LDS.
//
// The layer path moves every activation through HBM (about 690 KB per 64x64
// map in BF16 with FP32 input and output); here a map costs its FP32 input
// (7 channels) and output (3 channels), plus whatever activations a
// training forward asks to keep.
//
// LDS plan for an H x W map (bytes, BF16 NHWC, 16-byte channel chunks XOR-
// swizzled by column against bank conflicts):
//   R0 [0, 16HW)           h1 (E1 -> D1); u2 of the recompute kernel
//   R1 [16HW, 24HW)        h2 (E2 -> D2)
//   R2 [24HW, 32HW)        u3 (D3 -> D2)
//   R3 [32HW, ...)         h3 (E3 -> D3), then a ring of 9 u2 rows (D2 -> D1)
//   R1+R2                  x as BF16, 8 channels (staging -> E1)
//   then 256 bytes of zeros, read by taps that fall outside the map.
// 146 KB at 64x64 (one workgroup per CU), 41 KB at 32x32.
//
// Every GEMM uses the same weight values, K order and epilogue arithmetic as
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
    char* save[5];       // optional: h1 h2 h3 u3 u2 of every map, plain NHWC BF16 (null = not kept)
    int final_relu;
    const int32_t* roll;  // augmentation of the input (AUG kernels): per-map column roll and mirror flag
    const int32_t* flip;
};

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
        for (int e = 0; e < 4; ++e) v[e] = drc::relu(v[e]);
    }
    uint2 w;
    w.x = pack_bf16x2(v[0], v[1]);
    w.y = pack_bf16x2(v[2], v[3]);
    *(uint2*)(smem + region + loff<C, WI>(y, x, ch >> 3) + ((ch >> 2) & 1) * 8) = w;
}

__device__ __forceinline__ void mma(f4& acc, const uint4& a, const uint4& b) { Traits<P_BF16>::mma(acc, a, b); }

// Forward epilogue: bias + ReLU, BF16 into an LDS tensor of C channels, WO wide.
// Epilogue interface: prefetch(pre, m, ch, y, x) at the start of a tile
// (global inputs of the epilogue, in flight during the tile's MFMAs), then
// operator()(pre, m, ch, y, x, acc, bias) after the K loop.
template <int C, int WO>
struct LdsOut {
    char* smem;
    int region;
    struct Pre {};
    __device__ __forceinline__ void prefetch(Pre&, int, int, int, int) const {}
    __device__ __forceinline__ void operator()(const Pre&, int, int ch, int y, int x, const f4& acc,
                                               const float* bias) const {
        lds_store4<C, WO>(smem, region, y, x, ch, acc, bias, true);
    }
};

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
                o.x = pack_bf16x2(f[7 * px + 0], f[7 * px + 1]);
                o.y = pack_bf16x2(f[7 * px + 2], f[7 * px + 3]);
                o.z = pack_bf16x2(f[7 * px + 4], f[7 * px + 5]);
                o.w = pack_bf16x2(f[7 * px + 6], 0.0f);
                *(uint4*)(smem + xs + (4 * q + px) * 16) = o;
            }
        }
    }
}

// stage_x for an augmented map (a rotation / mirror of the input, see
// AugMap): each thread gathers whole source pixels of a row (7 floats) and
// turns their normals; the BF16 packing is stage_x's.
template <int H, int W>
__device__ __forceinline__ void stage_x_aug(char* smem, int xs, const float* xm, const AugMap& am) {
    for (int p = opaque_tid(); p < H * W; p += FT) {
        const int row = (int)((unsigned)p / W), u = (int)((unsigned)p % W);
        const float* src = xm + ((long)row * W + aug_src_col(am, u, W)) * 7;
        float f[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) f[c] = src[c];
        aug_normal(am, f[3], f[4]);
        uint4 o;
        o.x = pack_bf16x2(f[0], f[1]);
        o.y = pack_bf16x2(f[2], f[3]);
        o.z = pack_bf16x2(f[4], f[5]);
        o.w = pack_bf16x2(f[6], 0.0f);
        *(uint4*)(smem + xs + p * 16) = o;
    }
}

// The next map's input, staged while the decoder runs. After D2 band b has
// read them, rows [4b, 4b + 4) of h2 (region R1) and of u3 (region R2) are
// dead; the x staging region R1 + R2 holds x row r at 16 W r bytes, so those
// rows free x rows [8b, 8b + 8) and [H/2 + 8b, H/2 + 8b + 8). A piece is
// those 16 rows; each thread carries a pair of pixels (56 bytes of float32)
// from before D2 band b until its rows are free.
struct XPiece {
    float2 v[7];
};
template <int H, int W>
__device__ __forceinline__ bool x_piece_pair(int band, int& row, int& col) {
    constexpr int NPAIR = 8 * W;  // pixel pairs of a piece (16 rows of W)
    const int t = opaque_tid();
    const int q = 2 * t, r = q / W;
    col = q % W;
    row = r < 8 ? 8 * band + r : H / 2 + 8 * band + (r - 8);
    return NPAIR % FT == 0 || t < NPAIR;
}
template <int H, int W>
__device__ __forceinline__ void x_piece_load(XPiece& xp, const float* xm, int band) {
    int row, col;
    if (x_piece_pair<H, W>(band, row, col)) {
        const float2* src = (const float2*)(xm + ((long)row * W + col) * 7);
#pragma unroll
        for (int k = 0; k < 7; ++k) xp.v[k] = src[k];
    }
}
template <int H, int W>
__device__ __forceinline__ void x_piece_store(char* smem, int xs, const XPiece& xp, int band) {
    int row, col;
    if (x_piece_pair<H, W>(band, row, col)) {
        const float* f = (const float*)xp.v;
#pragma unroll
        for (int px = 0; px < 2; ++px) {
            uint4 o;
            o.x = pack_bf16x2(f[7 * px + 0], f[7 * px + 1]);
            o.y = pack_bf16x2(f[7 * px + 2], f[7 * px + 3]);
            o.z = pack_bf16x2(f[7 * px + 4], f[7 * px + 5]);
            o.w = pack_bf16x2(f[7 * px + 6], 0.0f);
            *(uint4*)(smem + xs + (row * W + col + px) * 16) = o;
        }
    }
}

// The x pieces of an augmented map: the two pixels' sources are gathered
// separately; their normals are turned when the piece is stored.
template <int H, int W>
__device__ __forceinline__ void x_piece_load_aug(XPiece& xp, const float* xm, int band, const AugMap& am) {
    int row, col;
    if (x_piece_pair<H, W>(band, row, col)) {
        float* f = (float*)xp.v;
#pragma unroll
        for (int px = 0; px < 2; ++px) {
            const float* src = xm + ((long)row * W + aug_src_col(am, col + px, W)) * 7;
#pragma unroll
            for (int c = 0; c < 7; ++c) f[7 * px + c] = src[c];
        }
    }
}
template <int H, int W>
__device__ __forceinline__ void x_piece_store_aug(char* smem, int xs, XPiece& xp, int band, const AugMap& am) {
    float* f = (float*)xp.v;
    aug_normal(am, f[3], f[4]);
    aug_normal(am, f[10], f[11]);
    x_piece_store<H, W>(smem, xs, xp, band);
}

// Stride-2 3x3 convolution, LDS -> LDS, bias + ReLU (E1, E2, E3). Weights:
// the layer pack [COUT][KSTEPS*32] (k = tap * CIN + c) in fragment order. Wave w owns the row blocks of group
// w % TR for the whole layer and loads their weights (its A panel) into
// registers once; it then walks the pixel tiles w / TR, w / TR + FW / TR, ...
// (NPW blocks of 16 consecutive output pixels each). Taps that fall outside
// the map read the zero block at zoff.
template <int HI, int WI, int CIN, int COUT, int MT, int NPW, class Epi>
__device__ __forceinline__ void conv_phase(char* smem, int in, int zoff, const uint16_t* wp, const float* bias_g,
                                           const Epi& epi) {
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
        for (int e = 0; e < 4; ++e) bias[m][e] = bias_g ? bg[(tr * MT + m) * 16 + g * 4 + e] : 0.0f;
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
            oy[p] = (int)((unsigned)pix / WO);
            ox[p] = (int)((unsigned)pix % WO);
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
                    // a pixel block is one output row here: the top taps of row oy + 1
                    // are the bottom taps of row oy, so the same offsets (and loads) serve
                    if constexpr (WO == 16)
                        if (p > 0) off[p][kw] = off[p - 1][6 + kw];
                }
            }
        }
        typename Epi::Pre pre[MT][NPW];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int p = 0; p < NPW; ++p) epi.prefetch(pre[m][p], m, (tr * MT + m) * 16 + g * 4, oy[p], ox[p]);
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
                epi(pre[m][p], m, ch, oy[p], ox[p], acc[m][p], bias[m]);
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
// Weights and biases a wave keeps in registers for a transposed-convolution
// layer: blocks of its set (5 or 4) for its MT row blocks, every K step.
template <int KSN, int MT>
struct PairsPanel {
    uint4 A[KSN][5][MT];
    float bias[MT][4];
};

template <int COUT, int CIN, int MT>
__device__ __forceinline__ void pairs_panel_load(PairsPanel<CIN / 32, MT>& P, const uint16_t* wp,
                                                 const float* bias_g, int tr, int set) {
    constexpr int KSN = CIN / 32;
    const int lane = opaque_tid() & 63;
    const int g = lane >> 4;
    const uint16_t* w = opaque(wp);
    const int q0 = set ? 5 : 0, nq = set ? 4 : 5;
#pragma unroll
    for (int ks = 0; ks < KSN; ++ks)
#pragma unroll
        for (int q = 0; q < 5; ++q)
#pragma unroll
            for (int m = 0; m < MT; ++m)
                if (q < nq)
                    P.A[ks][q][m] =
                        *(const uint4*)(w + ((size_t)(((q0 + q) * (COUT / 16) + tr * MT + m) * KSN + ks) * 64 + lane) * 8);
    const float* bg = opaque(bias_g);
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) P.bias[m][e] = bias_g ? bg[(tr * MT + m) * 16 + g * 4 + e] : 0.0f;
}

// IR0 / IR1 > 0: source 0 / 1 is a ring of that many rows in LDS (input row
// r at slot r % IR); 0: the whole tensor, row r at slot r.
template <int HI, int WI, int C0, int C1, int COUT, int MT, int NPW, int SET, int NPB, int ORING, class Epi,
          int IR0 = 0, int IR1 = 0>
__device__ __forceinline__ void pairs_tiles(const PairsPanel<(C0 + C1) / 32, MT>& P, char* smem, int in0, int in1,
                                            int zoff, int tr, int tp0, int tp_step, int pix0, const Epi& epi) {
    constexpr int CIN = C0 + C1, KSN = CIN / 32;
    constexpr int WO = 2 * WI;
    constexpr int TP = NPB / NPW;
    constexpr int ROW = WI * C0 * 2;
    constexpr int NSRC = C1 > 0 ? 2 : 1;
    constexpr int Q0 = SET ? 5 : 0, NQ = SET ? 4 : 5;   // weight blocks of the set
    constexpr int PH0 = SET ? 3 : 0, NPH = SET ? 1 : 3; // its phases
    constexpr int NNB = SET ? 4 : 3;                    // neighbours it reads
    const int lane = opaque_tid() & 63;
    const int g = lane >> 4, r16 = lane & 15;
    for (int tp = tp0; tp < TP; tp += tp_step) {
        int ia[NPW], ib[NPW];
        int off[NPW][NSRC][4];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = pix0 + (tp * NPW + p) * 16 + r16;
            ia[p] = (int)((unsigned)pix / WI);
            ib[p] = (int)((unsigned)pix % WI);
            const bool down = ia[p] + 1 < HI, right = ib[p] + 1 < WI;
#pragma unroll
            for (int s = 0; s < NSRC; ++s)
#pragma unroll
                for (int dj = 0; dj < 2; ++dj) {
                    constexpr int IR = 0;
                    const int ir = s ? IR1 : IR0;
                    int b, bd;
                    if (ir == IR) {
                        b = (s ? in1 : in0) + loff<C0, WI>(ia[p], ib[p] + dj, g);
                        bd = b + ROW;
                    } else {
                        const int c = (s ? in1 : in0) + loff<C0, WI>(0, ib[p] + dj, g);
                        b = c + (int)((unsigned)ia[p] % (unsigned)(ir > 0 ? ir : 1)) * ROW;
                        bd = c + (int)((unsigned)(ia[p] + 1) % (unsigned)(ir > 0 ? ir : 1)) * ROW;
                    }
                    off[p][s][dj] = (dj && !right) ? zoff : b;
                    off[p][s][2 + dj] = ((dj && !right) || !down) ? zoff : bd;
                    // a pixel block is one input row here: its upper neighbours are the
                    // lower neighbours of the block above, so the same offsets (and loads) serve
                    if constexpr (WI == 16)
                        if (p > 0) off[p][s][dj] = off[p - 1][s][2 + dj];
                }
        }
        // output row of phase PP (or its slot in a ring of ORING rows) and column
        auto orow_of = [&](int p, int PP) {
            return ORING ? (2 * ia[p] + (PP >> 1)) % (ORING > 0 ? ORING : 1) : 2 * ia[p] + (PP >> 1);
        };
        typename Epi::Pre pre[NPH][MT][NPW];
#pragma unroll
        for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int p = 0; p < NPW; ++p)
                    epi.prefetch(pre[ph][m][p], m, (tr * MT + m) * 16 + g * 4, orow_of(p, PH0 + ph),
                                 2 * ib[p] + ((PH0 + ph) & 1));
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
                    for (int p = 0; p < NPW; ++p) mma(acc[ph][m][p], P.A[ks][q][m], bv[nb][p]);
            }
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int ch = (tr * MT + m) * 16 + g * 4;
#pragma unroll
            for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
                for (int p = 0; p < NPW; ++p) {
                    const int PP = PH0 + ph;
                    epi(pre[ph][m][p], m, ch, orow_of(p, PP), 2 * ib[p] + (PP & 1), acc[ph][m][p], P.bias[m]);
                }
        }
    }
}

// Work split of a transposed-convolution layer: 2 * TR groups (row-block
// group x set), rotated by workgroup so that CUs start on different weights.
template <int HI, int WI, int C0, int C1, int COUT, int MT, int NPW, class Epi>
__device__ __forceinline__ void pairs_phase(char* smem, int in0, int in1, int zoff, const uint16_t* wp,
                                            const float* bias_g, const Epi& epi) {
    constexpr int NPB = HI * WI / 16, ORING = 0;
    const int pix0 = 0;
    constexpr int RB = COUT / 16, TR = RB / MT, NG = 2 * TR;
    static_assert(RB % MT == 0 && NPB % NPW == 0 && FW % NG == 0 && C0 % 32 == 0 && C1 % 32 == 0,
                  "tiles cover the layer");
    static_assert(C1 == 0 || C1 == C0, "both sources share one LDS layout");
    const int wave = opaque_tid() >> 6;
    const int gid = (wave + blockIdx.x) % NG;
    const int tr = gid >> 1, set = gid & 1;
    const int tp0 = wave / NG, step = FW / NG;
    PairsPanel<(C0 + C1) / 32, MT> P;
    pairs_panel_load<COUT, C0 + C1, MT>(P, wp, bias_g, tr, set);
    if (set == 0)
        pairs_tiles<HI, WI, C0, C1, COUT, MT, NPW, 0, NPB, ORING>(P, smem, in0, in1, zoff, tr, tp0, step, pix0, epi);
    else
        pairs_tiles<HI, WI, C0, C1, COUT, MT, NPW, 1, NPB, ORING>(P, smem, in0, in1, zoff, tr, tp0, step, pix0, epi);
}

// D1: transposed convolution [u2 | h1] (32 + 32 channels at HI x WI) -> 3
// channels, linear, float32 to global, for GEMM rows [row0, row0 + nrows).
// u2 row r is at row r % RING of its region when RING > 0. Merged rows
// r = phase * 3 + co (12 of 16 used), K = neighbour * 64 + c, pack [16][256]
// in fragment order.
struct D1Panel {
    uint4 a[8];
    float bias[4];
};

__device__ __forceinline__ void d1_panel_load(D1Panel& P, const uint16_t* wp, const float* bias_g) {
    const int lane = opaque_tid() & 63;
    const int g = lane >> 4;
    const uint16_t* w = opaque(wp);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) P.a[ks] = *(const uint4*)(w + ((size_t)ks * 64 + lane) * 8);
    const float* bg = opaque(bias_g);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = g * 4 + e;
        P.bias[e] = r < 12 ? bg[r % 3] : 0.0f;
    }
}

template <int HI, int WI, int NPW, int RING>
__device__ __forceinline__ void d1_phase(const D1Panel& P, char* smem, int u2, int h1, int zoff, float* ym,
                                         bool relu, int row0, int nrows) {
    constexpr int WO = 2 * WI, ROW = WI * 64;
    static_assert((WI / 16) % NPW == 0 || NPW == 1, "tiles cover whole rows");
    const int tid = opaque_tid();
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int TP = nrows * WI / 16 / NPW;
    for (int tp = wave; tp < TP; tp += FW) {
        int ia[NPW], ib[NPW];
        int ou[NPW][4], oh[NPW][4];  // byte offsets of the 4 neighbours in u2 and in h1
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = row0 * WI + (tp * NPW + p) * 16 + r16;
            ia[p] = (int)((unsigned)pix / WI);
            ib[p] = (int)((unsigned)pix % WI);
            const bool down = ia[p] + 1 < HI, right = ib[p] + 1 < WI;
            const int ru0 = RING ? ia[p] % (RING > 0 ? RING : 1) : ia[p];
            const int ru1 = RING ? (ia[p] + 1) % (RING > 0 ? RING : 1) : ia[p] + 1;
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
                const bool okr = !dj || right;
                const int cu = loff<32, WI>(0, ib[p] + dj, g);
                const int ch = loff<32, WI>(ia[p], ib[p] + dj, g);
                ou[p][dj] = okr ? u2 + ru0 * ROW + cu : zoff;
                ou[p][2 + dj] = (okr && down) ? u2 + ru1 * ROW + cu : zoff;
                oh[p][dj] = okr ? h1 + ch : zoff;
                oh[p][2 + dj] = (okr && down) ? h1 + ch + ROW : zoff;
            }
        }
        f4 acc[NPW];
#pragma unroll
        for (int p = 0; p < NPW; ++p) acc[p] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const int nb = ks >> 1;
#pragma unroll
            for (int p = 0; p < NPW; ++p)
                mma(acc[p], P.a[ks], lds16(smem, (ks & 1) ? oh[p][nb] : ou[p][nb]));
        }
#pragma unroll
        for (int p = 0; p < NPW; ++p)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = g * 4 + e;
                if (r >= 12) continue;
                const int ph = r / 3;
                const int opix = (2 * ia[p] + (ph >> 1)) * WO + 2 * ib[p] + (ph & 1);
                float v = acc[p][e] + P.bias[e];
                if (relu) v = drc::relu(v);
                ym[opix * 3 + (r - ph * 3)] = v;
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
        ((uint4*)dst)[i] = *(const uint4*)(smem + region + loff<C, WI>((int)((unsigned)pix / WI), (int)((unsigned)pix % WI), j));
    }
}
// Rows [row0, row0 + nrows) of a ring of RING rows (C channels, WI wide) to
// a plain NHWC tensor (dst = its row 0).
template <int C, int WI, int RING>
__device__ __forceinline__ void copy_rows_out(char* dst, const char* smem, int region, int row0, int nrows) {
    constexpr int CH = C / 8, PER_ROW = WI * CH;
    const int N = nrows * PER_ROW;
    for (int i = threadIdx.x; i < N; i += FT) {
        const int r = row0 + i / PER_ROW, rem = i % PER_ROW;
        const int x = rem / CH, j = rem - x * CH;
        ((uint4*)dst)[(long)row0 * PER_ROW + i] =
            *(const uint4*)(smem + region + (r % RING) * (WI * C * 2) + loff<C, WI>(0, x, j));
    }
}
template <int C, int HI, int WI>
__device__ __forceinline__ void copy_in(char* smem, int region, const char* src) {
    constexpr int CH = C / 8, N = HI * WI * CH;
    for (int i = threadIdx.x; i < N; i += FT) {
        const int pix = i / CH, j = i - pix * CH;
        *(uint4*)(smem + region + loff<C, WI>((int)((unsigned)pix / WI), (int)((unsigned)pix % WI), j)) = ((const uint4*)src)[i];
    }
}

// LDS layout of an H x W map (byte offsets).
template <int H, int W>
struct FusedLds {
    static constexpr int HW = H * W;
    static constexpr int R0 = 0, R1 = 16 * HW, R2 = 24 * HW, R3 = 32 * HW;
    static constexpr int BAND = 4;                      // input rows of D2 per band
    static constexpr int RING = 2 * BAND + 1;           // u2 rows kept for D1
    static constexpr int RING_BYTES = RING * (W / 2) * 64;
    static constexpr int ZO = (R3 + (RING_BYTES > 4 * HW ? RING_BYTES : 4 * HW) + 255) / 256 * 256;
    static constexpr int BYTES = ZO + kZeroBytes;
};

// MID = false: the whole network, x -> y. Every non-null save[k] receives
// that activation. D2 and D1 run in bands of 4 D2 input rows: a band's 8 u2
// rows go to a ring of 9 rows (in R3 after h3 is consumed) and D1 then
// consumes all u2 rows of the band but the last, whose lower neighbour comes
// with the next band (the last band takes all its rows); h1 stays in R0
// throughout.
// MID = true: the recompute of a training backward, h2 (read from save[1])
// -> h3, u3, u2 (written to save[2..4]); E1, E2 and D1 are skipped.
template <int H, int W, bool MID, bool AUG>
__global__ __launch_bounds__(FT) void cae_fused_forward_kernel(const FusedArgs a) {
    // static LDS: its address is a compile-time constant, so LDS offsets fold
    // into the instructions' immediate fields (a dynamic array's base is added
    // to every address at run time)
    __shared__ __align__(16) char smem[FusedLds<H, W>::BYTES];
    typedef FusedLds<H, W> L;
    constexpr int HW = H * W;
    constexpr int R0 = L::R0, R1 = L::R1, R2 = L::R2, R3 = L::R3, ZO = L::ZO;
    // tiles: a wave owns one group of row blocks (MT blocks of 16) per layer and
    // walks pixel tiles of NPW blocks; chosen so that 8 waves have work and
    // few waves load the same weights
    constexpr int E1N = (HW / 64) >= 8 * 4 * 2 ? 4 : 2;     // E1: 2 row blocks (one group), PB = HW/64
    constexpr int E2N = (HW / 256) >= 8 ? 4 : 1;            // E2: 4 groups of 1, PB = HW/256
    constexpr int E3N = (HW / 1024) >= 4 ? 4 : 1;           // E3: 8 groups of 1, PB = HW/1024
    constexpr int D3N = (HW / 1024) >= 4 ? 2 : 1;           // D3: 4 groups x 2 sets, PB = HW/1024
    constexpr int D2N = (HW / 256) >= 16 ? 2 : 1;           // D2 (whole layer): 2 groups x 2 sets, PB = HW/256
    constexpr int D2BPB = L::BAND * (W / 4) / 16;           // D2 pixel blocks per band
    constexpr int D2BN = D2BPB >= 4 ? 2 : 1;                // 2 waves per group share a band
    constexpr int D1N = (W / 2) >= 32 ? 2 : 1;              // D1: pixel blocks per tile (whole rows)
    constexpr int NBAND = (H / 4) / L::BAND;
    constexpr int HU = H / 2, WU = W / 2;                   // u2 size
    // per-map bytes of h1 h2 h3 u3 u2
    constexpr long B1 = 16L * HW, B2 = 8L * HW, B3 = 4L * HW, B4 = 8L * HW, B5 = 16L * HW;
    static_assert((H / 4) % L::BAND == 0, "whole bands");
    if (threadIdx.x < kZeroBytes / 16) *(uint4*)(smem + ZO + 16 * threadIdx.x) = uint4{0u, 0u, 0u, 0u};
    bool staged = false;  // x of map m already in LDS (staged during the previous map's decoder)
    for (int m = blockIdx.x; m < a.nmaps; m += gridDim.x) {
        if constexpr (!MID) {
            const float* xm = a.x + (a.x_off ? a.x_off[m] : (long)m * HW * 7);
            float* ym = a.y + (a.y_off ? a.y_off[m] : (long)m * HW * 3);
            const int mn = m + gridDim.x;  // this workgroup's next map
            const float* xn = mn < a.nmaps ? a.x + (a.x_off ? a.x_off[mn] : (long)mn * HW * 7) : nullptr;
            AugMap amn;  // augmentation of the next map
            if constexpr (AUG) amn = aug_map(a.roll, a.flip, xn ? mn : m, W);
            if (!staged) {
                if constexpr (AUG) stage_x_aug<H, W>(smem, R1, xm, aug_map(a.roll, a.flip, m, W));
                else stage_x<H, W>(smem, R1, xm);
            }
            __syncthreads();
            conv_phase<H, W, 8, 32, 2, E1N>(smem, R1, ZO, a.w[0], a.b[0], LdsOut<32, W / 2>{smem, R0});
            __syncthreads();
            if (a.save[0]) copy_out<32, H / 2, W / 2>(a.save[0] + m * B1, smem, R0);
            conv_phase<H / 2, W / 2, 32, 64, 1, E2N>(smem, R0, ZO, a.w[1], a.b[1], LdsOut<64, W / 4>{smem, R1});
            __syncthreads();
            if (a.save[1]) copy_out<64, H / 4, W / 4>(a.save[1] + m * B2, smem, R1);
            conv_phase<H / 4, W / 4, 64, 128, 1, E3N>(smem, R1, ZO, a.w[2], a.b[2], LdsOut<128, W / 8>{smem, R3});
            __syncthreads();
            if (a.save[2]) copy_out<128, H / 8, W / 8>(a.save[2] + m * B3, smem, R3);
            pairs_phase<H / 8, W / 8, 128, 0, 64, 1, D3N>(smem, R3, R3, ZO, a.w[3], a.b[3], LdsOut<64, W / 4>{smem, R2});
            __syncthreads();
            if (a.save[3]) copy_out<64, H / 4, W / 4>(a.save[3] + m * B4, smem, R2);
            {
                // D2's and D1's weights stay in registers across the bands
                constexpr int NG = 4;  // D2: 2 row blocks x 2 sets, one row block per group
                const int wave = opaque_tid() >> 6;
                const int gid = (wave + blockIdx.x) % NG;
                const int tr = gid >> 1, set = gid & 1;
                PairsPanel<4, 1> P2;
                pairs_panel_load<32, 128, 1>(P2, a.w[4], a.b[4], tr, set);
                D1Panel P1;
                d1_panel_load(P1, a.w[5], a.b[5]);
                static_assert(NBAND * 16 == H, "the x pieces of the bands cover the next map's input");
                for (int band = 0; band < NBAND; ++band) {
                    const int pix0 = band * L::BAND * (W / 4);
                    const LdsOut<32, W / 2> ring{smem, R3};
                    XPiece xp;
                    if (xn) {  // in flight during D2's MFMAs
                        if constexpr (AUG) x_piece_load_aug<H, W>(xp, xn, band, amn);
                        else x_piece_load<H, W>(xp, xn, band);
                    }
                    if (set == 0)
                        pairs_tiles<H / 4, W / 4, 64, 64, 32, 1, D2BN, 0, D2BPB, L::RING>(
                            P2, smem, R2, R1, ZO, tr, wave / NG, FW / NG, pix0, ring);
                    else
                        pairs_tiles<H / 4, W / 4, 64, 64, 32, 1, D2BN, 1, D2BPB, L::RING>(
                            P2, smem, R2, R1, ZO, tr, wave / NG, FW / NG, pix0, ring);
                    __syncthreads();
                    if (xn) {
                        if constexpr (AUG) x_piece_store_aug<H, W>(smem, R1, xp, band, amn);
                        else x_piece_store<H, W>(smem, R1, xp, band);
                    }
                    const int u0 = 2 * L::BAND * band;  // first u2 row of the band
                    if (a.save[4]) copy_rows_out<32, WU, L::RING>(a.save[4] + m * B5, smem, R3, u0, 2 * L::BAND);
                    // u2 rows [r0, r1): all rows of the band whose lower neighbour is
                    // known (the last band also takes the map's last row)
                    const int r0 = band ? u0 - 1 : 0;
                    const int r1 = band + 1 < NBAND ? u0 + 2 * L::BAND - 1 : HU;
                    d1_phase<HU, WU, D1N, L::RING>(P1, smem, R3, R0, ZO, ym, a.final_relu != 0, r0, r1 - r0);
                    __syncthreads();
                }
            }
            staged = xn != nullptr;
        } else {
            copy_in<64, H / 4, W / 4>(smem, R1, a.save[1] + m * B2);
            __syncthreads();
            conv_phase<H / 4, W / 4, 64, 128, 1, E3N>(smem, R1, ZO, a.w[2], a.b[2], LdsOut<128, W / 8>{smem, R3});
            __syncthreads();
            copy_out<128, H / 8, W / 8>(a.save[2] + m * B3, smem, R3);
            pairs_phase<H / 8, W / 8, 128, 0, 64, 1, D3N>(smem, R3, R3, ZO, a.w[3], a.b[3], LdsOut<64, W / 4>{smem, R2});
            __syncthreads();
            copy_out<64, H / 4, W / 4>(a.save[3] + m * B4, smem, R2);
            pairs_phase<H / 4, W / 4, 64, 64, 32, 1, D2N>(smem, R2, R1, ZO, a.w[4], a.b[4], LdsOut<32, W / 2>{smem, R0});
            __syncthreads();
            copy_out<32, H / 2, W / 2>(a.save[4] + m * B5, smem, R0);
            __syncthreads();
        }
    }
}

// ======================================================================
// E1, E2, E3, D3 and D2 of large maps (128 x 128) in one kernel, by bands
// of rows: x (float32) in; h1 (for D1), h2 (for D2) and u2 out; h3 and u3
// never leave LDS. One map per workgroup pass, in two sweeps over bands of
// two h3 rows (four h2 rows, eight h1 rows, sixteen x rows). Sweep 1: E1
// turns x rows 16j - 1 .. 16j + 15 (a ring of 17 rows as BF16, the next
// band's rows loaded during the MFMAs) into h1 rows 8j .. 8j + 7, written to
// HBM and to a ring of 9 rows; E2 turns h1 rows 8j - 1 .. 8j + 7 into h2
// rows 4j .. 4j + 3, written to HBM and to a ring of 5 h2 rows, from which
// E3 forms h3 rows 2j, 2j + 1 (h3 is kept whole, 64 KB). Sweep 2: D3 writes the four u3 rows of band j into a ring of 8
// rows (over the h1 ring), and D2 then turns the four u3 rows of band j - 1
// (with the next row, written by band j's D3, as their lower neighbours)
// and the same h2 rows (the ring, staged again from HBM) into eight u2
// rows, stored straight from the MFMA results. GEMMs and epilogues are the
// layer kernels', so h1, h2 and u2 are bitwise the layer path's.
//   RH3 [0, 256 H3 W3)  h3;  RXR x ring (17 rows of W x 8 ch);  RX h1 ring
//   (9 rows of W1 x 32 ch), then u3 ring (8 rows of W2 x 64 ch);  RH2 h2
//   ring (5 rows of W2 x 64 ch);  zeros.  154 KB at 128 x 128.

// Stride-2 3x3 convolution over a band of output pixel blocks (CIN >= 32),
// LDS -> epilogue, with the weights (MT row blocks of group tr, every K step)
// already in registers and the input a ring of IR rows (input row r at slot
// r % IR). Same taps, K order and epilogue as conv_phase.
template <int KSTEPS, int MT>
struct ConvPanel {
    uint4 A[KSTEPS][MT];
    float bias[MT][4];
};
template <int CIN, int MT>
__device__ __forceinline__ void conv_panel_load(ConvPanel<(9 * CIN + 31) / 32, MT>& P, const uint16_t* wp,
                                                const float* bias_g, int tr) {
    constexpr int KSTEPS = (9 * CIN + 31) / 32;
    const int lane = opaque_tid() & 63, g = lane >> 4;
    const uint16_t* w = opaque(wp);
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks)
#pragma unroll
        for (int m = 0; m < MT; ++m)
            P.A[ks][m] = *(const uint4*)(w + ((size_t)((tr * MT + m) * KSTEPS + ks) * 64 + lane) * 8);
    const float* bg = opaque(bias_g);
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) P.bias[m][e] = bg[(tr * MT + m) * 16 + g * 4 + e];
}
// E1 over a band of output blocks (CIN = 8: x staged as BF16, 16 bytes per
// pixel, no swizzle) from a ring of IR input rows, the weights already in
// registers: the lane group g takes tap 4 ks + g of K step ks, exactly as
// conv_phase does for CIN = 8.
template <int HI, int WI, int MT, int NPW, int NPB, int IR, class Epi>
__device__ __forceinline__ void conv8_tiles(const ConvPanel<3, MT>& P, char* smem, int in, int zoff, int tr, int tp0,
                                            int tp_step, int pix0, const Epi& epi) {
    constexpr int WO = WI / 2, KSTEPS = 3, ROW = WI * 16;
    constexpr int TP = NPB / NPW;
    static_assert(NPB % NPW == 0 && IR > 0, "band of whole tiles from a ring");
    const int lane = opaque_tid() & 63;
    const int g = lane >> 4, r16 = lane & 15;
    for (int tp = tp0; tp < TP; tp += tp_step) {
        int oy[NPW], ox[NPW], off[NPW][KSTEPS];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = pix0 + (tp * NPW + p) * 16 + r16;
            oy[p] = (int)((unsigned)pix / WO);
            ox[p] = (int)((unsigned)pix % WO);
            const bool top = oy[p] > 0, left = ox[p] > 0;
#pragma unroll
            for (int ks = 0; ks < KSTEPS; ++ks) {
                const int t = ks * 4 + g, kh = t / 3, kw = t - (t / 3) * 3;
                const bool ok = t < 9 && (top || kh != 0) && (left || kw != 0);
                const int r = 2 * oy[p] - 1 + kh, c = 2 * ox[p] - 1 + kw;
                off[p][ks] = ok ? in + (int)((unsigned)r % (unsigned)IR) * ROW + c * 16 : zoff;
            }
        }
        typename Epi::Pre pre[MT][NPW];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int p = 0; p < NPW; ++p) epi.prefetch(pre[m][p], m, (tr * MT + m) * 16 + g * 4, oy[p], ox[p]);
        f4 acc[MT][NPW];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int p = 0; p < NPW; ++p) acc[m][p] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            uint4 b[NPW];
#pragma unroll
            for (int p = 0; p < NPW; ++p) b[p] = lds16(smem, off[p][ks]);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int p = 0; p < NPW; ++p) mma(acc[m][p], P.A[ks][m], b[p]);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int ch = (tr * MT + m) * 16 + g * 4;
#pragma unroll
            for (int p = 0; p < NPW; ++p) epi(pre[m][p], m, ch, oy[p], ox[p], acc[m][p], P.bias[m]);
        }
    }
}

template <int HI, int WI, int CIN, int MT, int NPW, int NPB, int IR, class Epi>
__device__ __forceinline__ void conv_tiles(const ConvPanel<(9 * CIN + 31) / 32, MT>& P, char* smem, int in,
                                           int zoff, int tr, int tp0, int tp_step, int pix0, const Epi& epi) {
    constexpr int WO = WI / 2;
    constexpr int KSTEPS = (9 * CIN + 31) / 32;
    constexpr int ROW = WI * CIN * 2;
    constexpr int TP = NPB / NPW;
    static_assert(CIN >= 32 && NPB % NPW == 0 && IR > 0, "band of whole tiles from a ring");
    const int lane = opaque_tid() & 63;
    const int g = lane >> 4, r16 = lane & 15;
    for (int tp = tp0; tp < TP; tp += tp_step) {
        int oy[NPW], ox[NPW];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = pix0 + (tp * NPW + p) * 16 + r16;
            oy[p] = (int)((unsigned)pix / WO);
            ox[p] = (int)((unsigned)pix % WO);
        }
        int off[NPW][9];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const bool top = oy[p] > 0, left = ox[p] > 0;
#pragma unroll
            for (int kw = 0; kw < 3; ++kw) {
                const int c = in + loff<CIN, WI>(0, 2 * ox[p] + kw - 1, g);
#pragma unroll
                for (int kh = 0; kh < 3; ++kh) {
                    const int r = 2 * oy[p] - 1 + kh;
                    off[p][kh * 3 + kw] = ((kh == 0 && !top) || (kw == 0 && !left))
                                              ? zoff
                                              : c + (int)((unsigned)r % (unsigned)IR) * ROW;
                }
                if constexpr (WO == 16)
                    if (p > 0) off[p][kw] = off[p - 1][6 + kw];
            }
        }
        typename Epi::Pre pre[MT][NPW];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int p = 0; p < NPW; ++p) epi.prefetch(pre[m][p], m, (tr * MT + m) * 16 + g * 4, oy[p], ox[p]);
        f4 acc[MT][NPW];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int p = 0; p < NPW; ++p) acc[m][p] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            uint4 b[NPW];
            const int t = ks * 32 / CIN, c0 = ks * 32 % CIN;
#pragma unroll
            for (int p = 0; p < NPW; ++p) b[p] = lds16(smem, off[p][t] ^ (c0 / 8 * 16));
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int p = 0; p < NPW; ++p) mma(acc[m][p], P.A[ks][m], b[p]);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int ch = (tr * MT + m) * 16 + g * 4;
#pragma unroll
            for (int p = 0; p < NPW; ++p) epi(pre[m][p], m, ch, oy[p], ox[p], acc[m][p], P.bias[m]);
        }
    }
}

// Epilogue: bias + ReLU, BF16 into a plain NHWC tensor (C channels, WO wide) in global memory.
template <int C, int WO>
struct GlobalOut {
    uint16_t* dst;
    struct Pre {};
    __device__ __forceinline__ void prefetch(Pre&, int, int, int, int) const {}
    __device__ __forceinline__ void operator()(const Pre&, int, int ch, int y, int x, const f4& acc,
                                               const float* bias) const {
        uint2 w;
        w.x = pack_bf16x2(drc::relu(acc.x + bias[0]), drc::relu(acc.y + bias[1]));
        w.y = pack_bf16x2(drc::relu(acc.z + bias[2]), drc::relu(acc.w + bias[3]));
        *(uint2*)(dst + ((long)y * WO + x) * C + ch) = w;
    }
};

// Epilogue: bias + ReLU, BF16, into a ring of RING rows in LDS (C channels,
// WO wide, column swizzle) and into a plain NHWC tensor in global memory.
template <int C, int WO, int RING>
struct RingGlobalOut {
    char* smem;
    int region;
    uint16_t* dst;
    struct Pre {};
    __device__ __forceinline__ void prefetch(Pre&, int, int, int, int) const {}
    __device__ __forceinline__ void operator()(const Pre&, int, int ch, int y, int x, const f4& acc,
                                               const float* bias) const {
        uint2 w;
        w.x = pack_bf16x2(drc::relu(acc.x + bias[0]), drc::relu(acc.y + bias[1]));
        w.y = pack_bf16x2(drc::relu(acc.z + bias[2]), drc::relu(acc.w + bias[3]));
        *(uint2*)(smem + region + (int)((unsigned)y % RING) * (WO * C * 2) + loff<C, WO>(0, x, ch >> 3) +
                  ((ch >> 2) & 1) * 8) = w;
        *(uint2*)(dst + ((long)y * WO + x) * C + ch) = w;
    }
};

// Rows [r0, r1) of a plain NHWC tensor (C channels, WI wide; src = its row 0)
// into slots r % RING of an LDS ring with the column swizzle.
template <int C, int WI, int RING>
__device__ __forceinline__ void copy_rows_in(char* smem, int region, const char* src, int r0, int r1) {
    constexpr int CH = C / 8, PER_ROW = WI * CH;
    const int N = (r1 - r0) * PER_ROW;
    for (int i = threadIdx.x; i < N; i += FT) {
        const int r = r0 + (int)((unsigned)i / PER_ROW), rem = (int)((unsigned)i % PER_ROW);
        const int x = rem / CH, j = rem - x * CH;
        *(uint4*)(smem + region + (int)((unsigned)r % RING) * (WI * C * 2) + loff<C, WI>(0, x, j)) =
            ((const uint4*)src)[(long)r0 * PER_ROW + i];
    }
}

// NR rows of a plain NHWC tensor (C channels, WI wide) carried in registers
// from their global loads (issued before the MFMAs of a band) to their LDS
// stores (after it), rows at or past `rows` skipped.
template <int C, int WI, int NR>
struct RowsPiece {
    static constexpr int PER_ROW = WI * C / 8, N = NR * PER_ROW, K = (N + FT - 1) / FT;
    static_assert(K <= 4, "at most four 16-byte chunks per thread");
    // named members of a native vector type, not an array of uint4: the
    // latter's copies are memcpys that keep the whole piece in memory (LDS or
    // scratch) rather than in registers
    typedef unsigned V4 __attribute__((ext_vector_type(4)));
    V4 v0, v1, v2, v3;
    template <int k>
    __device__ __forceinline__ V4& at() {
        if constexpr (k == 0) return v0;
        else if constexpr (k == 1) return v1;
        else if constexpr (k == 2) return v2;
        else return v3;
    }
    template <int k>
    __device__ __forceinline__ const V4& at() const {
        if constexpr (k == 0) return v0;
        else if constexpr (k == 1) return v1;
        else if constexpr (k == 2) return v2;
        else return v3;
    }
    // every lane loads (chunks past the tensor read its first chunk and are
    // never stored), so the loads carry no branches
    template <int k>
    __device__ __forceinline__ void load1(const char* src, int r0, int rows) {
        if constexpr (k < K) {
            const int i = (int)threadIdx.x + k * FT;
            const bool ok = (N % FT == 0 || i < N) && r0 + i / PER_ROW < rows;
            at<k>() = ((const V4*)src)[ok ? (long)r0 * PER_ROW + i : 0L];
        }
    }
    template <int RING, int k>
    __device__ __forceinline__ void store1(char* smem, int region, int r0, int rows) const {
        if constexpr (k < K) {
            const int i = (int)threadIdx.x + k * FT;
            const int r = r0 + i / PER_ROW, rem = i % PER_ROW;
            const int x = rem / (C / 8), j = rem - x * (C / 8);
            if ((N % FT == 0 || i < N) && r < rows)
                *(V4*)(smem + region + (int)((unsigned)r % RING) * (WI * C * 2) + loff<C, WI>(0, x, j)) = at<k>();
        }
    }
    __device__ __forceinline__ void load(const char* src, int r0, int rows) {
        load1<0>(src, r0, rows);
        load1<1>(src, r0, rows);
        load1<2>(src, r0, rows);
        load1<3>(src, r0, rows);
    }
    template <int RING>
    __device__ __forceinline__ void store(char* smem, int region, int r0, int rows) const {
        store1<RING, 0>(smem, region, r0, rows);
        store1<RING, 1>(smem, region, r0, rows);
        store1<RING, 2>(smem, region, r0, rows);
        store1<RING, 3>(smem, region, r0, rows);
    }
};

// NR rows of x (float32, 7 channels, WI wide) for the E1 ring: each thread
// carries 4 consecutive pixels (7 float4 = 28 floats) from their global
// loads, issued before the MFMAs of a band, to their LDS stores as BF16 with
// 8 channels (channel 7 = 0, 16 bytes per pixel) after it. Native vector
// members keep the piece in registers.
template <int WI, int NR>
struct XRowsPiece {
    typedef float F4 __attribute__((ext_vector_type(4)));
    static constexpr int Q = NR * WI / 4;  // pixel quads
    static_assert(Q == FT, "one quad per thread");
    F4 v0, v1, v2, v3, v4, v5, v6;
    __device__ __forceinline__ void load(const float* xm, int r0) {
        const F4* src = (const F4*)(xm + (long)r0 * WI * 7) + 7 * (int)threadIdx.x;
        v0 = src[0]; v1 = src[1]; v2 = src[2]; v3 = src[3]; v4 = src[4]; v5 = src[5]; v6 = src[6];
    }
    template <int RING>
    __device__ __forceinline__ void store(char* smem, int region, int r0) const {
        const float f[28] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w, v2.x, v2.y, v2.z, v2.w, v3.x, v3.y,
                             v3.z, v3.w, v4.x, v4.y, v4.z, v4.w, v5.x, v5.y, v5.z, v5.w, v6.x, v6.y, v6.z, v6.w};
        const int px = 4 * (int)threadIdx.x, r = r0 + px / WI, c = px % WI;
        char* row = smem + region + (int)((unsigned)r % RING) * (WI * 16);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint4 o;
            o.x = pack_bf16x2(f[7 * k + 0], f[7 * k + 1]);
            o.y = pack_bf16x2(f[7 * k + 2], f[7 * k + 3]);
            o.z = pack_bf16x2(f[7 * k + 4], f[7 * k + 5]);
            o.w = pack_bf16x2(f[7 * k + 6], 0.0f);
            *(uint4*)(row + (c + k) * 16) = o;
        }
    }
};

struct TailArgs {
    const float* x;      // maps of H x W x 7 float32
    const long* x_off;   // element offset of each map in x (null: packed)
    uint16_t* h1;        // [n][H/2][W/2][32]
    uint16_t* h2;        // [n][H/4][W/4][64]
    uint16_t* u2;        // [n][H/2][W/2][32]
    int nmaps;
    const uint16_t* w[5];  // E1, E2, E3, D3, D2 forward packs in fragment order
    const float* b[5];
};

template <int H, int W>
struct TailLds {
    static constexpr int H3 = H / 8, W3 = W / 8, W2 = W / 4, W1 = W / 2;
    static constexpr int RH3 = 0;
    static constexpr int RXR = H3 * W3 * 256;            // x ring: 17 rows of W pixels, 16 bytes each
    static constexpr int RX = RXR + 17 * W * 16;
    static constexpr int RX_BYTES = 9 * W1 * 64 > 8 * W2 * 128 ? 9 * W1 * 64 : 8 * W2 * 128;
    static constexpr int RH2 = RX + RX_BYTES;
    static constexpr int ZO = RH2 + 5 * W2 * 128;
    static constexpr int BYTES = ZO + kZeroBytes;
};

template <int H, int W>
__global__ __launch_bounds__(FT) void cae_fused_tail_kernel(const TailArgs a) {
    __shared__ __align__(16) char smem[TailLds<H, W>::BYTES];
    typedef TailLds<H, W> L;
    constexpr int H3 = H / 8, W3 = W / 8, H2 = H / 4, W2 = W / 4, H1 = H / 2, W1 = W / 2;
    constexpr int NB = H3 / 2;  // bands of two h3 rows = four h2 rows = eight h1 rows
    constexpr long S1 = (long)H1 * W1 * 32, S2 = (long)H2 * W2 * 64, SU = (long)(H / 2) * (W / 2) * 32;
    constexpr int E1PB = 8 * W1 / 16;  // output pixel blocks of an E1 band
    static_assert(W3 == 16 && (2 * W3) % 16 == 0 && (4 * W2) % 16 == 0, "D3 pixel blocks are h3 rows");
    if (threadIdx.x < kZeroBytes / 16) *(uint4*)(smem + L::ZO + 16 * threadIdx.x) = uint4{0u, 0u, 0u, 0u};
    constexpr int E2PB = 4 * W2 / 16;  // output pixel blocks of an E2 band
    constexpr int E3PB = 2 * W3 / 16;  // output pixel blocks of an E3 band
    constexpr int D3PB = 2 * W3 / 16;  // pixel blocks of a D3 band
    constexpr int D2PB = 4 * W2 / 16;  // pixel blocks of a D2 band
    for (int m = blockIdx.x; m < a.nmaps; m += gridDim.x) {
        const float* xm = a.x + (a.x_off ? a.x_off[m] : (long)m * H * W * 7);
        const char* h2m = (const char*)(a.h2 + m * S2);
        // E2: 4 row blocks, two waves each; E3: 8 row blocks, one per wave;
        // D3: 4 row blocks x 2 sets, one group per wave; D2: 2 row blocks x 2
        // sets, two waves per group. Formed per map from the opaque thread
        // index, so that the weight addresses are not hoisted out of the map
        // loop (they would be kept in registers).
        const int wave = opaque_tid() >> 6;
        const int tr2e = (wave + blockIdx.x) % 4;
        const int tre = (wave + blockIdx.x) % 8;
        const int g3 = (wave + blockIdx.x) % 8, tr3 = g3 >> 1, set3 = g3 & 1;
        const int g2 = (wave + blockIdx.x) % 4, tr2 = g2 >> 1, set2 = g2 & 1;
        {   // sweep 1: E1 (x -> h1, to the ring and to HBM), E2 (h1 -> h2, to
            // the ring and to HBM), E3 (h2 -> h3). Band j: E3 of band j - 1
            // and E1 of band j, then E2 of band j. Each layer's weight panel
            // is loaded from L2 where the layer runs, band after band: kept in
            // registers across the whole sweep, the three panels (132 VGPRs)
            // pushed the band loop into scratch spills, and each spill reload
            // waited for every HBM store still in flight.
            {
                XRowsPiece<W, 16> xq;
                xq.load(xm, 0);
                xq.template store<17>(smem, L::RXR, 0);
            }
            const RingGlobalOut<32, W1, 9> h1out{smem, L::RX, a.h1 + m * S1};
            const RingGlobalOut<64, W2, 5> h2out{smem, L::RH2, a.h2 + m * S2};
            const LdsOut<128, W3> h3out{smem, L::RH3};
            __syncthreads();
            for (int j = 0; j < NB; ++j) {
                ConvPanel<3, 2> P1e;
                conv_panel_load<8, 2>(P1e, a.w[0], a.b[0], 0);
                if (j > 0) {
                    ConvPanel<18, 1> PE;
                    conv_panel_load<64, 1>(PE, a.w[2], a.b[2], tre);
                    conv_tiles<H2, W2, 64, 1, 2, E3PB, 5>(PE, smem, L::RH2, L::ZO, tre, 0, 1, (j - 1) * E3PB * 16,
                                                          h3out);
                }
                XRowsPiece<W, 16> xq;  // x rows 16j + 16 .. 16j + 31 of the next band
                if (j + 1 < NB) xq.load(xm, 16 * j + 16);
                conv8_tiles<H, W, 2, 2, E1PB, 17>(P1e, smem, L::RXR, L::ZO, 0, wave, 8, j * E1PB * 16, h1out);
                ConvPanel<9, 1> P2e;
                conv_panel_load<32, 1>(P2e, a.w[1], a.b[1], tr2e);
                __syncthreads();
                // E1 is done with x rows 16j - 1 .. 16j + 14: their slots take the next band's rows
                if (j + 1 < NB) xq.template store<17>(smem, L::RXR, 16 * j + 16);
                conv_tiles<H1, W1, 32, 1, 2, E2PB, 9>(P2e, smem, L::RX, L::ZO, tr2e, wave / 4, 2, j * E2PB * 16,
                                                      h2out);
                __syncthreads();
            }
            {
                ConvPanel<18, 1> PE;
                conv_panel_load<64, 1>(PE, a.w[2], a.b[2], tre);
                conv_tiles<H2, W2, 64, 1, 2, E3PB, 5>(PE, smem, L::RH2, L::ZO, tre, 0, 1, (NB - 1) * E3PB * 16,
                                                      h3out);
            }
            __syncthreads();
        }
        PairsPanel<4, 1> P3, P2;
        pairs_panel_load<64, 128, 1>(P3, a.w[3], a.b[3], tr3, set3);
        pairs_panel_load<32, 128, 1>(P2, a.w[4], a.b[4], tr2, set2);
        copy_rows_in<64, W2, 5>(smem, L::RH2, h2m, 0, 5);
        const LdsOut<64, W2> u3ring{smem, L::RX};
        const GlobalOut<32, W / 2> u2out{a.u2 + m * SU};
        __syncthreads();
        for (int j = 0; j <= NB; ++j) {
            // D3 band j: h3 rows [2j, 2j + 2) -> u3 rows [4j, 4j + 4)
            if (j < NB) {
                if (set3 == 0)
                    pairs_tiles<H3, W3, 128, 0, 64, 1, 2, 0, D3PB, 8>(P3, smem, L::RH3, L::RH3, L::ZO, tr3, 0, 1,
                                                                     j * D3PB * 16, u3ring);
                else
                    pairs_tiles<H3, W3, 128, 0, 64, 1, 2, 1, D3PB, 8>(P3, smem, L::RH3, L::RH3, L::ZO, tr3, 0, 1,
                                                                     j * D3PB * 16, u3ring);
            }
            __syncthreads();
            if (j == 0) continue;
            // D2 band j - 1: [u3 | h2] rows [4j - 4, 4j) -> u2 rows [8j - 8, 8j)
            const int jb = j - 1;
            if (set2 == 0)
                pairs_tiles<H2, W2, 64, 64, 32, 1, 1, 0, D2PB, 0, GlobalOut<32, W / 2>, 8, 5>(
                    P2, smem, L::RX, L::RH2, L::ZO, tr2, wave / 4, 2, jb * D2PB * 16, u2out);
            else
                pairs_tiles<H2, W2, 64, 64, 32, 1, 1, 1, D2PB, 0, GlobalOut<32, W / 2>, 8, 5>(
                    P2, smem, L::RX, L::RH2, L::ZO, tr2, wave / 4, 2, jb * D2PB * 16, u2out);
            __syncthreads();
            // h2 rows 4j + 1 .. 4j + 4 of D2 band j (row 4j is already in the ring)
            if (j < NB) copy_rows_in<64, W2, 5>(smem, L::RH2, h2m, 4 * j + 1, 4 * j + 5 < H2 ? 4 * j + 5 : H2);
        }
    }
}

template <int H, int W>
drc_status launch_tail(const TailArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((cae_fused_tail_kernel<H, W>), dim3(grid), dim3(FT), 0, s, a);
    return check_launch("fused tail");
}

// ======================================================================
// Data-gradient chain of the training backward (Sec. 4.3), one map per
// workgroup pass: dy -> D1^T -> D2^T
// -> D3^T -> E3^T -> E2^T, each a stride-2 (transposed) convolution with the
// layer's transposed weights, the ReLU masks of the saved activations and
// the skip-gradient sums applied in the epilogues. Every output gradient the
// weight gradients need (dz_u2, dz_u3, dz_h3, dz_h2, dz_h1) and the skip
// gradient dh1s go to HBM; the chain's inputs stay in LDS:
//   RA [0, 16HW): dy as BF16 (8 channels), then dz_u3 [0, 8HW) and dh2s [8HW, 16HW),
//     then dh1s (staged from HBM for E2^T's epilogue)
//   RB [16HW, 32HW): dz_u2, then dz_h3 [16HW, 20HW) and dz_h2 [20HW, 28HW)
//   zeros at 32HW.
// K order, rounding and epilogue order (add, then mask) are the layer
// kernels', so the results are bitwise equal to the layer path.
struct GSeg {
    int region;            // LDS tensor receiving the value (< 0: none)
    uint16_t* gdst;        // global tensor of the map (plain NHWC; null: none)
    const uint16_t* mask;  // ReLU output of the layer below (value kept where > 0; null: none)
    const uint16_t* gadd;  // global tensor added first (null: none)
    int ladd;              // LDS tensor added first (< 0: none)
};

constexpr GSeg kNoSeg = {-1, nullptr, nullptr, nullptr, -1};
constexpr int kBiasSlots = 323;  // biases of E1 E2 E3 D3 D2 D1 at 0, 32, 96, 224, 288, 320

__device__ __forceinline__ void bf16x4_to_f32(uint2 w, float (&o)[4]) {
    o[0] = bf16_to_f32((uint16_t)(w.x & 0xffffu));
    o[1] = bf16_to_f32((uint16_t)(w.x >> 16));
    o[2] = bf16_to_f32((uint16_t)(w.y & 0xffffu));
    o[3] = bf16_to_f32((uint16_t)(w.y >> 16));
}

// Global epilogue inputs of one 4-channel store, fetched ahead of the tile.
struct GradPre {
    uint2 mk, ad;
};

template <int C, int WO>
__device__ __forceinline__ void grad_prefetch(const GSeg& sg, int lc, int y, int x, GradPre& pr) {
    const long pix = (long)y * WO + x;
    if (sg.mask) pr.mk = *(const uint2*)(sg.mask + pix * C + lc);
    if (sg.gadd) pr.ad = *(const uint2*)(sg.gadd + pix * C + lc);
}

template <int C, int WO>
__device__ __forceinline__ void grad_store(char* smem, const GSeg& sg, const GradPre& pr, int lc, int y, int x,
                                           float (&v)[4], float* bsum) {
    const long pix = (long)y * WO + x;
    const int loffs = loff<C, WO>(y, x, lc >> 3) + ((lc >> 2) & 1) * 8;
    if (sg.gadd) {
        float ad[4];
        bf16x4_to_f32(pr.ad, ad);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] += ad[e];
    }
    if (sg.ladd >= 0) {
        float ad[4];
        bf16x4_to_f32(*(const uint2*)(smem + sg.ladd + loffs), ad);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] += ad[e];
    }
    if (sg.mask) {
        float mk[4];
        bf16x4_to_f32(pr.mk, mk);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (mk[e] > 0.0f) ? v[e] : 0.0f;
    }
    uint2 w;
    w.x = pack_bf16x2(v[0], v[1]);
    w.y = pack_bf16x2(v[2], v[3]);
    if (sg.region >= 0) *(uint2*)(smem + sg.region + loffs) = w;
    if (sg.gdst) *(uint2*)(sg.gdst + pix * C + lc) = w;
    if (bsum) {  // bias gradient: column sums of the stored (rounded) values
        float r[4];
        bf16x4_to_f32(w, r);
#pragma unroll
        for (int e = 0; e < 4; ++e) bsum[e] += r[e];
    }
}

// Epilogue of a data-gradient GEMM whose rows are [segment 0 (C0 channels) |
// segment 1 (C1 channels)], WO pixels per output row.
// bsum (optional): per-lane sums of segment 0's stored values, 4 per row
// block m of the wave (the bias gradient of the layer that produced them).
template <int C0, int C1, int WO>
struct GradOut {
    char* smem;
    GSeg s0, s1;
    float* bsum;
    typedef GradPre Pre;
    __device__ __forceinline__ void prefetch(Pre& pr, int, int ch, int y, int x) const {
        if (C1 == 0 || ch < C0)
            grad_prefetch<C0, WO>(s0, ch, y, x, pr);
        else
            grad_prefetch<(C1 > 0 ? C1 : 8), WO>(s1, ch - C0, y, x, pr);
    }
    __device__ __forceinline__ void operator()(const Pre& pr, int m, int ch, int y, int x, const f4& acc,
                                               const float* bias) const {
        float v[4] = {acc.x + bias[0], acc.y + bias[1], acc.z + bias[2], acc.w + bias[3]};
        if (C1 == 0 || ch < C0)
            grad_store<C0, WO>(smem, s0, pr, ch, y, x, v, bsum ? bsum + 4 * m : nullptr);
        else
            grad_store<(C1 > 0 ? C1 : 8), WO>(smem, s1, pr, ch - C0, y, x, v, nullptr);
    }
};

// Adds a wave's per-lane column sums (4 per row block, MT row blocks of group
// tr) into red[wave][slot0 + channel] for the channels below nrows: first over
// the 16 lanes that share the channels (fixed butterfly), then one lane per
// group of 4 channels writes.
template <int MT>
__device__ __forceinline__ void dump_bias(float* red, int slot0, const float* bsum, int tr, int nrows) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
#pragma unroll
    for (int k = 0; k < 4 * MT; ++k) {
        float v = bsum[k];
        v += __shfl_xor(v, 1, 16);
        v += __shfl_xor(v, 2, 16);
        v += __shfl_xor(v, 4, 16);
        v += __shfl_xor(v, 8, 16);
        const int ch = (tr * MT + k / 4) * 16 + 4 * g + (k & 3);
        if (r16 == 0 && ch < nrows) red[wave * kBiasSlots + slot0 + ch] = v;
    }
}

struct DgradArgs {
    const float* dy;   // [n, H, W, 3] float32
    int nmaps;
    const uint16_t* w[6];  // backward-data packs in fragment order (layers 1..5 used)
    const uint16_t *u2, *u3, *h3, *h2, *h1;              // saved activations (masks)
    uint16_t *dz_u2, *dh1s, *dz_u3, *dz_h3, *dz_h2, *dz_h1;  // outputs
    float* bias_part;  // [workgroup][kBiasSlots] column sums (bias gradients before the batch sum)
};

// dy (float32, 3 channels) -> LDS as BF16 with 8 channels (3..7 = 0).
template <int H, int W>
__device__ __forceinline__ void stage_dy(char* smem, int xs, const float* dm, float (&bs)[3]) {
    constexpr int Q = H * W / 4;  // groups of 4 pixels = 12 floats = 3 float4
    const int tid = opaque_tid();
    for (int q = tid; q < Q; q += FT) {
        float4 v[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) v[k] = ((const float4*)dm)[q * 3 + k];
        const float* f = (const float*)v;
#pragma unroll
        for (int px = 0; px < 4; ++px)  // D1's bias gradient sums dy itself (float32)
#pragma unroll
            for (int c = 0; c < 3; ++c) bs[c] += f[3 * px + c];
#pragma unroll
        for (int px = 0; px < 4; ++px) {
            uint4 o;
            o.x = pack_bf16x2(f[3 * px + 0], f[3 * px + 1]);
            o.y = pack_bf16x2(f[3 * px + 2], 0.0f);
            o.z = 0u;
            o.w = 0u;
            *(uint4*)(smem + xs + (4 * q + px) * 16) = o;
        }
    }
}

template <int H, int W>
__global__ __launch_bounds__(FT) void cae_fused_dgrad_kernel(const DgradArgs a) {
    __shared__ __align__(16) char smem[32 * H * W + kZeroBytes];  // static: see the forward kernel
    constexpr int HW = H * W;
    constexpr int RA = 0, RB = 16 * HW, ZO = 32 * HW;
    constexpr long S1 = 8L * HW, S2 = 4L * HW, S3 = 2L * HW;  // elements per map at H/2, H/4, H/8
    constexpr int P3N = (HW / 256) >= 8 ? 4 : 2;
    constexpr int P4N = (HW / 1024) >= 4 ? 4 : 1;
    constexpr int P5N = (HW / 1024) >= 4 ? 2 : 1;
    constexpr int P6N = (HW / 256) >= 16 ? 2 : 1;
    if (threadIdx.x < kZeroBytes / 16) *(uint4*)(smem + ZO + 16 * threadIdx.x) = uint4{0u, 0u, 0u, 0u};
    // bias-gradient column sums over this workgroup's maps, per lane
    float bs_u2[8] = {}, bs_u3[8] = {}, bs_h3[4] = {}, bs_h2[4] = {}, bs_h1[4] = {}, bs_dy[3] = {};
    for (int m = blockIdx.x; m < a.nmaps; m += gridDim.x) {
        stage_dy<H, W>(smem, RA, a.dy + (long)m * HW * 3, bs_dy);
        __syncthreads();
        {   // D1^T: dy -> [dz_u2 (masked by u2) | dh1s]
            GradOut<32, 32, W / 2> e{smem, GSeg{RB, a.dz_u2 + m * S1, a.u2 + m * S1, nullptr, -1},
                                     GSeg{-1, a.dh1s + m * S1, nullptr, nullptr, -1}, bs_u2};
            conv_phase<H, W, 8, 64, 2, 4>(smem, RA, ZO, a.w[5], nullptr, e);
        }
        __syncthreads();
        {   // D2^T: dz_u2 -> [dz_u3 (masked by u3) | dh2s]
            GradOut<64, 64, W / 4> e{smem, GSeg{RA, a.dz_u3 + m * S2, a.u3 + m * S2, nullptr, -1},
                                     GSeg{RA + 8 * HW, nullptr, nullptr, nullptr, -1}, bs_u3};
            conv_phase<H / 2, W / 2, 32, 128, 2, P3N>(smem, RB, ZO, a.w[4], nullptr, e);
        }
        __syncthreads();
        {   // D3^T: dz_u3 -> dz_h3 (masked by h3)
            GradOut<128, 0, W / 8> e{smem, GSeg{RB, a.dz_h3 + m * S3, a.h3 + m * S3, nullptr, -1}, kNoSeg, bs_h3};
            conv_phase<H / 4, W / 4, 64, 128, 1, P4N>(smem, RA, ZO, a.w[3], nullptr, e);
        }
        __syncthreads();
        {   // E3^T: dz_h3 -> dz_h2 = (. + dh2s) masked by h2
            GradOut<64, 0, W / 4> e{smem, GSeg{RB + 4 * HW, a.dz_h2 + m * S2, a.h2 + m * S2, nullptr, RA + 8 * HW},
                                    kNoSeg, bs_h2};
            pairs_phase<H / 8, W / 8, 128, 0, 64, 1, P5N>(smem, RB, RB, ZO, a.w[2], nullptr, e);
        }
        __syncthreads();
        {   // E2^T: dz_h2 -> dz_h1 = (. + dh1s) masked by h1; dh1s is staged in RA first
            copy_in<32, H / 2, W / 2>(smem, RA, (const char*)(a.dh1s + m * S1));
            __syncthreads();
            GradOut<32, 0, W / 2> e{smem, GSeg{-1, a.dz_h1 + m * S1, a.h1 + m * S1, nullptr, RA}, kNoSeg,
                                    bs_h1};
            pairs_phase<H / 4, W / 4, 64, 0, 32, 1, P6N>(smem, RB + 4 * HW, RB + 4 * HW, ZO, a.w[1], nullptr, e);
        }
        __syncthreads();
    }
    // Per-workgroup bias partials: lanes -> red[wave][slot] (LDS) -> fixed-order sums over the waves.
    // The row-block group of each wave per layer is the one the phase functions used.
    float* red = (float*)smem;
    float* rdy = red + FW * kBiasSlots;
    for (int i = threadIdx.x; i < FW * kBiasSlots; i += FT) red[i] = 0.0f;
    __syncthreads();
    const int wave = threadIdx.x >> 6;
    dump_bias<2>(red, 288, bs_u2, (wave + blockIdx.x) % 2, 32);   // D2 bias: dz_u2 (rows 0-31 of D1^T)
    dump_bias<2>(red, 224, bs_u3, (wave + blockIdx.x) % 4, 64);   // D3 bias: dz_u3 (rows 0-63 of D2^T)
    dump_bias<1>(red, 96, bs_h3, (wave + blockIdx.x) % 8, 128);   // E3 bias: dz_h3
    dump_bias<1>(red, 32, bs_h2, ((wave + blockIdx.x) % 8) >> 1, 64);  // E2 bias: dz_h2 (pairs: group = 2 tr + set)
    dump_bias<1>(red, 0, bs_h1, ((wave + blockIdx.x) % 4) >> 1, 32);   // E1 bias: dz_h1
#pragma unroll
    for (int c = 0; c < 3; ++c) rdy[threadIdx.x * 3 + c] = bs_dy[c];
    __syncthreads();
    if (threadIdx.x < kBiasSlots) {
        const int c = threadIdx.x;
        float v = 0.0f;
        if (c < 320) {
            for (int w = 0; w < FW; ++w) v += red[w * kBiasSlots + c];
        } else {
            for (int t = 0; t < FT; ++t) v += rdy[t * 3 + (c - 320)];
        }
        a.bias_part[(long)blockIdx.x * kBiasSlots + c] = v;
    }
}

// Bias gradients from the per-workgroup partials: dparams[bias of layer l][i]
// = scale * (sum over workgroups, in order) of partial[.][slot(l) + i].
struct BiasFinalArgs {
    const float* part;
    int nrows;
    float scale;
    float* dparams;
    long boff[6];  // offsets of the six bias vectors in dparams
};
__global__ __launch_bounds__(256) void bias_final_kernel(const BiasFinalArgs a) {
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int r = threadIdx.x; r < a.nrows; r += 256) s += a.part[(long)r * kBiasSlots + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int l = c < 32 ? 0 : c < 96 ? 1 : c < 224 ? 2 : c < 288 ? 3 : c < 320 ? 4 : 5;
        const int s0[6] = {0, 32, 96, 224, 288, 320};
        a.dparams[a.boff[l] + (c - s0[l])] = red[0] * a.scale;
    }
}

template <int H, int W>
drc_status launch_dgrad(const DgradArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((cae_fused_dgrad_kernel<H, W>), dim3(grid), dim3(FT), 0, s, a);
    return check_launch("fused dgrad");
}

template <int H, int W, bool MID>
drc_status launch_fused(const FusedArgs& a, int grid, hipStream_t s) {
    if (!MID && a.roll)
        hipLaunchKernelGGL((cae_fused_forward_kernel<H, W, false, true>), dim3(grid), dim3(FT), 0, s, a);
    else
        hipLaunchKernelGGL((cae_fused_forward_kernel<H, W, MID, false>), dim3(grid), dim3(FT), 0, s, a);
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

// Map sizes whose D3 and D2 run fused (fused_tail).
bool fused_tail_size(int H, int W) { return H == 128 && W == 128; }

drc_status fused_tail(drc_cae* h, int n, int H, int W, const float* x, const long* x_off, void* h1, void* h2,
                      void* u2, hipStream_t s) {
    if (h->prec != P_BF16 || !fused_tail_size(H, W) || h->desc.pad_w != DRC_PAD_ZERO)
        return drc_fail(DRC_ERR_UNSUPPORTED, "fused tail: BF16 maps of 128x128 with zero padding only");
    if ((uintptr_t)x % 16 != 0) return drc_fail(DRC_ERR_INVALID_ARG, "fused tail: x is not 16-byte aligned");
    if (n < 1) return DRC_OK;
    TailArgs a;
    memset(&a, 0, sizeof a);
    a.x = x;
    a.x_off = x_off;
    a.h1 = (uint16_t*)h1;
    a.h2 = (uint16_t*)h2;
    a.u2 = (uint16_t*)u2;
    a.nmaps = n;
    for (int l = 0; l < 5; ++l) {
        a.w[l] = (const uint16_t*)h->wfrag[l];
        a.b[l] = h->bias + bias_slot(l);
    }
    // one workgroup per map: the dispatcher hands maps to CUs as they free
    // up, also to CUs that another stream's launch leaves idle
    const int grid = std::max(1, n);
    const long tok = prof_begin(h, PROF_FWD + 0, s);
    const drc_status st = launch_tail<128, 128>(a, grid, s);
    prof_end(h, tok, s);
    return st;
}

// Workgroups of one fused launch over n maps of H x W.
int fused_forward_grid(const drc_cae* h, int n, int H, int W) {
    const int per_cu = (H * W >= 4096) ? 1 : 2;
    return std::max(1, std::min(n, h->num_cu * per_cu));
}

// Scratch bytes of one fused launch: none (every activation stays on chip
// unless saved).
size_t fused_forward_scratch(const drc_cae*, int, int, int) { return 0; }

drc_status fused_forward(drc_cae* h, const float* x, float* y, int n, int H, int W, const long* x_off,
                         const long* y_off, void* scratch, size_t scratch_bytes, hipStream_t s,
                         char* const* save, const int32_t* roll, const int32_t* flip) {
    if (h->prec != P_BF16 || !fused_forward_size(H, W))
        return drc_fail(DRC_ERR_UNSUPPORTED, "fused forward: BF16 maps of 32x32 or 64x64 only");
    if ((roll != nullptr) != (flip != nullptr) || (roll && x_off))
        return drc_fail(DRC_ERR_INVALID_ARG, "fused forward: augmentation needs roll and flip and packed maps");
    if (n < 1) return DRC_OK;
    FusedArgs a = fused_args(h, n);
    a.roll = roll;
    a.flip = flip;
    if (save)
        for (int k = 0; k < 5; ++k) a.save[k] = save[k];
    (void)scratch_bytes;
    a.x = x;
    a.y = y;
    a.x_off = x_off;
    a.y_off = y_off;
    (void)scratch;
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

drc_status fused_dgrad(drc_cae* h, int n, int H, int W, const float* dy, const void* u2, const void* u3,
                       const void* h3, const void* h2, const void* h1, void* dz_u2, void* dh1s, void* dz_u3,
                       void* dz_h3, void* dz_h2, void* dz_h1, float* bias_part, size_t bias_part_bytes,
                       float* dparams, float gscale, hipStream_t s, GradFinal* defer) {
    if (h->prec != P_BF16 || !fused_forward_size(H, W))
        return drc_fail(DRC_ERR_UNSUPPORTED, "fused dgrad: BF16 maps of 32x32 or 64x64 only");
    if (n < 1) return DRC_OK;
    const int grid = fused_forward_grid(h, n, H, W);
    if ((size_t)grid * kBiasSlots * sizeof(float) > bias_part_bytes)
        return drc_fail(DRC_ERR_WORKSPACE, "fused dgrad: bias partials need %zu bytes",
                        (size_t)grid * kBiasSlots * sizeof(float));
    DgradArgs a;
    memset(&a, 0, sizeof a);
    a.dy = dy;
    a.nmaps = n;
    for (int l = 1; l < 6; ++l) a.w[l] = (const uint16_t*)h->wbfrag[l];
    a.u2 = (const uint16_t*)u2;
    a.u3 = (const uint16_t*)u3;
    a.h3 = (const uint16_t*)h3;
    a.h2 = (const uint16_t*)h2;
    a.h1 = (const uint16_t*)h1;
    a.dz_u2 = (uint16_t*)dz_u2;
    a.dh1s = (uint16_t*)dh1s;
    a.dz_u3 = (uint16_t*)dz_u3;
    a.dz_h3 = (uint16_t*)dz_h3;
    a.dz_h2 = (uint16_t*)dz_h2;
    a.dz_h1 = (uint16_t*)dz_h1;
    a.bias_part = bias_part;
    const long tok = prof_begin(h, PROF_FUSED_BWD, s);
    drc_status st = (H == 64) ? launch_dgrad<64, 64>(a, grid, s) : launch_dgrad<32, 32>(a, grid, s);
    prof_end(h, tok, s);
    if (st != DRC_OK) return st;
    if (defer) {
        static const int s0[7] = {0, 32, 96, 224, 288, 320, kBiasSlots};
        defer->bpart = bias_part;
        defer->bnrows = grid;
        defer->bslots = kBiasSlots;
        defer->bscale = gscale;
        defer->bdparams = dparams;
        for (int l = 0; l < 6; ++l) defer->boff[l] = layer_b_offset(l);
        for (int l = 0; l < 7; ++l) defer->bs0[l] = s0[l];
        return DRC_OK;
    }
    BiasFinalArgs b;
    b.part = bias_part;
    b.nrows = grid;
    b.scale = gscale;
    b.dparams = dparams;
    for (int l = 0; l < 6; ++l) b.boff[l] = layer_b_offset(l);
    const long tb = prof_begin(h, PROF_BIAS, s);
    hipLaunchKernelGGL(bias_final_kernel, dim3(kBiasSlots), dim3(256), 0, s, b);
    prof_end(h, tb, s);
    return check_launch("fused dgrad/bias");
}
