// Whole-network FP8 (OCP e4m3) forward of the autoencoder (Sec. 4.3; the
// FP8 inference form of this library: every layer GEMM on e4m3 operands
// with per-tensor scales and float32 accumulation), one map per workgroup
// pass with every activation of the map in LDS.
//
// The FP8 layer path moves each activation through HBM; here a map costs
// its float32 input and output only. With one byte per activation value a
// 64x64 map needs 80 KB of LDS, so two workgroups share a CU and one's
// input staging and barriers overlap the other's MFMAs.
//
// LDS plan for an H x W map (bytes; e4m3 NHWC, 16-byte channel chunks
// XOR-swizzled by column; x with 8 bytes per pixel):
//   R0 [0, 8HW)           h1 (E1 -> D1)
//   R1 [8HW, 16HW)        x (staging -> E1); then h2 [8HW, 12HW) (E2 -> D2),
//                         h3 [12HW, 14HW) (E3 -> D3), later the ring of
//                         u2 rows (D2 -> D1) at 12HW; a 256-byte zero block
//                         at the end of R1 (written after E1 has read x)
//   R2 [16HW, 20HW)       u3 (D3 -> D2)
// 80 KB at 64x64; at 32x32 the ring needs its own region after R2.
//
// Operands, K order, rounding and epilogue arithmetic are those of the FP8
// layer kernels (the band-staged E1 and D1, the generic convolution and the
// (phase, neighbour) transposed convolution), so the outputs are bitwise
// equal to the layer path:
//   E1: one K step of 128, lane group g holds taps 4g .. 4g+3 (8 bytes each);
//   E2: K steps of 128 = 4 taps of 32 channels, lane group g takes tap 4ks + g;
//   E3: K steps of 128 = 2 taps of 64 channels, lane group g takes tap
//       2ks + g/2, channels 32 (g % 2) .. + 32;
//   D3, D2: one K step per (phase, neighbour) block, lane group g takes
//       channels 32 g .. + 32 of [u3 | h2] (D2) or h3 (D3);
//   D1: rows (phase, channel), 2 K steps, lane group g of step ks takes
//       neighbour 2ks + g/2, channels 32 (g % 2) .. + 32 of [u2 | h1];
//   epilogue: v = acc * acc_scale + bias, ReLU, e4m3(v * scale of the output).
#include <hip/hip_runtime.h>
#include <string.h>

#include "drc_cae.h"
#include "common.h"
#include "conv_layer.h"
#include "internal.h"

using namespace drc;

namespace {

constexpr int NT = 256;      // threads per workgroup
constexpr int NW = NT / 64;  // waves
typedef Traits<P_FP8> TR;
typedef TR::V V;             // 32 bytes per lane

struct F8Args {
    const float* x;     // [.., H, W, 7] float32
    float* y;           // [.., H, W, 3] float32
    int nmaps;
    const long* x_off;  // element offset of each map (null: packed)
    const long* y_off;
    const uint8_t* w[6];  // FP8 layer packs, row-major ([9] blocks for D3, D2)
    int kstride[6];
    const float* b[6];
    float acc_scale[6];   // 1 / (input scale x weight scale)
    float qout[6];        // scale of the layer's stored output (E1..D2)
    float xscale;
    int final_relu;
};

__device__ __forceinline__ int otid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}
template <typename T>
__device__ __forceinline__ const T* opq(const T* p) {
    int z = 0;
    asm volatile("" : "+s"(z));
    return p + z;
}

// Byte offset of 16-byte chunk `ch` of pixel (y, x) in a tensor of C e4m3
// channels and rows of WI pixels; chunks XOR-swizzled by column.
template <int C, int WI>
__device__ __forceinline__ int l8(int y, int x, int ch) {
    constexpr int CH = C / 16;
    int s;
    if constexpr (CH == 2) s = (x >> 2) & 1;
    else if constexpr (CH == 4) s = (x >> 1) & 3;
    else s = x & 7;
    return (y * WI + x) * C + ((ch ^ s) & (CH - 1)) * 16;
}

// 32 bytes (two 16-byte chunks) as one MFMA operand.
__device__ __forceinline__ V ld32(const char* smem, int o0, int o1) {
    uint4 t[2];
    t[0] = *(const uint4*)(smem + o0);
    t[1] = *(const uint4*)(smem + o1);
    return __builtin_bit_cast(V, t);
}

__device__ __forceinline__ void mma8(f4& acc, const V& a, const V& b) { TR::mma(acc, a, b); }

// Stores channels [ch, ch+4) of an output pixel: v = acc * scale + bias, ReLU,
// e4m3(v * qout), 4 bytes at `off`.
__device__ __forceinline__ void st4(char* smem, int off, const f4& acc, float scale, const float* bias, float qout) {
    *(uint32_t*)(smem + off) = e4m3_act4(acc.x * scale + bias[0], acc.y * scale + bias[1], acc.z * scale + bias[2],
                                         acc.w * scale + bias[3], qout, true);
}

// x (float32, 7 channels) -> e4m3(x * s) with 8 channels (channel 7 = 0), 8
// bytes per pixel; 4 consecutive pixels (7 float4) per thread and pass.
template <int H, int W>
__device__ __forceinline__ void stage_x8(char* smem, int xs, const float* xm, float s) {
    constexpr int Q = H * W / 4;
    const int tid = otid();
#pragma unroll 2
    for (int q = tid; q < Q; q += NT) {
        float4 v[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) v[k] = ((const float4*)xm)[q * 7 + k];
        const float* f = (const float*)v;
#pragma unroll
        for (int px = 0; px < 4; ++px) {
            const float* c = f + 7 * px;
            uint2 o;
            o.x = e4m3_act4(c[0], c[1], c[2], c[3], s, false);
            o.y = e4m3_act4(c[4], c[5], c[6], 0.0f, s, false);
            *(uint2*)(smem + xs + (4 * q + px) * 8) = o;
        }
    }
}

// E1: stride-2 conv of x (8 channels, 8 bytes per pixel) -> h1 (32 channels).
template <int H, int W, int NPW>
__device__ __forceinline__ void e1_phase(char* smem, int xs, int h1, const F8Args& a) {
    constexpr int HO = H / 2, WO = W / 2, PB = HO * WO / 16, TP = PB / NPW;
    const int tid = otid();
    const int lane = tid & 63, wave = tid >> 6, g = lane >> 4, r16 = lane & 15;
    const uint8_t* w = opq(a.w[0]);
    const int ks0 = a.kstride[0];
    V A[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) A[m] = *(const V*)(w + (size_t)(16 * m + r16) * ks0 + 32 * g);
    float bias[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[m][e] = opq(a.b[0])[16 * m + 4 * g + e];
    for (int tp = wave; tp < TP; tp += NW) {
        f4 acc[2][NPW];
        V bv[NPW];
        int oy[NPW], ox[NPW];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = (tp * NPW + p) * 16 + r16;
            oy[p] = (int)((unsigned)pix / WO);
            ox[p] = (int)((unsigned)pix % WO);
            uint2 hh[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int t = 4 * g + s, kh = t / 3, kw = t - 3 * (t / 3);
                const int y = 2 * oy[p] + kh - 1, x = 2 * ox[p] + kw - 1;
                const bool ok = t < 9 && y >= 0 && x >= 0;
                const uint2 v = *(const uint2*)(smem + xs + ((ok ? y : 0) * W + (ok ? x : 0)) * 8);
                hh[s] = ok ? v : make_uint2(0u, 0u);
            }
            bv[p] = __builtin_bit_cast(V, hh);
#pragma unroll
            for (int m = 0; m < 2; ++m) acc[m][p] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int p = 0; p < NPW; ++p) mma8(acc[m][p], A[m], bv[p]);
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int p = 0; p < NPW; ++p)
                st4(smem, h1 + l8<32, WO>(oy[p], ox[p], m) + 4 * g, acc[m][p], a.acc_scale[0], bias[m], a.qout[0]);
    }
}

// Stride-2 conv, LDS -> LDS (E2: CIN 32 -> 64; E3: CIN 64 -> 128). Wave w
// owns the MT row blocks of group w % TR and walks pixel tiles of NPW blocks.
template <int L, int HI, int WI, int CIN, int COUT, int MT, int NPW>
__device__ __forceinline__ void conv_phase8(char* smem, int in, int out, int zo, const F8Args& a) {
    constexpr int HO = HI / 2, WO = WI / 2;
    constexpr int PB = HO * WO / 16, RB = COUT / 16, TR_ = RB / MT, TP = PB / NPW;
    constexpr int KSTEPS = (9 * CIN + 127) / 128;
    static_assert(RB % MT == 0 && PB % NPW == 0 && NW % TR_ == 0, "tiles cover the layer");
    const int tid = otid();
    const int lane = tid & 63, wave = tid >> 6, g = lane >> 4, r16 = lane & 15;
    const int tr = (wave + blockIdx.x) % TR_;
    const uint8_t* w = opq(a.w[L]);
    const int kst = a.kstride[L];
    V A[KSTEPS][MT];
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks)
#pragma unroll
        for (int m = 0; m < MT; ++m)
            A[ks][m] = *(const V*)(w + (size_t)((tr * MT + m) * 16 + r16) * kst + ks * 128 + 32 * g);
    float bias[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[m][e] = opq(a.b[L])[(tr * MT + m) * 16 + 4 * g + e];
    for (int tp = wave / TR_; tp < TP; tp += NW / TR_) {
        int oy[NPW], ox[NPW];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = (tp * NPW + p) * 16 + r16;
            oy[p] = (int)((unsigned)pix / WO);
            ox[p] = (int)((unsigned)pix % WO);
        }
        f4 acc[MT][NPW];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int p = 0; p < NPW; ++p) acc[m][p] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            // lane group g: tap t, channels [c, c + 32) (two chunks)
            const int k = ks * 128 + 32 * g;
            const int t = k / CIN, c = k % CIN;
            const int kh = t / 3, kw = t - 3 * (t / 3);
            V bv[NPW];
#pragma unroll
            for (int p = 0; p < NPW; ++p) {
                const int y = 2 * oy[p] + kh - 1, x = 2 * ox[p] + kw - 1;
                const bool ok = t < 9 && y >= 0 && x >= 0;
                const int o0 = ok ? in + l8<CIN, WI>(y, x, c / 16) : zo;
                const int o1 = ok ? in + l8<CIN, WI>(y, x, c / 16 + 1) : zo + 16;
                bv[p] = ld32(smem, o0, o1);
            }
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int p = 0; p < NPW; ++p) mma8(acc[m][p], A[ks][m], bv[p]);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int ch = (tr * MT + m) * 16 + 4 * g;
#pragma unroll
            for (int p = 0; p < NPW; ++p)
                st4(smem, out + l8<COUT, WO>(oy[p], ox[p], ch / 16) + ch % 16, acc[m][p], a.acc_scale[L], bias[m],
                    a.qout[L]);
        }
    }
}

// Weights of a transposed-convolution layer a wave keeps in registers:
// the (phase, neighbour) blocks of its set for its MT row blocks.
template <int MT>
struct Panel8 {
    V A[5][MT];
    float bias[MT][4];
};

template <int L, int COUT, int MT>
__device__ __forceinline__ void panel8_load(Panel8<MT>& P, const F8Args& a, int tr, int set) {
    const int lane = otid() & 63, g = lane >> 4, r16 = lane & 15;
    const uint8_t* w = opq(a.w[L]);
    const int kst = a.kstride[L];
    const int q0 = set ? 5 : 0, nq = set ? 4 : 5;
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int m = 0; m < MT; ++m)
            if (q < nq)
                P.A[q][m] = *(const V*)(w + (size_t)((q0 + q) * COUT + (tr * MT + m) * 16 + r16) * kst + 32 * g);
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) P.bias[m][e] = opq(a.b[L])[(tr * MT + m) * 16 + 4 * g + e];
}

// Transposed conv over the four output phases for GEMM pixel blocks
// [pix0/16 + tp*NPW ...): input [in0 (C0) | in1 (C1)] at HI x WI; output of
// COUT channels at (2 HI) x (2 WI), row r stored at row r % RING of `out`
// (RING = 0: no ring).
template <int L, int HI, int WI, int C0, int C1, int COUT, int MT, int NPW, int SET, int NPB, int RING>
__device__ __forceinline__ void pairs8(const Panel8<MT>& P, char* smem, int in0, int in1, int out, int zo, int tr,
                                       int tp0, int tp_step, int pix0, const F8Args& a) {
    constexpr int WO = 2 * WI, TP = NPB / NPW;
    constexpr int Q0 = SET ? 5 : 0, NQ = SET ? 4 : 5;
    constexpr int PH0 = SET ? 3 : 0, NPH = SET ? 1 : 3;
    constexpr int NNB = SET ? 4 : 3;
    const int lane = otid() & 63, g = lane >> 4, r16 = lane & 15;
    // lane group g: channels [32 g, 32 g + 32) of [in0 | in1]
    const int src = (32 * g) >= C0 ? 1 : 0;
    const int cb = 32 * g - src * C0;
    const int base = src ? in1 : in0;
    for (int tp = tp0; tp < TP; tp += tp_step) {
        int ia[NPW], ib[NPW];
        V bv[NNB][NPW];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = pix0 + (tp * NPW + p) * 16 + r16;
            ia[p] = (int)((unsigned)pix / WI);
            ib[p] = (int)((unsigned)pix % WI);
#pragma unroll
            for (int nb = 0; nb < NNB; ++nb) {
                const int di = nb >> 1, dj = nb & 1;
                const bool ok = ia[p] + di < HI && ib[p] + dj < WI;
                int o0, o1;
                if (src == 0) {
                    o0 = ok ? base + l8<C0, WI>(ia[p] + di, ib[p] + dj, cb / 16) : zo;
                    o1 = ok ? base + l8<C0, WI>(ia[p] + di, ib[p] + dj, cb / 16 + 1) : zo + 16;
                } else {
                    o0 = ok ? base + l8<(C1 > 0 ? C1 : 32), WI>(ia[p] + di, ib[p] + dj, cb / 16) : zo;
                    o1 = ok ? base + l8<(C1 > 0 ? C1 : 32), WI>(ia[p] + di, ib[p] + dj, cb / 16 + 1) : zo + 16;
                }
                bv[nb][p] = ld32(smem, o0, o1);
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
        for (int q = 0; q < NQ; ++q) {
            const int ph = pair_phase(Q0 + q) - PH0, nb = pair_nb(Q0 + q);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int p = 0; p < NPW; ++p) mma8(acc[ph][m][p], P.A[q][m], bv[nb][p]);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int ch = (tr * MT + m) * 16 + 4 * g;
#pragma unroll
            for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
                for (int p = 0; p < NPW; ++p) {
                    const int PP = PH0 + ph;
                    int oy = 2 * ia[p] + (PP >> 1);
                    if constexpr (RING > 0) oy %= RING;
                    const int ox = 2 * ib[p] + (PP & 1);
                    st4(smem, out + l8<COUT, WO>(oy, ox, ch / 16) + ch % 16, acc[ph][m][p], a.acc_scale[L],
                        P.bias[m], a.qout[L]);
                }
        }
    }
}

// D1: rows (phase, channel), K = (neighbour, channel of [u2 | h1]) in 2 steps;
// GEMM rows [row0, row0 + nrows) of the u2 grid (u2 row r at ring row r % RING).
struct D1P8 {
    V A[2];
    float bias[4];
};

template <int HI, int WI, int NPW, int RING>
__device__ __forceinline__ void d1_phase8(const D1P8& P, char* smem, int u2, int h1, int zo, float* ym, int relu,
                                          int row0, int nrows, float scale) {
    constexpr int WO = 2 * WI;
    const int tid = otid();
    const int lane = tid & 63, wave = tid >> 6, g = lane >> 4, r16 = lane & 15;
    const int TP = nrows * WI / 16 / NPW;
    for (int tp = wave; tp < TP; tp += NW) {
        int ia[NPW], ib[NPW];
        f4 acc[NPW];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = row0 * WI + (tp * NPW + p) * 16 + r16;
            ia[p] = (int)((unsigned)pix / WI);
            ib[p] = (int)((unsigned)pix % WI);
            acc[p] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int nb = 2 * ks + (g >> 1), di = nb >> 1, dj = nb & 1;
#pragma unroll
            for (int p = 0; p < NPW; ++p) {
                const int y = ia[p] + di, x = ib[p] + dj;
                const bool ok = y < HI && x < WI;
                int o0, o1;
                if (g & 1) {  // h1
                    o0 = ok ? h1 + l8<32, WI>(y, x, 0) : zo;
                    o1 = ok ? h1 + l8<32, WI>(y, x, 1) : zo + 16;
                } else {      // u2 (ring)
                    const int yr = RING > 0 ? y % (RING > 0 ? RING : 1) : y;
                    o0 = ok ? u2 + l8<32, WI>(yr, x, 0) : zo;
                    o1 = ok ? u2 + l8<32, WI>(yr, x, 1) : zo + 16;
                }
                mma8(acc[p], P.A[ks], ld32(smem, o0, o1));
            }
        }
#pragma unroll
        for (int p = 0; p < NPW; ++p)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 4 * g + e;
                if (r >= 12) continue;
                const int ph = r / 3;
                const int opix = (2 * ia[p] + (ph >> 1)) * WO + 2 * ib[p] + (ph & 1);
                float v = acc[p][e] * scale + P.bias[e];
                if (relu) v = drc::relu(v);
                ym[opix * 3 + (r - ph * 3)] = v;
            }
    }
}

template <int H, int W>
struct F8Lds {
    static constexpr int HW = H * W;
    static constexpr int R0 = 0, R1 = 8 * HW, R2 = 16 * HW;
    static constexpr int H2 = R1, H3 = R1 + 4 * HW;
    static constexpr int BAND = 4;                      // D2 input rows per band
    static constexpr int RING = 2 * BAND + 1;           // u2 rows kept for D1
    static constexpr int RING_BYTES = RING * (W / 2) * 32;
    static constexpr bool RING_IN_R1 = RING_BYTES <= 4 * HW - 256;
    static constexpr int RG = RING_IN_R1 ? R1 + 4 * HW : 20 * HW;
    static constexpr int ZO = R1 + 8 * HW - 256;
    static constexpr int BYTES = RING_IN_R1 ? 20 * HW : 20 * HW + RING_BYTES;
};

template <int H, int W>
__global__ __launch_bounds__(NT, 2) void cae_fused_fp8_kernel(const F8Args a) {
    // static LDS: LDS offsets fold into the instructions' immediate fields
    __shared__ __align__(16) char smem[F8Lds<H, W>::BYTES];
    typedef F8Lds<H, W> L;
    constexpr int HW = H * W;
    constexpr int E1N = (HW / 64) >= 4 * 4 * 4 ? 4 : 2;     // E1: PB = HW/64
    constexpr int E2N = (HW / 256) >= 8 ? 4 : 1;            // E2: 2 groups of 2, PB = HW/256
    constexpr int E3N = (HW / 1024) >= 4 ? 2 : 1;           // E3: 4 groups of 2, PB = HW/1024
    constexpr int D3N = 1;                                  // D3: 2 groups x 2 sets, PB = HW/1024
    constexpr int D2BPB = L::BAND * (W / 4) / 16;           // D2 pixel blocks per band
    constexpr int D2BN = 1;
    constexpr int D1N = (W / 2) >= 32 ? 2 : 1;
    constexpr int NBAND = (H / 4) / L::BAND;
    constexpr int HU = H / 2, WU = W / 2;
    static_assert((H / 4) % L::BAND == 0, "whole bands");
    for (int m = blockIdx.x; m < a.nmaps; m += gridDim.x) {
        const float* xm = a.x + (a.x_off ? a.x_off[m] : (long)m * HW * 7);
        float* ym = a.y + (a.y_off ? a.y_off[m] : (long)m * HW * 3);
        stage_x8<H, W>(smem, L::R1, xm, a.xscale);
        __syncthreads();
        e1_phase<H, W, E1N>(smem, L::R1, L::R0, a);
        __syncthreads();
        // x is dead: the zero block at the end of R1 (after h2 and h3). Every
        // wave clears it before its own first read (LDS operations of a wave
        // complete in order), so no barrier is needed between this store and
        // E2's taps outside the map; the other waves only write zeros there.
        if ((threadIdx.x & 63) < 16) *(uint4*)(smem + L::ZO + 16 * (threadIdx.x & 63)) = uint4{0u, 0u, 0u, 0u};
        conv_phase8<1, H / 2, W / 2, 32, 64, 2, E2N>(smem, L::R0, L::H2, L::ZO, a);
        __syncthreads();
        conv_phase8<2, H / 4, W / 4, 64, 128, 2, E3N>(smem, L::H2, L::H3, L::ZO, a);
        __syncthreads();
        {   // D3: h3 -> u3, 2 row-block groups x 2 sets, one per wave
            constexpr int NG = 4;
            const int wave = otid() >> 6;
            const int gid = (wave + blockIdx.x) % NG, tr = gid >> 1, set = gid & 1;
            Panel8<2> P;
            panel8_load<3, 64, 2>(P, a, tr, set);
            constexpr int NPB = (H / 8) * (W / 8) / 16;
            if (set == 0)
                pairs8<3, H / 8, W / 8, 128, 0, 64, 2, D3N, 0, NPB, 0>(P, smem, L::H3, L::H3, L::R2, L::ZO, tr, 0, 1, 0,
                                                                         a);
            else
                pairs8<3, H / 8, W / 8, 128, 0, 64, 2, D3N, 1, NPB, 0>(P, smem, L::H3, L::H3, L::R2, L::ZO, tr, 0, 1, 0,
                                                                         a);
        }
        __syncthreads();
        {   // D2 in bands into the u2 ring, each band followed by D1 on its rows
            constexpr int NG = 2;  // both row blocks per wave, 2 sets
            const int wave = otid() >> 6;
            const int set = (wave + blockIdx.x) % NG;
            Panel8<2> P2;
            panel8_load<4, 32, 2>(P2, a, 0, set);
            D1P8 P1;
            {
                const int lane = otid() & 63, g = lane >> 4, r16 = lane & 15;
                const uint8_t* w = opq(a.w[5]);
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) P1.A[ks] = *(const V*)(w + (size_t)r16 * a.kstride[5] + ks * 128 + 32 * g);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = 4 * g + e;
                    P1.bias[e] = r < 12 ? opq(a.b[5])[r % 3] : 0.0f;
                }
            }
            for (int band = 0; band < NBAND; ++band) {
                const int pix0 = band * L::BAND * (W / 4);
                if (set == 0)
                    pairs8<4, H / 4, W / 4, 64, 64, 32, 2, D2BN, 0, D2BPB, L::RING>(P2, smem, L::R2, L::H2, L::RG, L::ZO,
                                                                                   0, wave / NG, NW / NG, pix0, a);
                else
                    pairs8<4, H / 4, W / 4, 64, 64, 32, 2, D2BN, 1, D2BPB, L::RING>(P2, smem, L::R2, L::H2, L::RG, L::ZO,
                                                                                   0, wave / NG, NW / NG, pix0, a);
                __syncthreads();
                const int u0 = 2 * L::BAND * band;
                const int r0 = band ? u0 - 1 : 0;
                const int r1 = band + 1 < NBAND ? u0 + 2 * L::BAND - 1 : HU;
                d1_phase8<HU, WU, D1N, L::RING>(P1, smem, L::RG, L::R0, L::ZO, ym, a.final_relu, r0, r1 - r0,
                                                a.acc_scale[5]);
                __syncthreads();
            }
        }
    }
}

template <int H, int W>
drc_status launch_fp8(const F8Args& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((cae_fused_fp8_kernel<H, W>), dim3(grid), dim3(NT), 0, s, a);
    return check_launch("fused fp8 forward");
}

}  // namespace

// Whole-network FP8 forward of n maps of H x W (32x32 or 64x64).
drc_status fused_fp8_forward(drc_cae* h, const float* x, float* y, int n, int H, int W, const long* x_off,
                             const long* y_off, hipStream_t s) {
    if (h->prec != P_FP8 || !fused_forward_size(H, W))
        return drc_fail(DRC_ERR_UNSUPPORTED, "fused fp8 forward: FP8 maps of 32x32 or 64x64 only");
    if (n < 1) return DRC_OK;
    static const int kIn[6] = {6, 7, 8, 9, 8, 7};
    static const int kOut[6] = {7, 8, 9, 8, 7, -1};
    const float* sc = h->host_scales;
    F8Args a;
    memset(&a, 0, sizeof a);
    a.x = x;
    a.y = y;
    a.nmaps = n;
    a.x_off = x_off;
    a.y_off = y_off;
    for (int l = 0; l < 6; ++l) {
        a.w[l] = (const uint8_t*)h->wf[l];
        a.kstride[l] = gemm_geom(l, false, P_FP8).kstride;
        a.b[l] = h->bias + bias_slot(l);
        a.acc_scale[l] = 1.0f / (sc[kIn[l]] * sc[l]);
        a.qout[l] = kOut[l] >= 0 ? sc[kOut[l]] : 1.0f;
    }
    a.xscale = sc[6];
    a.final_relu = h->desc.final_relu;
    // two workgroups per CU (80 KB of LDS and 4 waves each at 64x64)
    const int grid = std::max(1, std::min(n, 2 * h->num_cu));
    const long tok = prof_begin(h, PROF_FUSED, s);
    const drc_status st = (H == 64) ? launch_fp8<64, 64>(a, grid, s) : launch_fp8<32, 32>(a, grid, s);
    prof_end(h, tok, s);
    return st;
}
