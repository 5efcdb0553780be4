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
// swizzled per pixel against bank conflicts):
//   R0 [0, 16HW)           h1 (E1 -> E2), then u2 (D2 -> D1)
//   R1 [16HW, 24HW)        h2 (E2 -> D2)
//   R2 [24HW, 32HW)        u3 (D3 -> D2)
//   R3 [32HW, 36HW)        h3 (E3 -> D3)
//   R1+R2                  x as BF16, 8 channels (staging -> E1), and h1
//                          again for D1 (reloaded from the workgroup's slot)
// 36 HW bytes in all: 144 KB at 64x64 (one workgroup per CU), 36 KB at 32x32.
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

struct FusedArgs {
    const float* x;      // [.., H, W, 7] float32
    float* y;            // [.., H, W, 3] float32
    int nmaps;
    const long* x_off;   // element offset of each map (null: packed)
    const long* y_off;
    const uint16_t* w[6];  // forward packs (layer path layout)
    const float* b[6];
    char* scratch;       // one h1 slot of 16 H W bytes per workgroup
    int final_relu;
};

__device__ __forceinline__ uint16_t bf16_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

// Byte offset of 16-byte chunk `chunk` of pixel p in an LDS tensor of C
// channels. The chunk index is XORed with bits of p so that 16 lanes reading
// the same chunk of pixels 1 or 2 apart spread over the banks.
template <int C>
__device__ __forceinline__ int loff(int p, int chunk) {
    constexpr int CH = C / 8;
    int sw;
    if constexpr (CH == 1) sw = 0;
    else if constexpr (CH == 4) sw = (p >> 2) & 3;
    else if constexpr (CH == 8) sw = (p >> 1) & 7;
    else sw = p & 15;
    return p * (C * 2) + ((chunk ^ sw) & (CH - 1)) * 16;
}

// Stores channels [ch, ch+4) of pixel p (bias added, optional ReLU) as BF16.
template <int C>
__device__ __forceinline__ void lds_store4(char* t, int p, int ch, const f4& acc, const float* bias, bool relu) {
    float v[4] = {acc.x + bias[0], acc.y + bias[1], acc.z + bias[2], acc.w + bias[3]};
    if (relu) {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (v[e] < 0.0f) ? 0.0f : v[e];
    }
    uint2 w;
    w.x = (uint32_t)bf16_bits(v[0]) | ((uint32_t)bf16_bits(v[1]) << 16);
    w.y = (uint32_t)bf16_bits(v[2]) | ((uint32_t)bf16_bits(v[3]) << 16);
    *(uint2*)(t + loff<C>(p, ch >> 3) + ((ch >> 2) & 1) * 8) = w;
}

__device__ __forceinline__ void mma(f4& acc, const uint4& a, const uint4& b) { Traits<P_BF16>::mma(acc, a, b); }

// Hides a uniform pointer's value from the optimiser: weight loads are then
// issued inside the tile loop instead of being hoisted out of the map loop
// (where they would pin hundreds of registers across every layer).
template <typename T>
__device__ __forceinline__ const T* opaque(const T* p) {
    asm volatile("" : "+s"(p));
    return p;
}
// The same for the thread index: per-lane addresses of a layer are then
// recomputed inside the map loop rather than kept live across all layers.
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// x (float32, 7 channels) -> LDS as BF16 with 8 channels (channel 7 = 0).
// Flat float4 loads (coalesced), in groups of up to 8 per thread in flight.
template <int H, int W>
__device__ __forceinline__ void stage_x(char* xs, const float* xm) {
    constexpr int NF4 = H * W * 7 / 4;
    constexpr int IT = (NF4 + FT - 1) / FT;
    constexpr int GRP = IT < 8 ? IT : 8;
    const int tid = opaque_tid();
    for (int p = tid; p < H * W; p += FT) *(uint16_t*)(xs + p * 16 + 14) = 0;
#pragma unroll
    for (int g0 = 0; g0 < IT; g0 += GRP) {
        float4 v[GRP];
#pragma unroll
        for (int it = 0; it < GRP; ++it) {
            const int i = tid + (g0 + it) * FT;
            if (g0 + it < IT && (NF4 % FT == 0 || i < NF4)) v[it] = ((const float4*)xm)[i];
        }
#pragma unroll
        for (int it = 0; it < GRP; ++it) {
            const int i = tid + (g0 + it) * FT;
            if (g0 + it < IT && (NF4 % FT == 0 || i < NF4)) {
                const float vv[4] = {v[it].x, v[it].y, v[it].z, v[it].w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int f = 4 * i + k, p = f / 7, c = f - p * 7;
                    *(uint16_t*)(xs + p * 16 + c * 2) = bf16_bits(vv[k]);
                }
            }
        }
    }
}

// Stride-2 3x3 convolution, LDS -> LDS, bias + ReLU (E1, E2, E3). Pack
// [COUT][KSTEPS*32], k = tap * CIN + c. A wave owns tiles of MT row blocks
// x NPW pixel blocks (16 consecutive output pixels each).
template <int HI, int WI, int CIN, int COUT, int MT, int NPW>
__device__ __forceinline__ void conv_phase(const char* in, char* out, const uint16_t* wp, const float* bias_g) {
    constexpr int HO = HI / 2, WO = WI / 2;
    constexpr int PB = HO * WO / 16, RB = COUT / 16;
    constexpr int KSTEPS = (9 * CIN + 31) / 32, KSTRIDE = KSTEPS * 32;
    constexpr int TR = RB / MT, TP = PB / NPW;
    static_assert(RB % MT == 0 && PB % NPW == 0, "tiles cover the layer");
    const int tid = opaque_tid();
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    for (int tile = wave; tile < TR * TP; tile += FW) {
        const int tr = tile % TR, tp = tile / TR;
        const uint16_t* w = opaque(wp);
        int oy[NPW], ox[NPW];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = (tp * NPW + p) * 16 + r16;
            oy[p] = pix / WO;
            ox[p] = pix % WO;
        }
        f4 acc[MT][NPW];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int p = 0; p < NPW; ++p) acc[m][p] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            int t, chunk;
            if constexpr (CIN >= 32) {
                t = ks * 32 / CIN;
                chunk = (ks * 32 % CIN) / 8 + g;
            } else {  // CIN == 8: one tap per lane group
                t = ks * 4 + g;
                chunk = 0;
            }
            uint4 a[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m)
                a[m] = *(const uint4*)(w + (size_t)((tr * MT + m) * 16 + r16) * KSTRIDE + ks * 32 + g * 8);
            const int kh = t / 3, kw = t - (t / 3) * 3;
            uint4 b[NPW];
#pragma unroll
            for (int p = 0; p < NPW; ++p) {
                const int iy = 2 * oy[p] + kh - 1, ix = 2 * ox[p] + kw - 1;
                const bool ok = t < 9 && iy >= 0 && ix >= 0;
                b[p] = ok ? *(const uint4*)(in + loff<CIN>(iy * WI + ix, chunk)) : uint4{0u, 0u, 0u, 0u};
            }
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int p = 0; p < NPW; ++p) mma(acc[m][p], a[m], b[p]);
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int ch = (tr * MT + m) * 16 + g * 4;
            const float* bg = opaque(bias_g);
            const float bias[4] = {bg[ch], bg[ch + 1], bg[ch + 2], bg[ch + 3]};
#pragma unroll
            for (int p = 0; p < NPW; ++p) lds_store4<COUT>(out, oy[p] * WO + ox[p], ch, acc[m][p], bias, true);
        }
    }
}

// Stride-2 3x3 transposed convolution over all four output phases, LDS ->
// LDS, bias + ReLU (D3, D2). Input = [in0 (C0 ch) | in1 (C1 ch)] at HI x WI;
// GEMM pixel (a, b) gathers its neighbours (a + di, b + dj) and feeds the 9
// (phase, neighbour) weight blocks, pack [q][COUT][C0 + C1].
template <int HI, int WI, int C0, int C1, int COUT, int MT, int NPW>
__device__ __forceinline__ void pairs_phase(const char* in0, const char* in1, char* out, const uint16_t* wp,
                                            const float* bias_g) {
    constexpr int CIN = C0 + C1, PB = HI * WI / 16, RB = COUT / 16, KSN = CIN / 32;
    constexpr int WO = 2 * WI;
    constexpr int TR = RB / MT, TP = PB / NPW;
    static_assert(RB % MT == 0 && PB % NPW == 0 && C0 % 32 == 0 && C1 % 32 == 0, "tiles cover the layer");
    static_assert(C1 == 0 || C1 == C0, "both sources share one LDS layout");
    const int tid = opaque_tid();
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    for (int tile = wave; tile < TR * TP; tile += FW) {
        const int tr = tile % TR, tp = tile / TR;
        const uint16_t* w = opaque(wp);
        int ia[NPW], ib[NPW];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = (tp * NPW + p) * 16 + r16;
            ia[p] = pix / WI;
            ib[p] = pix % WI;
        }
        f4 acc[4][MT][NPW];
#pragma unroll
        for (int ph = 0; ph < 4; ++ph)
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int p = 0; p < NPW; ++p) acc[ph][m][p] = f4{0.f, 0.f, 0.f, 0.f};
        // K steps stay rolled: unrolled, the 9 weight loads of every step are
        // hoisted together and overflow the register file
#pragma unroll 1
        for (int ks = 0; ks < KSN; ++ks) {
            const bool second = ks * 32 >= C0;
            const char* src0 = second ? in1 : in0;
            const int chunk = (second ? (ks * 32 - C0) / 8 : ks * 4) + g;
            uint4 bv[4][NPW];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const int di = nb >> 1, dj = nb & 1;
#pragma unroll
                for (int p = 0; p < NPW; ++p) {
                    const int y = ia[p] + di, x = ib[p] + dj;
                    const bool ok = y < HI && x < WI;
                    bv[nb][p] = ok ? *(const uint4*)(src0 + loff<C0>(y * WI + x, chunk)) : uint4{0u, 0u, 0u, 0u};
                }
            }
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int ph = pair_phase(q), nb = pair_nb(q);
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    const int row = q * COUT + (tr * MT + m) * 16 + r16;
                    const uint4 a = *(const uint4*)(w + (size_t)row * CIN + ks * 32 + g * 8);
#pragma unroll
                    for (int p = 0; p < NPW; ++p) mma(acc[ph][m][p], a, bv[nb][p]);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int ch = (tr * MT + m) * 16 + g * 4;
            const float* bg = opaque(bias_g);
            const float bias[4] = {bg[ch], bg[ch + 1], bg[ch + 2], bg[ch + 3]};
#pragma unroll
            for (int ph = 0; ph < 4; ++ph)
#pragma unroll
                for (int p = 0; p < NPW; ++p) {
                    const int opix = (2 * ia[p] + (ph >> 1)) * WO + 2 * ib[p] + (ph & 1);
                    lds_store4<COUT>(out, opix, ch, acc[ph][m][p], bias, true);
                }
        }
    }
}

// D1: transposed convolution [u2 | h1] (32 + 32 channels at HI x WI) -> 3
// channels, linear, float32 to global. Merged rows r = phase * 3 + co (12 of
// 16 used), K = neighbour * 64 + c, pack [16][256].
template <int HI, int WI, int NPW>
__device__ __forceinline__ void d1_phase(const char* u2, const char* h1, float* ym, const uint16_t* wp,
                                         const float* bias_g, bool relu) {
    constexpr int PB = HI * WI / 16, WO = 2 * WI, TP = PB / NPW;
    static_assert(PB % NPW == 0, "tiles cover the layer");
    const int tid = opaque_tid();
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    uint4 a[8];
    const uint16_t* w = opaque(wp);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) a[ks] = *(const uint4*)(w + (size_t)r16 * 256 + ks * 32 + g * 8);
    float bias[4];
    int rph[4], rco[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = g * 4 + e;
        rph[e] = r / 3;
        rco[e] = r - (r / 3) * 3;
        bias[e] = r < 12 ? bias_g[rco[e]] : 0.0f;
    }
    for (int tp = wave; tp < TP; tp += FW) {
        int ia[NPW], ib[NPW];
#pragma unroll
        for (int p = 0; p < NPW; ++p) {
            const int pix = (tp * NPW + p) * 16 + r16;
            ia[p] = pix / WI;
            ib[p] = pix % WI;
        }
        f4 acc[NPW];
#pragma unroll
        for (int p = 0; p < NPW; ++p) acc[p] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const int nb = ks >> 1, di = nb >> 1, dj = nb & 1;
            const char* src = (ks & 1) ? h1 : u2;
#pragma unroll
            for (int p = 0; p < NPW; ++p) {
                const int y = ia[p] + di, x = ib[p] + dj;
                const bool ok = y < HI && x < WI;
                const uint4 b = ok ? *(const uint4*)(src + loff<32>(y * WI + x, g)) : uint4{0u, 0u, 0u, 0u};
                mma(acc[p], a[ks], b);
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

// 16-byte copies of `bytes` between LDS and global (both 16-byte aligned).
__device__ __forceinline__ void copy_out(char* dst, const char* lds, int bytes) {
    for (int i = threadIdx.x; i < bytes / 16; i += FT) ((uint4*)dst)[i] = ((const uint4*)lds)[i];
}
__device__ __forceinline__ void copy_in(char* lds, const char* src, int bytes) {
    for (int i = threadIdx.x; i < bytes / 16; i += FT) ((uint4*)lds)[i] = ((const uint4*)src)[i];
}

template <int H, int W>
__global__ __launch_bounds__(FT) void cae_fused_forward_kernel(const FusedArgs a) {
    extern __shared__ __align__(16) char smem[];
    constexpr int HW = H * W;
    char* R0 = smem;
    char* R1 = smem + 16 * HW;
    char* R2 = smem + 24 * HW;
    char* R3 = smem + 32 * HW;
    char* slot = a.scratch + (size_t)blockIdx.x * (16 * HW);
    // pixel blocks per wave: enough tiles for 8 waves at both map sizes
    constexpr int E1N = (HW / 64) >= 8 * 4 * 2 ? 4 : 2;     // E1: 2 row blocks x PB = HW/64
    constexpr int E2N = (HW / 256) >= 4 * 4 ? 4 : 1;        // E2: 2 pairs of row blocks x PB = HW/256
    constexpr int E3M = (HW / 1024) >= 4 ? 2 : 1;           // E3: 8 row blocks x PB = HW/1024
    constexpr int E3N = (HW / 1024) >= 4 ? 2 : 1;
    constexpr int D3N = (HW / 1024) >= 4 ? 2 : 1;           // D3: 4 row blocks x PB = HW/1024
    constexpr int D2N = (HW / 256) >= 16 ? 4 : 1;           // D2: 2 row blocks x PB = HW/256
    constexpr int D1N = (HW / 64) >= 8 * 4 ? 4 : 2;         // D1: PB = HW/64
    for (int m = blockIdx.x; m < a.nmaps; m += gridDim.x) {
        const float* xm = a.x + (a.x_off ? a.x_off[m] : (long)m * HW * 7);
        float* ym = a.y + (a.y_off ? a.y_off[m] : (long)m * HW * 3);
        stage_x<H, W>(R1, xm);
        __syncthreads();
        conv_phase<H, W, 8, 32, 2, E1N>(R1, R0, a.w[0], a.b[0]);
        __syncthreads();
        copy_out(slot, R0, 16 * HW);
        conv_phase<H / 2, W / 2, 32, 64, 2, E2N>(R0, R1, a.w[1], a.b[1]);
        __syncthreads();
        conv_phase<H / 4, W / 4, 64, 128, E3M, E3N>(R1, R3, a.w[2], a.b[2]);
        __syncthreads();
        pairs_phase<H / 8, W / 8, 128, 0, 64, 1, D3N>(R3, nullptr, R2, a.w[3], a.b[3]);
        __syncthreads();
        pairs_phase<H / 4, W / 4, 64, 64, 32, 1, D2N>(R2, R1, R0, a.w[4], a.b[4]);
        __syncthreads();
        copy_in(R1, slot, 16 * HW);
        __syncthreads();
        d1_phase<H / 2, W / 2, D1N>(R0, R1, ym, a.w[5], a.b[5], a.final_relu != 0);
        __syncthreads();
    }
}

template <int H, int W>
drc_status launch_fused(const FusedArgs& a, int grid, hipStream_t s) {
    const int lds = 36 * H * W;
    auto kern = cae_fused_forward_kernel<H, W>;
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
            return drc_fail(DRC_ERR_HIP, "fused forward: cannot raise the LDS limit to %d bytes", lds);
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(FT), lds, s, a);
    return check_launch("fused forward");
}

}  // namespace

// Map sizes the fused kernel is built for.
bool fused_forward_size(int H, int W) { return (H == 64 && W == 64) || (H == 32 && W == 32); }

// Workgroups of one fused launch over n maps of H x W.
int fused_forward_grid(const drc_cae* h, int n, int H, int W) {
    const int per_cu = (H * W >= 4096) ? 1 : 2;
    return std::max(1, std::min(n, h->num_cu * per_cu));
}

// Scratch bytes of one fused launch (one h1 slot per workgroup).
size_t fused_forward_scratch(const drc_cae* h, int n, int H, int W) {
    return (size_t)fused_forward_grid(h, n, H, W) * 16 * H * W;
}

drc_status fused_forward(drc_cae* h, const float* x, float* y, int n, int H, int W, const long* x_off,
                         const long* y_off, void* scratch, size_t scratch_bytes, hipStream_t s) {
    if (h->prec != P_BF16 || !fused_forward_size(H, W))
        return drc_fail(DRC_ERR_UNSUPPORTED, "fused forward: BF16 maps of 32x32 or 64x64 only");
    if (n < 1) return DRC_OK;
    if (scratch_bytes < fused_forward_scratch(h, n, H, W))
        return drc_fail(DRC_ERR_WORKSPACE, "fused forward: scratch %zu < %zu bytes", scratch_bytes,
                        fused_forward_scratch(h, n, H, W));
    FusedArgs a;
    memset(&a, 0, sizeof a);
    a.x = x;
    a.y = y;
    a.nmaps = n;
    a.x_off = x_off;
    a.y_off = y_off;
    for (int l = 0; l < 6; ++l) {
        a.w[l] = (const uint16_t*)h->wf[l];
        a.b[l] = h->bias + bias_slot(l);
    }
    a.scratch = (char*)scratch;
    a.final_relu = h->desc.final_relu;
    const int grid = fused_forward_grid(h, n, H, W);
    const long tok = prof_begin(h, PROF_FUSED, s);
    drc_status st = (H == 64) ? launch_fused<64, 64>(a, grid, s) : launch_fused<32, 32>(a, grid, s);
    prof_end(h, tok, s);
    return st;
}
