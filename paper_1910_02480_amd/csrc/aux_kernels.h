// Small kernels around the layer GEMMs: weight packing, FP8 amax, the L1
// loss and its gradient, bias gradients, weight gradients, and Adam.
#pragma once
#include "common.h"
#include "conv_layer.h"

namespace drc {

// ------------------------------------------------------------------ packing
// Packs one layer's W[co][kh][kw][ci] (float32) into the A operand of the
// layer GEMM: dst[phase][row][k], k = tap * cin_eff + c, zero padded.
// Forward pack: row = co, c = ci. Transposed pack (backward data pass):
// row = ci, c = co, with the GEMM mode of the adjoint layer.
struct PackArgs {
    const float* w;
    int cout, cin;      // layer shape
    int gemm_mode;      // M_CONV, M_TCONV_PAIRS or M_TCONV_MERGED: the GEMM this pack feeds
    int transpose;
    int cin_eff;        // K elements per tap / neighbour
    int rows_pad;       // GEMM rows per block, padded to 16
    int kstride;        // K elements per row
    int nblk;           // blocks of rows: 1, or 9 (phase, neighbour) pairs
    int prec;
    const float* scale; // FP8: device pointer to the weight scale, else null
    void* dst;
    void* frag;         // BF16: optional second copy in MFMA fragment order (kstride % 32 == 0)
};

// Weight pack element e of the layout [blk][row][k]:
//  M_CONV          k = tap * cin_eff + c, tap = 3 kh + kw;
//  M_TCONV_PAIRS   block = (phase, neighbour) pair, k = c;
//  M_TCONV_MERGED  row = phase * rows + r, k = neighbour * cin_eff + c,
//                  zero where the phase does not use the neighbour.
// Forward pack: row = co, c = ci. Transposed pack (backward data pass):
// row = ci, c = co.
//
// The fragment-ordered copy: fragment (row block rb, K step ks) is 64 lanes
// x 8 elements, lane g * 16 + r holding row 16 rb + r, K [32 ks + 8 g, +8),
// so one wave loads a whole MFMA A fragment as 1 KB of contiguous memory.
__device__ __forceinline__ void pack_range(const PackArgs& a, long e0, long step) {
    const long total = (long)a.nblk * a.rows_pad * a.kstride;
    const int rows = a.transpose ? a.cin : a.cout;
    const int chans = a.transpose ? a.cout : a.cin;
    for (long e = e0; e < total; e += step) {
        const int k = (int)(e % a.kstride);
        int row = (int)((e / a.kstride) % a.rows_pad);
        const int blk = (int)(e / ((long)a.kstride * a.rows_pad));
        float v = 0.0f;
        int kh = 0, kw = 0, c = 0;
        bool ok = false;
        if (a.gemm_mode == M_CONV) {
            const int t = k / a.cin_eff;
            c = k % a.cin_eff;
            kh = t / 3;
            kw = t % 3;
            ok = t < 9 && row < rows;
        } else if (a.gemm_mode == M_TCONV_PAIRS) {
            const int ph = pair_phase(blk), nb = pair_nb(blk);
            kh = tap_kh(ph, nb);
            kw = tap_kw(ph, nb);
            c = k;
            ok = row < rows;
        } else {  // merged rows: (phase, r)
            const int ph = row / rows, nb = k / a.cin_eff;
            c = k % a.cin_eff;
            ok = ph < 4 && nb < 4 && phase_uses(ph, nb);
            if (ok) {
                kh = tap_kh(ph, nb);
                kw = tap_kw(ph, nb);
                row -= ph * rows;
            }
        }
        if (ok && c < chans) {
            const int co = a.transpose ? c : row;
            const int ci = a.transpose ? row : c;
            v = a.w[((co * 3 + kh) * 3 + kw) * a.cin + ci];
        }
        if (a.prec == P_F32) {
            ((float*)a.dst)[e] = v;
        } else if (a.prec == P_BF16) {
            const uint16_t hb = f32_to_bf16(v);
            ((uint16_t*)a.dst)[e] = hb;
            if (a.frag) {
                const long R = e / a.kstride;  // row over all blocks
                const int ksteps = a.kstride / 32, kk = k & 31;
                const long f = ((R / 16) * ksteps + k / 32) * 64 + (kk >> 3) * 16 + (R & 15);
                ((uint16_t*)a.frag)[f * 8 + (kk & 7)] = hb;
            }
        } else {
            ((uint8_t*)a.dst)[e] = f32_to_e4m3(v * a.scale[0]);
        }
    }
}

// Every pack of a handle in one launch: blockIdx.y selects the pack; the
// last y index copies the biases (float32) into their compact slots.
constexpr int kMaxPacks = 18;
struct PackAllArgs {
    PackArgs p[kMaxPacks];
    int np;
    const float* bsrc[6];  // bias vectors of E1..D1 in the parameter vector
    int bcount[6], bslot[6];
    float* bdst;
};
static __global__ void pack_all_kernel(const PackAllArgs a) {
    const long e0 = blockIdx.x * (long)blockDim.x + threadIdx.x, step = (long)gridDim.x * blockDim.x;
    if ((int)blockIdx.y < a.np) {
        pack_range(a.p[blockIdx.y], e0, step);
        return;
    }
    for (int l = 0; l < 6; ++l)
        for (long i = e0; i < a.bcount[l]; i += step) a.bdst[a.bslot[l] + i] = a.bsrc[l][i];
}

// ------------------------------------------------------------------ amax
// out[0] = max(out[0], max |x|) over float32 data. Non-negative floats order
// like their bit patterns, so an integer atomic max is exact and
// order-independent. out must start at 0.
static __global__ void amax_f32_kernel(const float* x, long count, unsigned int* out) {
    float m = 0.0f;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count;
         e += (long)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(x[e]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// scale[i] = 448 / amax[i] (1 when amax is 0), for FP8 e4m3 per-tensor scaling.
static __global__ void fp8_scale_kernel(const unsigned int* amax, float* scale, int count) {
    const int i = threadIdx.x;
    if (i < count) {
        const float m = __uint_as_float(amax[i]);
        scale[i] = (m > 0.0f) ? 448.0f / m : 1.0f;
    }
}

// ------------------------------------------------------------------ L1 loss
// dy = sign(y - t) * dscale (sign(0) = 0); partial[b] = sum |y - t| over the
// block's fixed range, in double. With roll / flip the target is read as
// its augmented map (AugMap; maps of H x W x 3).
static __global__ __launch_bounds__(256) void l1_partial_kernel(const float* y, const float* t, long count,
                                                         long per_block, float dscale, float* dy,
                                                         double* partial, const int32_t* roll,
                                                         const int32_t* flip, int H, int W) {
    // per_block = 16 elements per thread: four 16-byte loads of y and of t per
    // thread, all issued before the arithmetic (count is a multiple of 4)
    __shared__ double red[256];
    const long b0 = blockIdx.x * per_block;
    double s = 0.0;
    float4 yv[4], tv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const long e = b0 + 4 * (threadIdx.x + 256 * k);
        const bool ok = e < count;
        yv[k] = ok ? *(const float4*)(y + e) : make_float4(0.f, 0.f, 0.f, 0.f);
        if (roll) {
            float tt[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const long q = ok ? e + j : 0, p = q / 3, hw = (long)H * W;
                const long m = p / hw, rem = p - m * hw, row = rem / W;
                const int u = (int)(rem - row * W);
                tt[j] = ok ? t[((m * H + row) * W + aug_src_col(roll, flip, m, u, W)) * 3 + (q - 3 * p)] : 0.0f;
            }
            tv[k] = make_float4(tt[0], tt[1], tt[2], tt[3]);
        } else {
            tv[k] = ok ? *(const float4*)(t + e) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const long e = b0 + 4 * (threadIdx.x + 256 * k);
        const float d[4] = {yv[k].x - tv[k].x, yv[k].y - tv[k].y, yv[k].z - tv[k].z, yv[k].w - tv[k].w};
        float g[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            s += fabs((double)d[c]);
            g[c] = (d[c] > 0.0f ? 1.0f : (d[c] < 0.0f ? -1.0f : 0.0f)) * dscale;
        }
        if (e < count) *(float4*)(dy + e) = make_float4(g[0], g[1], g[2], g[3]);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// loss = (sum of partials, fixed order) / count.
static __global__ void l1_final_kernel(const double* partial, int nparts, long count, float* loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(red[0] / (double)count);
}

// ------------------------------------------------------------------ bias gradient
// Column sums of a contiguous [npix][C] tensor (bias gradients), in two
// fixed-order stages. Stage 1 views the tensor as a flat array read with
// VW-element vector loads; the grid stride (in elements) is a multiple of C,
// so every lane of a thread always adds the same channel. The workgroup then
// folds its 256 x VW lane sums into C channel sums through LDS (first S =
// 256 / C interleaved subsets per channel, then the S subset sums) and
// writes partial[block][C]. Stage 2 adds the block rows per channel.
template <typename TG, int VW>
__global__ __launch_bounds__(256) void colsum_partial_kernel(const TG* g, long nelem, int C, float* partial) {
    __shared__ float red[256 * VW];
    __shared__ float red2[256];
    float acc[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) acc[k] = 0.0f;
    const long tid = blockIdx.x * 256L + threadIdx.x;
    const long stride = (long)gridDim.x * 256 * VW;
    for (long e = tid * VW; e < nelem; e += stride) {
        if (e + VW <= nelem) {
            if constexpr (sizeof(TG) == 4) {
                const float4 v = *(const float4*)((const float*)g + e);
                acc[0] += v.x; acc[1] += v.y; acc[2] += v.z; acc[3] += v.w;
            } else {
                const uint4 v = *(const uint4*)((const uint16_t*)g + e);
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    acc[2 * k] += bf16_to_f32((uint16_t)(w[k] & 0xffffu));
                    acc[2 * k + 1] += bf16_to_f32((uint16_t)(w[k] >> 16));
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < VW; ++k)
                if (e + k < nelem) acc[k] += to_float<TG>(g[e + k]);
        }
    }
#pragma unroll
    for (int k = 0; k < VW; ++k) red[threadIdx.x * VW + k] = acc[k];
    __syncthreads();
    // flat LDS index f holds channel (base + f) % C
    const int S = 256 / C;
    const int base_mod = (int)(((long)blockIdx.x * 256 * VW) % C);
    const int t = threadIdx.x;
    if (t < S * C) {
        const int c = t % C, j = t / C;
        const int f0 = (c - base_mod + C) % C;
        float v = 0.0f;
        for (int f = f0 + C * j; f < 256 * VW; f += C * S) v += red[f];
        red2[t] = v;
    }
    __syncthreads();
    if (t < C) {
        float v = 0.0f;
        for (int j = 0; j < S; ++j) v += red2[t + C * j];
        partial[(long)blockIdx.x * C + t] = v;
    }
}

static __global__ __launch_bounds__(256) void colsum_final_kernel(const float* partial, int nrows, int C,
                                                                  float scale, float* out) {
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.0f;
    for (int r = threadIdx.x; r < nrows; r += 256) s += partial[(long)r * C + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0] * scale;
}

// ------------------------------------------------------------------ weight gradient
// dW of a 3x3 layer (stride s = 2, or 1 for a stride-1 convolution) as one
// reduction over "reduction pixels" (n,u,v) on an Hr x Wr grid, with two
// operands:
//   plain    P[n,u,v][cp]                       (tap independent)
//   gathered Q[n, s u+kh-1, s v+kw-1][cq]        (zero outside Hq x Wq)
//   D[j = t*cq + c][cp] = sum_(n,u,v) Q_t[.][c] * P[.][cp],  t = 3 kh + kw.
// Convolution layer: reduction over its output pixels, P = output gradient
// (cp = Cout), Q = layer input (cq = Cin): dW[co][t][ci] = D[t*Cin+ci][co].
// Transposed convolution layer: reduction over its input pixels, P = layer
// input (cp = Cin), Q = output gradient (cq = Cout), since output pixel
// 2i+kh-1 receives input pixel i through row kh: dW[co][t][ci] = D[t*Cout+co][ci].
// MFMA rows are the flattened (tap, channel) pairs j, so 3- and 7-channel
// layers waste little, and all nine taps come out of one pass over the data.
//
// Schedule: FP32 MFMA 16x16x4, K = 4 reduction pixels per MFMA (one per
// 16-lane group). A workgroup owns one tile of JB x PB blocks of 16x16 and a
// range of reduction pixels split into 4 contiguous quarters, one per wave.
// With VEC = 4 a lane loads 4 consecutive channels at once and feeds them to
// 4 MFMA blocks (block i holds rows/columns 4r+i of its 64-wide group); the
// loads of the next U pixel groups are issued before the MFMAs of the
// current ones. Each wave writes its own partial tile (no atomics); partial
// tiles are added later in a fixed order.
struct WgradArgs {
    const void* p; const void* p2;  // plain operand: channels [0, pc0) from p, the rest from p2
    int p_raw, pc, pc0, pld, p2ld;  // p_raw: float32 source
    const void* q;                  // gathered operand
    int q_raw, qc, qld;
    int nmaps, Hr, Wr, Hq, Wq;
    int circ;                       // 1: gathered columns wrap (circular width), 0: zero outside
    int stride;                     // of the layer (2: the autoencoder; 1: the paper's U-Net)
    long per_block;                 // reduction pixels per workgroup
    int jtiles;                     // tiles along j (blockIdx.y = jt + jtiles * pt)
    float* partial;                 // [slot = 4*chunk + wave][9*qc][pc]
};

template <typename T, int VEC>
__device__ __forceinline__ void ld_vec(const void* base, bool raw, long idx, int navail, float (&o)[VEC]) {
    if constexpr (VEC == 1) {
        o[0] = navail > 0 ? (raw ? ((const float*)base)[idx] : to_float<T>(((const T*)base)[idx])) : 0.0f;
    } else {
        if (navail >= 4) {
            if (raw) {
                const float4 v = *(const float4*)((const float*)base + idx);
                o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
            } else if constexpr (sizeof(T) == 4) {
                const float4 v = *(const float4*)((const float*)base + idx);
                o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
            } else {
                const uint2 v = *(const uint2*)((const T*)base + idx);
                o[0] = bf16_to_f32((uint16_t)(v.x & 0xffff));
                o[1] = bf16_to_f32((uint16_t)(v.x >> 16));
                o[2] = bf16_to_f32((uint16_t)(v.y & 0xffff));
                o[3] = bf16_to_f32((uint16_t)(v.y >> 16));
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                o[e] = (e < navail) ? (raw ? ((const float*)base)[idx + e] : to_float<T>(((const T*)base)[idx + e]))
                                    : 0.0f;
        }
    }
}

template <typename T, int JB, int PB, int VEC>
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a) {
    static_assert(JB % VEC == 0 && PB % VEC == 0, "vector loads feed VEC blocks");
    constexpr int U = 4;           // pixel groups in flight per wave
    constexpr int JG = JB / VEC;   // load groups along j
    constexpr int PG = PB / VEC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, r16 = lane & 15;
    const int jt = blockIdx.y % a.jtiles, pt = blockIdx.y / a.jtiles;
    const int J = 9 * a.qc;
    // Row j of block (group jg, element i) for this lane: VEC == 4 ->
    // jg*64 + 4*r16 + i; VEC == 1 -> block jg*16 + r16.
    int tkh[JG], tkw[JG], tch[JG], jav[JG];
#pragma unroll
    for (int b = 0; b < JG; ++b) {
        const int j = (jt * JB) * 16 + b * 16 * VEC + VEC * r16;
        const int t = j < J ? j / a.qc : 9;
        tch[b] = j < J ? j - t * a.qc : 0;
        tkh[b] = t / 3;
        tkw[b] = t - 3 * (t / 3);
        // channels of this tap available from j on (vector loads never cross a tap)
        jav[b] = j < J ? min(VEC, a.qc - tch[b]) : 0;
    }
    int pch[PG], pav[PG];
#pragma unroll
    for (int b = 0; b < PG; ++b) {
        pch[b] = (pt * PB) * 16 + b * 16 * VEC + VEC * r16;
        pav[b] = pch[b] < a.pc ? min(VEC, a.pc - pch[b]) : 0;
    }
    const int hw = a.Hr * a.Wr;
    const long K = (long)a.nmaps * hw;
    const long k_begin = blockIdx.x * a.per_block;
    const long k_end = min(K, k_begin + a.per_block);
    const long quarter = ((a.per_block + 15) / 16) * 4;  // multiple of 4 pixels
    const long w_begin = k_begin + wave * quarter;
    const long w_end = min(k_end, w_begin + quarter);

    f4 acc[JB][PB];
#pragma unroll
    for (int i = 0; i < JB; ++i)
#pragma unroll
        for (int j = 0; j < PB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    float qv[2][U][JG][VEC], pv[2][U][PG][VEC];
    auto load = [&](int buf, long k0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long k = k0 + 4 * u + kq;
            const bool ok = k < w_end;
            const int kk = ok ? (int)k : 0;
            const int n = kk / hw;
            const int rem = kk - n * hw;
            const int uu = rem / a.Wr, vv = rem - (rem / a.Wr) * a.Wr;
#pragma unroll
            for (int b = 0; b < PG; ++b) {
                const int c = pch[b];
                if (c < a.pc0)
                    ld_vec<T, VEC>(a.p, a.p_raw, (long)kk * a.pld + c, ok ? pav[b] : 0, pv[buf][u][b]);
                else
                    ld_vec<T, VEC>(a.p2, false, (long)kk * a.p2ld + (c - a.pc0), ok ? pav[b] : 0, pv[buf][u][b]);
            }
#pragma unroll
            for (int b = 0; b < JG; ++b) {
                const int i = a.stride * uu + tkh[b] - 1;
                int jj = a.stride * vv + tkw[b] - 1;
                if (a.circ && jj < 0) jj += a.Wq;  // only column -1 falls outside
                const bool in = ok && (unsigned)i < (unsigned)a.Hq && (unsigned)jj < (unsigned)a.Wq;
                ld_vec<T, VEC>(a.q, a.q_raw, (((long)n * a.Hq + (in ? i : 0)) * a.Wq + (in ? jj : 0)) * a.qld + tch[b],
                               in ? jav[b] : 0, qv[buf][u][b]);
            }
        }
    };
    int cur = 0;
    if (w_begin < w_end) load(0, w_begin);
    for (long k0 = w_begin; k0 < w_end; k0 += 4 * U) {
        if (k0 + 4 * U < w_end) load(cur ^ 1, k0 + 4 * U);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int bj = 0; bj < JG; ++bj)
#pragma unroll
                for (int ej = 0; ej < VEC; ++ej)
#pragma unroll
                    for (int bp = 0; bp < PG; ++bp)
#pragma unroll
                        for (int ep = 0; ep < VEC; ++ep)
                            acc[bj * VEC + ej][bp * VEC + ep] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                qv[cur][u][bj][ej], pv[cur][u][bp][ep], acc[bj * VEC + ej][bp * VEC + ep], 0, 0, 0);
        cur ^= 1;
    }

    // D row (4*kq + r) of block (bj*VEC + ej) <-> j; column r16 of block (bp*VEC + ep) <-> cp.
    float* out = a.partial + ((long)blockIdx.x * 4 + wave) * J * a.pc;
#pragma unroll
    for (int bj = 0; bj < JG; ++bj)
#pragma unroll
        for (int ej = 0; ej < VEC; ++ej)
#pragma unroll
            for (int bp = 0; bp < PG; ++bp)
#pragma unroll
                for (int ep = 0; ep < VEC; ++ep)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 4 * kq + r;
                        const int j = (jt * JB) * 16 + bj * 16 * VEC + VEC * row + ej;
                        const int cp = (pt * PB) * 16 + bp * 16 * VEC + VEC * r16 + ep;
                        if (j < J && cp < a.pc) out[(long)j * a.pc + cp] = acc[bj * VEC + ej][bp * VEC + ep][r];
                    }
}

// BF16 weight gradient (same D[j][cp] as wgrad_kernel) with both operands
// staged in LDS so that the reduction runs on v_mfma_f32_16x16x32_bf16,
// whose operands need 8 consecutive reduction pixels per lane.
// A workgroup walks strips of R rows x Wr columns of reduction pixels of one
// map (Wr a multiple of 8, R*Wr a multiple of 32). Per strip:
// * the gathered operand's rows 2u0-1 .. 2u0+2R-1 are staged as
//   Qs[c][row][kw][v] = Q[2u0-1+row][2v+kw-1][c] (zero outside), i.e. three
//   column views, one per kernel column kw, so that tap (kh, kw) of pixels
//   (u, v..v+7) is one aligned 16-byte read at row 2(u-u0)+kh;
// * the plain operand's channel tile [cp0, cp0+16 PB) is staged transposed,
//   Pt[cp][k], k = (u-u0)*Wr + v.
// Wave w owns the (tap, channel) row blocks w, w+4, ... and all PB column
// blocks, accumulating over the workgroup's strips; each workgroup writes
// its own partial tile (summed later in a fixed order).
// 8 x 8 transpose of 16-bit elements: in[i] holds elements 0..7 of row i,
// out[c] holds element c of rows 0..7.
__device__ __forceinline__ void transpose8x8_b16(const uint4 (&in)[8], uint4 (&out)[8]) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        uint32_t o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint4& r0 = in[2 * j];
            const uint4& r1 = in[2 * j + 1];
            const uint32_t a = (c >> 1) == 0 ? r0.x : (c >> 1) == 1 ? r0.y : (c >> 1) == 2 ? r0.z : r0.w;
            const uint32_t b = (c >> 1) == 0 ? r1.x : (c >> 1) == 1 ? r1.y : (c >> 1) == 2 ? r1.z : r1.w;
            o[j] = (c & 1) ? ((a >> 16) | (b & 0xffff0000u)) : ((a & 0xffffu) | (b << 16));
        }
        out[c] = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

struct WgradBArgs {
    const void* p; const void* p2;  // plain operand (bf16), channels [0, pc0) from p, the rest from p2
    int pc, pc0, pld, p2ld;
    const void* q;                  // gathered operand: bf16, or float32 when q_raw
    int q_raw, qc, qld;
    int nmaps, Hr, Wr, Hq, Wq;
    int circ;                       // 1: gathered column -1 is column Wq - 1 (circular width)
    int R, strips_per_map, total_strips, strips_per_chunk;
    int qcs;                        // LDS elements per staged channel (padded)
    float* partial;                 // [chunk][9*qc][pc]
};

template <int JBW, int PB, int QCP>
__global__ __launch_bounds__(256) void wgrad_bf16_kernel(WgradBArgs a) {
    extern __shared__ __align__(16) char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int Wr = a.Wr, R = a.R, K = R * Wr;
    const int qrows = 2 * R + 1;
    uint16_t* Qs = (uint16_t*)smem;
    uint16_t* Pt = Qs + (size_t)QCP * a.qcs;
    const int ptld = K + 8;
    const int cp0 = blockIdx.y * PB * 16;
    const int J = 9 * a.qc;

    // this lane's (tap, channel) row per owned row block
    int jc[JBW], jrow[JBW], jview[JBW];
    bool jv[JBW];
#pragma unroll
    for (int i = 0; i < JBW; ++i) {
        const int j = (wave + 4 * i) * 16 + r16;
        jv[i] = j < J;
        const int t = jv[i] ? j / a.qc : 0;
        jc[i] = jv[i] ? j - t * a.qc : 0;
        jrow[i] = t / 3;           // kh
        jview[i] = t - 3 * (t / 3); // kw
    }
    f4 acc[JBW][PB];
#pragma unroll
    for (int i = 0; i < JBW; ++i)
#pragma unroll
        for (int b = 0; b < PB; ++b) acc[i][b] = f4{0.f, 0.f, 0.f, 0.f};

    const int s_begin = blockIdx.x * a.strips_per_chunk;
    const int s_end = min(a.total_strips, s_begin + a.strips_per_chunk);
    for (int s = s_begin; s < s_end; ++s) {
        const int n = s / a.strips_per_map;
        const int u0 = (s - n * a.strips_per_map) * R;
        __syncthreads();  // the previous strip's LDS reads are done
        if constexpr (QCP == 8) {
            // few channels (raw float32 input or gradient): one thread per loaded pixel
            // ---- stage the gathered operand (three column views)
            const int ncols = 2 * Wr + 1;  // columns -1 .. 2 Wr - 1
            constexpr int CG = QCP / 8;
            for (int e = threadIdx.x; e < qrows * ncols * CG; e += 256) {
                const int cg = e % CG;
                const int rest = e / CG;
                const int colp = rest % ncols, row = rest / ncols;
                const int qi = 2 * u0 - 1 + row, qj = colp - 1;
                const int qs = (a.circ && qj < 0) ? qj + a.Wq : qj;  // column read
                float v8[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) v8[k] = 0.0f;
                if ((unsigned)qi < (unsigned)a.Hq && (unsigned)qs < (unsigned)a.Wq) {
                    const long base = (((long)n * a.Hq + qi) * a.Wq + qs) * a.qld + cg * 8;
                    if (a.q_raw) {
#pragma unroll
                        for (int k = 0; k < 8; ++k)
                            if (cg * 8 + k < a.qc) v8[k] = ((const float*)a.q)[base + k];
                    } else {
                        const uint4 w = *(const uint4*)((const uint16_t*)a.q + base);
                        const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            v8[2 * k] = bf16_to_f32((uint16_t)(ww[k] & 0xffffu));
                            v8[2 * k + 1] = bf16_to_f32((uint16_t)(ww[k] >> 16));
                        }
                    }
                }
                // column qj feeds view kw at v = (qj + 1 - kw) / 2 when that is an integer in [0, Wr)
#pragma unroll
                for (int kw = 0; kw < 3; ++kw) {
                    const int t2 = qj + 1 - kw;
                    if (t2 < 0 || (t2 & 1)) continue;
                    const int v = t2 >> 1;
                    if (v >= Wr) continue;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const __bf16 b = (__bf16)v8[k];
                        Qs[(size_t)(cg * 8 + k) * a.qcs + (row * 3 + kw) * Wr + v] = __builtin_bit_cast(uint16_t, b);
                    }
                }
            }
        } else {
            // ---- stage the gathered operand (three column views). A task reads 17
            // consecutive columns (16 b - 1 .. 16 b + 15) of one row for 8 channels
            // and writes, per view, 8 consecutive v of each channel (v in [8 b, 8 b + 8)):
            // view kw takes column 2 v + kw - 1, i.e. task column 2 i + kw. Each
            // view is an 8 x 8 transpose in registers and 8 16-byte LDS writes.
            constexpr int CG = QCP / 8;
            const int ncb = Wr / 8;
            for (int e = threadIdx.x; e < qrows * ncb * CG; e += 256) {
                const int cg = e % CG;
                const int rest = e / CG;
                const int cb = rest % ncb, row = rest / ncb;
                const int qi = 2 * u0 - 1 + row;
                const bool row_ok = (unsigned)qi < (unsigned)a.Hq;
                uint4 col[17];
#pragma unroll
                for (int t = 0; t < 17; ++t) {
                    int qj = 16 * cb - 1 + t;
                    if (a.circ && qj < 0) qj += a.Wq;
                    col[t] = make_uint4(0, 0, 0, 0);
                    if (row_ok && (unsigned)qj < (unsigned)a.Wq) {
                        const long base = (((long)n * a.Hq + qi) * a.Wq + qj) * a.qld + cg * 8;
                        if (a.q_raw) {
                            uint16_t h8[8];
#pragma unroll
                            for (int k = 0; k < 8; ++k) {
                                const float f = cg * 8 + k < a.qc ? ((const float*)a.q)[base + k] : 0.0f;
                                h8[k] = __builtin_bit_cast(uint16_t, (__bf16)f);
                            }
                            col[t] = make_uint4((uint32_t)h8[0] | ((uint32_t)h8[1] << 16),
                                                (uint32_t)h8[2] | ((uint32_t)h8[3] << 16),
                                                (uint32_t)h8[4] | ((uint32_t)h8[5] << 16),
                                                (uint32_t)h8[6] | ((uint32_t)h8[7] << 16));
                        } else {
                            col[t] = *(const uint4*)((const uint16_t*)a.q + base);
                        }
                    }
                }
#pragma unroll
                for (int kw = 0; kw < 3; ++kw) {
                    uint4 in[8], out[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) in[i] = col[2 * i + kw];
                    transpose8x8_b16(in, out);
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        *(uint4*)(Qs + (size_t)(cg * 8 + c) * a.qcs + (row * 3 + kw) * Wr + 8 * cb) = out[c];
                }
            }
        }
        // ---- stage the plain operand, transposed: a task reads 8 consecutive
        // reduction pixels (one row, Wr % 8 == 0) x 8 channels and writes 8
        // channels x 8 pixels
        for (int e = threadIdx.x; e < (K / 8) * PB * 2; e += 256) {
            const int cg = e % (PB * 2);
            const int k = (e / (PB * 2)) * 8;
            const int u = u0 + k / Wr, v = k % Wr;
            const int c = cp0 + cg * 8;
            uint4 in[8], out[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                in[i] = make_uint4(0, 0, 0, 0);
                if (u < a.Hr && c < a.pc) {
                    const long pix = ((long)n * a.Hr + u) * a.Wr + v + i;
                    in[i] = (c < a.pc0) ? *(const uint4*)((const uint16_t*)a.p + pix * a.pld + c)
                                        : *(const uint4*)((const uint16_t*)a.p2 + pix * a.p2ld + (c - a.pc0));
                }
            }
            transpose8x8_b16(in, out);
#pragma unroll
            for (int cc = 0; cc < 8; ++cc) *(uint4*)(Pt + (size_t)(cg * 8 + cc) * ptld + k) = out[cc];
        }
        __syncthreads();
        // ---- MFMAs over the strip
        for (int ks = 0; ks < K / 32; ++ks) {
            const int k0 = ks * 32 + 8 * g;
            const int ul = k0 / Wr, v0 = k0 - (k0 / Wr) * Wr;
            uint4 bfr[PB];
#pragma unroll
            for (int b = 0; b < PB; ++b) bfr[b] = *(const uint4*)(Pt + (size_t)(b * 16 + r16) * ptld + k0);
#pragma unroll
            for (int i = 0; i < JBW; ++i) {
                uint4 afr = make_uint4(0, 0, 0, 0);
                if (jv[i])
                    afr = *(const uint4*)(Qs + (size_t)jc[i] * a.qcs + ((2 * ul + jrow[i]) * 3 + jview[i]) * Wr + v0);
#pragma unroll
                for (int b = 0; b < PB; ++b)
                    acc[i][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, afr),
                                                                      __builtin_bit_cast(bf16x8, bfr[b]), acc[i][b],
                                                                      0, 0, 0);
            }
        }
    }
    // ---- partial tile: lane holds rows 4*g + r of row block (wave + 4 i), column r16 of block b
    float* out = a.partial + (long)blockIdx.x * J * a.pc;
#pragma unroll
    for (int i = 0; i < JBW; ++i)
#pragma unroll
        for (int b = 0; b < PB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = (wave + 4 * i) * 16 + 4 * g + r;
                const int cp = cp0 + b * 16 + r16;
                if (j < J && cp < a.pc) out[(long)j * a.pc + cp] = acc[i][b][r];
            }
}

// ---------------------------------------------------------------------------
// BF16 weight gradient with a 16-bit gathered operand (E2, E3, D3, D2), fed by
// LDS transpose reads. Both operands are staged per strip of R reduction rows
// as plain NHWC copies (16-byte chunks, pixel stride padded by 8 elements so
// that the 4 pixels one 16-lane group reads fall on different banks), and the
// MFMA operands (16 channels x 8 pixels per lane) come from ds_read_b64_tr_b16:
// within a group of 16 lanes, lane i's slot j is element i % 4 of the 8 bytes
// that lane 4 j + i / 4 addressed (measured on gfx950). So lane 4 j' + q of a
// group addresses channels [4 q, 4 q + 4) of the group's pixel j', and two
// reads (pixels 0-3 and 4-7) give each lane 8 pixels of one channel. The
// stride-2 gather of the 3 x 3 taps is per-lane address arithmetic; the halo
// column -1 reads a zero block. Rows and columns of the result, partial tiles
// and their reduction are those of wgrad_bf16_kernel.
struct WgradTArgs {
    const void* p; const void* p2;  // plain operand (bf16), channels [0, pc0) from p, the rest from p2
    int pc, pc0, pld, p2ld;
    const void* q;                  // gathered operand: bf16, or float32 with QR channels
    int qc, qld;                    // channels (QC, or QR when float32), elements per pixel
    int Hr, Wr, Hq, Wq;
    int circ;                       // 1: column -1 is column Wq - 1 of the same row (circular width)
    int R, strips_per_map, total_strips, strips_per_chunk;
    float* partial;                 // [chunk][9*qc][pc]
    const int32_t* roll;            // float32 x read augmented (AugMap of each map), or null
    const int32_t* flip;
};

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4i16 lds_v4i16;

__device__ __forceinline__ uint2 lds_read_tr16(const uint16_t* p) {
    const v4i16 v = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
        (lds_v4i16*)((__attribute__((address_space(3))) uint16_t*)p));
    return __builtin_bit_cast(uint2, v);
}

// QC: staged gathered channels (a multiple of 4; 16-row MFMA blocks of
// (tap, channel) rows may span several taps); QR > 0: the gathered operand
// is float32 with QR <= QC channels and dense pixels (qld == QR, rows of
// whole 16-byte chunks), rounded to bf16 (RNE) when staged and zero-padded
// to QC; it is staged as 16-byte chunks of the strip's rows (TG per
// thread), so every load is a full 16-byte one rather than QR scattered
// 4-byte loads per pixel.
template <int NW, int JBW, int PB, int QC, int TG, int TP, int QR>
__global__ __launch_bounds__(64 * NW) void wgrad_tr_kernel(WgradTArgs a) {
    constexpr int NT = 64 * NW;
    constexpr int GS = QC + 8;       // elements per staged gathered pixel
    constexpr int PS = PB * 16 + 8;  // elements per staged plain pixel
    constexpr int J = 9 * QC;
    extern __shared__ __align__(16) char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int jq = r16 >> 2, qq = r16 & 3;  // this lane's pixel and channel quad in a transpose read
    const int Wr = a.Wr, Wq = a.Wq, R = a.R, K = R * Wr;
    uint16_t* Gs = (uint16_t*)smem;
    uint16_t* Ps = Gs + (2 * R + 1) * Wq * GS;
    uint16_t* zero = Ps + R * Wr * PS;
    const int cp0 = blockIdx.y * PB * 16;
    if (threadIdx.x < 2) *(uint4*)(zero + 8 * threadIdx.x) = make_uint4(0, 0, 0, 0);
    if constexpr (QR > 0) {
        // the staging writes channels [0, QR) only: the pad channels stay zero
        for (int i = threadIdx.x; i < (2 * R + 1) * Wq * GS / 8; i += NT)
            *(uint4*)(Gs + 8 * i) = make_uint4(0, 0, 0, 0);
    }

    // per owned row block: LDS offset of this lane's gathered address relative
    // to the pixel (2 ul, 2 v) of the staged strip (its 4 rows are channels
    // c .. c + 3 of tap t), whether kw == 0, and whether the rows exist
    int aoff[JBW];
    bool alane[JBW], akw0[JBW];
#pragma unroll
    for (int i = 0; i < JBW; ++i) {
        const int rb = wave + NW * i;
        const int row = rb * 16 + 4 * qq;
        alane[i] = row < J;
        const int t = alane[i] ? row / QC : 0, c = alane[i] ? row % QC : 0;
        const int kh = t / 3, kw = t - 3 * (t / 3);
        akw0[i] = kw == 0;
        aoff[i] = (kh * Wq + kw - 1) * GS + c;
    }
    f4 acc[JBW][PB];
#pragma unroll
    for (int i = 0; i < JBW; ++i)
#pragma unroll
        for (int b = 0; b < PB; ++b) acc[i][b] = f4{0.f, 0.f, 0.f, 0.f};

    // Staging of a strip: gathered rows 2 u0 - 1 .. 2 u0 + 2 R - 1 (all
    // columns) and plain rows u0 .. u0 + R - 1 (channels [cp0, cp0 + 16 PB)),
    // 8 channels (float32: one 16-byte chunk) per task, at most TG and TP
    // tasks per thread. The next strip's loads are issued before this
    // strip's MFMAs and land in registers; they are written to LDS after the
    // MFMAs.
    constexpr int CGQ = QC / 8, CGP = PB * 2;
    const int ntq = QR ? (2 * R + 1) * Wq * QR / 4 : (2 * R + 1) * Wq * CGQ, ntp = K * CGP;
    const int rowf = Wq * QR;  // float32: floats per gathered row
    uint4 vq[QR ? 1 : TG], vp[TP];
    float4 vf[QR ? TG : 1];
    auto load_strip = [&](int s) {
        const int n = s / a.strips_per_map;
        const int u0 = (s - n * a.strips_per_map) * R;
        const long base = ((long)n * a.Hq + 2 * u0 - 1) * Wq * a.qld;
        bool gathered = false;
        if constexpr (QR == 7) {
            if (a.roll) {
                // augmented x: float f of a gathered row is channel f % 7 of
                // augmented column f / 7, read from its source column; the
                // normal's channels are turned (both read, one kept)
                const AugMap am = aug_map(a.roll, a.flip, n, Wq);
#pragma unroll
                for (int t = 0; t < TG; ++t) {
                    const int e = threadIdx.x + NT * t;
                    const int r = (4 * e) / rowf;
                    const int qi = 2 * u0 - 1 + r;
                    const bool ok = e < ntq && (unsigned)qi < (unsigned)a.Hq;
                    const float* xrow = (const float*)a.q + ((long)n * a.Hq + (ok ? qi : 0)) * rowf;
                    float f[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int fi = ok ? 4 * e + j - r * rowf : 0;
                        const int u = fi / 7, c = fi - 7 * (fi / 7);
                        const float* px = xrow + aug_src_col(am, u, Wq) * 7;
                        float nx = px[3], ny = px[4];
                        aug_normal(am, nx, ny);
                        const float v = px[c];
                        f[j] = ok ? (c == 3 ? nx : (c == 4 ? ny : v)) : 0.0f;
                    }
                    vf[t] = make_float4(f[0], f[1], f[2], f[3]);
                }
                gathered = true;
            }
        }
        if (gathered) {
            // (the augmented gather above)
        } else if constexpr (QR > 0) {
            // every lane loads (rows outside the map read the operand's first
            // chunk and are zeroed): a load under a per-lane condition would
            // make the compiler wait for all loads in flight
#pragma unroll
            for (int t = 0; t < TG; ++t) {
                const int e = threadIdx.x + NT * t;
                const int qi = 2 * u0 - 1 + (4 * e) / rowf;
                const bool ok = e < ntq && (unsigned)qi < (unsigned)a.Hq;
                const float4 v = *(const float4*)((const float*)a.q + (ok ? base + 4L * e : 0L));
                vf[t] = ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        } else {
#pragma unroll
            for (int t = 0; t < TG; ++t) {
                const int e = threadIdx.x + NT * t;
                const int cg = e % CGQ, pix = e / CGQ;
                const int row = pix / Wq;
                const int qi = 2 * u0 - 1 + row;
                const bool ok = e < ntq && (unsigned)qi < (unsigned)a.Hq;
                const long off = base + ((long)row * Wq + (pix - row * Wq)) * a.qld;
                vq[t] = make_uint4(0, 0, 0, 0);
                if (ok) vq[t] = *(const uint4*)((const uint16_t*)a.q + off + cg * 8);
            }
        }
#pragma unroll
        for (int t = 0; t < TP; ++t) {
            const int e = threadIdx.x + NT * t;
            const int cg = e % CGP, k = e / CGP;
            const int u = u0 + k / Wr, v = k - (k / Wr) * Wr;
            const int c = cp0 + cg * 8;
            vp[t] = make_uint4(0, 0, 0, 0);
            if (e < ntp && u < a.Hr && c < a.pc) {
                const long pix = ((long)n * a.Hr + u) * Wr + v;
                vp[t] = (c < a.pc0) ? *(const uint4*)((const uint16_t*)a.p + pix * a.pld + c)
                                    : *(const uint4*)((const uint16_t*)a.p2 + pix * a.p2ld + (c - a.pc0));
            }
        }
    };
    auto store_strip = [&]() {
#pragma unroll
        for (int t = 0; t < TG; ++t) {
            const int e = threadIdx.x + NT * t;
            if (e >= ntq) continue;
            if constexpr (QR > 0) {
                // float j of chunk e is channel (4 e + j) % QR of staged pixel (4 e + j) / QR
                const float f[4] = {vf[t].x, vf[t].y, vf[t].z, vf[t].w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = 4 * e + j, pix = k / QR;
                    Gs[pix * GS + (k - pix * QR)] = f32_to_bf16(f[j]);
                }
            } else {
                *(uint4*)(Gs + (e / CGQ) * GS + (e % CGQ) * 8) = vq[t];
            }
        }
#pragma unroll
        for (int t = 0; t < TP; ++t) {
            const int e = threadIdx.x + NT * t;
            if (e < ntp) *(uint4*)(Ps + (e / CGP) * PS + (e % CGP) * 8) = vp[t];
        }
    };

    const int s_begin = blockIdx.x * a.strips_per_chunk;
    const int s_end = min(a.total_strips, s_begin + a.strips_per_chunk);
    if (s_begin < s_end) load_strip(s_begin);
    for (int s = s_begin; s < s_end; ++s) {
        __syncthreads();  // the previous strip's LDS reads are done
        store_strip();
        __syncthreads();
        if (s + 1 < s_end) load_strip(s + 1);
        // ---- MFMAs: this lane group's 8 reduction pixels are (ul, v0 .. v0 + 7)
        for (int ks = 0; ks < K / 32; ++ks) {
            const int k0 = ks * 32 + 8 * g;
            const int ul = k0 / Wr, v0 = k0 - (k0 / Wr) * Wr;
            uint4 bfr[PB];
            const uint16_t* pb = Ps + (k0 + jq) * PS + 4 * qq;
#pragma unroll
            for (int b = 0; b < PB; ++b) {
                const uint2 lo = lds_read_tr16(pb + b * 16);
                const uint2 hi = lds_read_tr16(pb + 4 * PS + b * 16);
                bfr[b] = make_uint4(lo.x, lo.y, hi.x, hi.y);
            }
            const uint16_t* gb = Gs + (2 * ul * Wq + 2 * (v0 + jq)) * GS;
            const bool left = v0 + jq == 0;  // column -1 for kw == 0
            // (circular width: column -1 is the last column of the same staged row)
            // every owned row block's fragment is read before the first MFMA so
            // that the LDS latencies overlap; blocks past the last (tap,
            // channel) row read the zero block and their sums are never stored
            uint4 afr[JBW];
#pragma unroll
            for (int i = 0; i < JBW; ++i) {
                const uint16_t* lo_p = !alane[i] ? zero + 4 * qq
                                                 : (left && akw0[i] ? (a.circ ? gb + aoff[i] + Wq * GS : zero + 4 * qq)
                                                                    : gb + aoff[i]);
                const uint2 lo = lds_read_tr16(lo_p);
                const uint2 hi = lds_read_tr16(alane[i] ? gb + aoff[i] + 8 * GS : zero + 4 * qq);
                afr[i] = make_uint4(lo.x, lo.y, hi.x, hi.y);
            }
#pragma unroll
            for (int i = 0; i < JBW; ++i)
#pragma unroll
                for (int b = 0; b < PB; ++b)
                    acc[i][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, afr[i]),
                                                                      __builtin_bit_cast(bf16x8, bfr[b]), acc[i][b],
                                                                      0, 0, 0);
        }
    }
    // ---- partial tile: lane holds rows 4*g + r of row block (wave + NW i), column r16 of block b
    float* out = a.partial + (long)blockIdx.x * 9 * a.qc * a.pc;
#pragma unroll
    for (int i = 0; i < JBW; ++i)
#pragma unroll
        for (int b = 0; b < PB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int jp = (wave + NW * i) * 16 + 4 * g + r;  // (tap, staged channel) row
                const int t = jp / QC, c = jp - (jp / QC) * QC;
                const int cp = cp0 + b * 16 + r16;
                if (jp < J && c < a.qc && cp < a.pc) out[((long)t * a.qc + c) * a.pc + cp] = acc[i][b][r];
            }
}

// dW in the parameter layout from partial[chunk][j][cp] (fixed-order sum).
// q_is_cout: 1 for transposed-convolution layers (j = t*Cout + co, cp = ci),
// 0 for convolution layers (j = t*Cin + ci, cp = co).
static __global__ __launch_bounds__(1024) void wgrad_final_kernel(const float* partial, int nchunks, int qc,
                                                                  int pc, int q_is_cout, float scale, float* dw) {
    // 64 consecutive outputs per workgroup; wave w adds rows w, w + 16, ...
    // (coalesced 256-byte row segments), then wave sums are added in order.
    __shared__ float red[16][64];
    const long count = 9L * qc * pc;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long e = blockIdx.x * 64L + lane;
    float s = 0.0f;
    if (e < count) {
        int k = wv;
        for (; k + 48 < nchunks; k += 64) {
            const float a0 = partial[(long)k * count + e], a1 = partial[(long)(k + 16) * count + e];
            const float a2 = partial[(long)(k + 32) * count + e], a3 = partial[(long)(k + 48) * count + e];
            s += a0; s += a1; s += a2; s += a3;
        }
        for (; k < nchunks; k += 16) s += partial[(long)k * count + e];
    }
    red[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && e < count) {
        float v = 0.0f;
#pragma unroll
        for (int w = 0; w < 16; ++w) v += red[w][lane];
        const int cp = (int)(e % pc);
        const int j = (int)(e / pc);
        const int t = j / qc, c = j - t * qc;
        const int co = q_is_cout ? c : cp, ci = q_is_cout ? cp : c;
        const int cin = q_is_cout ? pc : qc;
        dw[((long)co * 9 + t) * cin + ci] = v * scale;
    }
}

// ------------------------------------------------------------------ Adam
// PyTorch's Adam: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// theta -= (lr / bc1) * m / (sqrt(v) / sqrt(bc2) + eps). The factors 1-b1,
// 1-b2, lr/bc1 and 1/sqrt(bc2) arrive precomputed in double precision and
// rounded once, as PyTorch forms them from Python floats.
static __global__ void adam_kernel(float* theta, float* m, float* v, const float* g, long count, float b1,
                                   float omb1, float b2, float omb2, float step_size, float inv_sqrt_bc2,
                                   float eps) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count;
         e += (long)gridDim.x * blockDim.x) {
        const float gv = g[e];
        const float mv = b1 * m[e] + omb1 * gv;
        const float vv = b2 * v[e] + omb2 * gv * gv;
        m[e] = mv;
        v[e] = vv;
        theta[e] -= step_size * mv / (sqrtf(vv) * inv_sqrt_bc2 + eps);
    }
}

// Copy the biases out of the flat parameter vector (fixed layer offsets).
static __global__ void gather_kernel(const float* src, const long* src_off, const int* len,
                              const int* dst_off, int nseg, float* dst) {
    const int s = blockIdx.x;
    if (s >= nseg) return;
    for (int e = threadIdx.x; e < len[s]; e += blockDim.x) dst[dst_off[s] + e] = src[src_off[s] + e];
}

}  // namespace drc
