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
    int gemm_mode;      // M_CONV or M_TCONV: the GEMM this pack feeds
    int transpose;
    int cin_eff;        // K elements per tap
    int rows_pad;       // GEMM rows, padded to 16
    int kstride;        // K elements per row
    int nphase;         // 1 (conv) or 4 (tconv)
    int prec;
    const float* scale; // FP8: device pointer to the weight scale, else null
    void* dst;
};

static __global__ void pack_weights_kernel(PackArgs a) {
    const long total = (long)a.nphase * a.rows_pad * a.kstride;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int k = (int)(e % a.kstride);
        const int row = (int)((e / a.kstride) % a.rows_pad);
        const int phase = (int)(e / ((long)a.kstride * a.rows_pad));
        const int t = k / a.cin_eff, c = k % a.cin_eff;
        const int rows = a.transpose ? a.cin : a.cout;
        const int chans = a.transpose ? a.cout : a.cin;
        float v = 0.0f;
        int kh, kw, ntaps;
        if (a.gemm_mode == M_CONV) {
            ntaps = 9;
            kh = t / 3;
            kw = t % 3;
        } else {
            const int py = phase >> 1, px = phase & 1;
            ntaps = (py ? 2 : 1) * (px ? 2 : 1);
            const int tr = px ? (t >> 1) : t, tc = px ? (t & 1) : 0;
            kh = py ? (tr == 0 ? 0 : 2) : 1;
            kw = px ? (tc == 0 ? 0 : 2) : 1;
        }
        if (row < rows && c < chans && t < ntaps) {
            const int co = a.transpose ? c : row;
            const int ci = a.transpose ? row : c;
            v = a.w[((co * 3 + kh) * 3 + kw) * a.cin + ci];
        }
        if (a.prec == P_F32)
            ((float*)a.dst)[e] = v;
        else if (a.prec == P_BF16)
            ((uint16_t*)a.dst)[e] = f32_to_bf16(v);
        else
            ((uint8_t*)a.dst)[e] = f32_to_e4m3(v * a.scale[0]);
    }
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
// block's fixed range, in double.
static __global__ __launch_bounds__(256) void l1_partial_kernel(const float* y, const float* t, long count,
                                                         long per_block, float dscale, float* dy,
                                                         double* partial) {
    __shared__ double red[256];
    const long b0 = blockIdx.x * per_block;
    const long b1 = min(count, b0 + per_block);
    double s = 0.0;
    for (long e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
        const float d = y[e] - t[e];
        s += fabs((double)d);
        dy[e] = (d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f)) * dscale;
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
// partial[b][c] = sum over the block's pixel range of g[pix][c].
template <typename TG>
__global__ __launch_bounds__(256) void bias_partial_kernel(const TG* g, int C, int cpow2, int ld,
                                                           long npix, long per_block, float* partial) {
    __shared__ float red[256];
    const int c = threadIdx.x % cpow2, po = threadIdx.x / cpow2, stride = 256 / cpow2;
    const long b0 = blockIdx.x * per_block, b1 = min(npix, b0 + per_block);
    float s = 0.0f;
    if (c < C)
        for (long p = b0 + po; p < b1; p += stride) s += to_float<TG>(g[p * ld + c]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = stride >> 1; o > 0; o >>= 1) {
        if (po < o) red[threadIdx.x] += red[threadIdx.x + o * cpow2];
        __syncthreads();
    }
    if (po == 0 && c < C) partial[(long)blockIdx.x * C + c] = red[threadIdx.x];
}

// out[e] = scale * sum_s partial[s][e], fixed order over s.
static __global__ void sum_partials_kernel(const float* partial, int nslots, long count, float scale,
                                    float* out) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count;
         e += (long)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int k = 0; k < nslots; ++k) s += partial[(long)k * count + e];
        out[e] = s * scale;
    }
}

// ------------------------------------------------------------------ weight gradient
// dW[co][kh][kw][ci] = sum_k G_t[k][co] * A_t[k][ci] with t = 3 kh + kw.
// Convolution layer: k runs over output pixels (n,p,q); G_t = g[n,p,q];
//   A_t = a[n, 2p+kh-1, 2q+kw-1] (0 outside).
// Transposed convolution layer: k runs over input pixels (n,i,j);
//   G_t = g[n, 2i+kh-1, 2j+kw-1] (0 outside); A_t = a[n,i,j].
// One workgroup handles one tap, one 64x64 (co, ci) tile and one range of
// k; each of its 4 waves takes every 4th group of 4 pixels and writes its
// own partial sum slot, reduced later in a fixed order. FP32 MFMA
// (16x16x4): lane l feeds pixel k0 + l/16 and the 4 channels
// 4 (l % 16) .. +3 of the tile, issuing one MFMA per (A element, B element)
// pair, so block (ja, jb) holds channels (4i + ja, 4i' + jb).
struct WgradArgs {
    const void* g; int gc; int gld; int g_raw;  // g_raw: g is float32
    Src s0, s1; int a_raw_c;                    // a_raw_c > 0: s0 float32 with that many channels
    int mode;                                   // layer kind: M_CONV or M_TCONV
    int nmaps, Hin, Win, Hout, Wout;
    int cout, cin;
    long per_block;                             // reduction pixels per workgroup
    int co_tiles, ci_tiles;
    float* partial;                             // [slot][9][cout][cin]
};

template <typename TG, typename TA>
__device__ __forceinline__ f4 ld4(const TG* p, int navail) {
    f4 v = {0.f, 0.f, 0.f, 0.f};
    if (navail >= 4) {
        v.x = to_float<TG>(p[0]); v.y = to_float<TG>(p[1]);
        v.z = to_float<TG>(p[2]); v.w = to_float<TG>(p[3]);
    } else {
        if (navail > 0) v.x = to_float<TG>(p[0]);
        if (navail > 1) v.y = to_float<TG>(p[1]);
        if (navail > 2) v.z = to_float<TG>(p[2]);
    }
    return v;
}

template <typename T>
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, r16 = lane & 15;
    const int t = blockIdx.y;
    const int kh = t / 3, kw = t % 3;
    const int cot = blockIdx.z % a.co_tiles, cit = blockIdx.z / a.co_tiles;
    const int co0 = cot * 64 + 4 * r16, ci0 = cit * 64 + 4 * r16;
    const long Kh = (a.mode == M_CONV) ? a.Hout : a.Hin;
    const long Kw = (a.mode == M_CONV) ? a.Wout : a.Win;
    const long K = (long)a.nmaps * Kh * Kw;
    const long k_begin = blockIdx.x * a.per_block;
    const long k_end = min(K, k_begin + a.per_block);

    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    for (long kb = k_begin + wave * 4; kb < k_end; kb += 16) {
        const long k = kb + kq;
        f4 gv = {0.f, 0.f, 0.f, 0.f}, av = {0.f, 0.f, 0.f, 0.f};
        if (k < k_end) {
            const int n = (int)(k / (Kh * Kw));
            const int rem = (int)(k - (long)n * Kh * Kw);
            const int u = rem / (int)Kw, v = rem % (int)Kw;
            long gpix = -1, apix = -1;
            if (a.mode == M_CONV) {
                gpix = k;
                const int i = 2 * u + kh - 1, j = 2 * v + kw - 1;
                if ((unsigned)i < (unsigned)a.Hin && (unsigned)j < (unsigned)a.Win)
                    apix = ((long)n * a.Hin + i) * a.Win + j;
            } else {
                apix = k;
                const int p = 2 * u + kh - 1, q = 2 * v + kw - 1;
                if ((unsigned)p < (unsigned)a.Hout && (unsigned)q < (unsigned)a.Wout)
                    gpix = ((long)n * a.Hout + p) * a.Wout + q;
            }
            if (gpix >= 0 && apix >= 0) {
                if (a.g_raw)
                    gv = ld4<float, float>((const float*)a.g + gpix * a.gld + co0, a.cout - co0);
                else
                    gv = ld4<T, T>((const T*)a.g + gpix * a.gld + co0, a.cout - co0);
                if (a.a_raw_c > 0) {
                    av = ld4<float, float>((const float*)a.s0.p + apix * a.s0.ld + ci0, a.cin - ci0);
                } else if (ci0 < a.s0.c) {
                    av = ld4<T, T>((const T*)a.s0.p + apix * a.s0.ld + ci0, a.s0.c - ci0);
                } else {
                    av = ld4<T, T>((const T*)a.s1.p + apix * a.s1.ld + (ci0 - a.s0.c),
                                   a.cin - ci0);
                }
            }
        }
        const float ga[4] = {gv.x, gv.y, gv.z, gv.w};
        const float aa[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[i], aa[j], acc[i][j], 0, 0, 0);
    }

    // D[row][col] of block (i, j): lane holds rows 4*kq + r, column r16.
    const long slot = (long)blockIdx.x * 4 + wave;
    float* out = a.partial + (slot * 9 + t) * (long)a.cout * a.cin;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = cot * 64 + 4 * (4 * kq + r) + i;
                const int ci = cit * 64 + 4 * r16 + j;
                if (co < a.cout && ci < a.cin) out[(long)co * a.cin + ci] = acc[i][j][r];
            }
}

// dW in parameter layout from partial[slot][t][co][ci]: fixed-order sum.
static __global__ void wgrad_final_kernel(const float* partial, int nslots, int cout, int cin, float scale,
                                   float* dw) {
    const long count = 9L * cout * cin;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count;
         e += (long)gridDim.x * blockDim.x) {
        // e indexes the partial layout [t][co][ci]
        const int ci = (int)(e % cin);
        const int co = (int)((e / cin) % cout);
        const int t = (int)(e / ((long)cin * cout));
        float s = 0.0f;
        for (int k = 0; k < nslots; ++k) s += partial[(long)k * count + e];
        dw[((long)co * 9 + t) * cin + ci] = s * scale;
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
