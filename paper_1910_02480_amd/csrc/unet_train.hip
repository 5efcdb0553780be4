// The paper's own network (Sec. 4.3 and Sec. 5) in its training form, FP32:
// batch normalisation with the statistics of the batch (and the running
// statistics updated with momentum 0.1), the mean L1 loss, the gradient of
// every trainable parameter (convolution weights and biases, batch-norm gamma
// and beta), and Adam on the trainable entries. The layer list and the flat
// parameter layout are the inference form's (unet.hip): per layer W
// [cout][3][3][cin] (or [cout][cin] for the 1x1 output), b, then gamma, beta,
// running mean, running variance for batch-normalised layers.
//
// Kernels (NHWC float32):
// * ut_conv_kernel: stride-1 3x3 convolution as an implicit GEMM on
//   v_mfma_f32_16x16x4_f32: rows = output channels (A = the weights read in
//   place from the parameter vector, K = (tap, channel) contiguous per row),
//   columns = pixels (B gathered from NHWC). A lane loads 4 consecutive K
//   values of its row and of its pixel as one 16-byte vector and feeds them
//   to 4 MFMAs (MFMA m takes element m, so the 4 lane groups cover K
//   positions 4 g + m). The data gradient is the same kernel on a
//   flipped, channel-transposed copy of the weights.
// * weight gradients: the autoencoder's FP32 weight-gradient kernel
//   (wgrad_kernel) with stride 1;
// * batch-norm statistics and its backward reductions: per-channel partial
//   sums in double per workgroup, added in a fixed order (deterministic);
// * max-pool (forward, and backward routing to the first maximum of each
//   window), bilinear 2x upsampling fused with the skip concatenation and its
//   adjoint (a gather over the high-resolution pixels that read each source
//   pixel), the 1x1 output convolution with ReLU and its gradients.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "drc_cae.h"
#include "aux_kernels.h"
#include "common.h"
#include "internal.h"

using namespace drc;

namespace {

constexpr int kLayersU = 15;
constexpr float kSlopeU = 0.01f;
constexpr double kEpsU = 1e-5;
constexpr double kMomentum = 0.1;

struct LayerU {
    int cin, cout, bn;
};
constexpr LayerU kU[kLayersU] = {
    {7, 64, 1},    {64, 64, 1},   {64, 128, 1},  {128, 128, 1}, {128, 256, 1},
    {256, 256, 1}, {256, 256, 1}, {256, 256, 1}, {512, 256, 1}, {256, 256, 1},
    {384, 128, 1}, {128, 128, 1}, {192, 64, 0},  {64, 64, 0},   {64, 3, 0},
};
// stage of each 3x3 layer: resolution divisor
constexpr int kDiv[kLayersU] = {1, 1, 2, 2, 4, 4, 8, 8, 4, 4, 2, 2, 1, 1, 1};

long woff_u(int l) {  // offset of layer l's weight in the flat vector
    long off = 0;
    for (int k = 0; k < l; ++k) {
        const LayerU& L = kU[k];
        off += (long)L.cout * L.cin * (k == 14 ? 1 : 9) + L.cout + (L.bn ? 4L * L.cout : 0);
    }
    return off;
}
long nparams_u() { return woff_u(kLayersU); }
long boff_u(int l) { return woff_u(l) + (long)kU[l].cout * kU[l].cin * (l == 14 ? 1 : 9); }

// ------------------------------------------------------------------ convolution
struct ConvF {
    const float* in;    // [npix][cin]
    const float* w;     // [cout][9][cin] (K contiguous per row)
    const float* bias;  // [cout] or null
    float* out;         // [npix][cout]
    int n, H, W, cin, cout;
};

template <int MT, int NPW>
__global__ __launch_bounds__(256) void ut_conv_kernel(ConvF a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const long npix = (long)a.n * a.H * a.W;
    const int rb0 = blockIdx.y * MT;
    long pbase[NPW];
    int py[NPW], px[NPW];
    bool pv[NPW];
#pragma unroll
    for (int j = 0; j < NPW; ++j) {
        const long p = ((long)blockIdx.x * 4 * NPW + wave * NPW + j) * 16 + r16;
        pv[j] = p < npix;
        const long pp = pv[j] ? p : 0;
        px[j] = (int)(pp % a.W);
        py[j] = (int)((pp / a.W) % a.H);
        pbase[j] = pp;
    }
    f4 acc[MT][NPW];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NPW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    const int chunks = (a.cin + 15) / 16;   // 16 channels per step
    const int steps = 9 * chunks;
    const long krow = 9L * a.cin;
    // step s: tap t = s / chunks, channels c0 + 4 g .. + 4 of it
    auto load = [&](int s, float4 (&af)[MT], float4 (&bf)[NPW]) {
        const int t = s / chunks, c = (s - t * chunks) * 16 + 4 * g;
        const bool cok = c < a.cin;
        const int dy = t / 3 - 1, dx = t - 3 * (t / 3) - 1;
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const int row = (rb0 + i) * 16 + r16;
            const float* src = a.w + (long)row * krow + (long)t * a.cin + (cok ? c : 0);
            const float4 v = *(const float4*)src;
            af[i] = cok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int j = 0; j < NPW; ++j) {
            const int yy = py[j] + dy, xx = px[j] + dx;
            const bool ok = pv[j] && cok && (unsigned)yy < (unsigned)a.H && (unsigned)xx < (unsigned)a.W;
            const float* src = a.in + (ok ? (pbase[j] + (long)dy * a.W + dx) * a.cin + c : 0);
            const float4 v = *(const float4*)src;
            bf[j] = ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    float4 af[MT], bf[NPW];
    load(0, af, bf);
    for (int s = 0; s < steps; ++s) {
        float4 an[MT], bn[NPW];
        load(min(s + 1, steps - 1), an, bn);  // unconditional: the last step reloads its own operands
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NPW; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i].x, bf[j].x, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i].y, bf[j].y, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i].z, bf[j].z, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i].w, bf[j].w, acc[i][j], 0, 0, 0);
            }
#pragma unroll
        for (int i = 0; i < MT; ++i) af[i] = an[i];
#pragma unroll
        for (int j = 0; j < NPW; ++j) bf[j] = bn[j];
    }
    // lane holds rows 16 rb + 4 g .. + 3 of pixel 16 pb + r16
#pragma unroll
    for (int j = 0; j < NPW; ++j) {
        if (!pv[j]) continue;
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const int c0 = (rb0 + i) * 16 + 4 * g;
            float4 v = make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
            if (a.bias) {
                v.x += a.bias[c0];
                v.y += a.bias[c0 + 1];
                v.z += a.bias[c0 + 2];
                v.w += a.bias[c0 + 3];
            }
            *(float4*)(a.out + pbase[j] * a.cout + c0) = v;
        }
    }
}

// W'[ci][t][co] = W[co][8 - t][ci] (the data gradient's weights); ci padded to
// cin_pad rows (zero rows).
__global__ void ut_flip_kernel(const float* w, float* wt, int cin, int cin_pad, int cout) {
    const long total = (long)cin_pad * 9 * cout;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int co = (int)(e % cout);
        const long r = e / cout;
        const int t = (int)(r % 9), ci = (int)(r / 9);
        wt[e] = ci < cin ? w[((long)co * 9 + (8 - t)) * cin + ci] : 0.0f;
    }
}

// x [npix][7] -> [npix][8] (channel 7 = 0)
__global__ void ut_pad_x_kernel(const float* x, float* x8, long npix) {
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < npix; p += (long)gridDim.x * blockDim.x) {
        float4 lo, hi;
        lo.x = x[7 * p]; lo.y = x[7 * p + 1]; lo.z = x[7 * p + 2]; lo.w = x[7 * p + 3];
        hi.x = x[7 * p + 4]; hi.y = x[7 * p + 5]; hi.z = x[7 * p + 6]; hi.w = 0.0f;
        ((float4*)x8)[2 * p] = lo;
        ((float4*)x8)[2 * p + 1] = hi;
    }
}

// ------------------------------------------------------------------ per-channel reductions
// partial[b][0..C) = sum over the block's pixels of f(p, c), in double; the
// block's pixels are [b * per, (b + 1) * per). A thread takes channel
// c = tid % C and pixels tid / C, tid / C + 256 / C, ...
// MODE 0: v = z; MODE 1: v = (z - mean)^2; MODE 2: dq and dq * xhat (two
// partial rows), with dq = da * lrelu'(a).
struct RedArgs {
    const float* z;
    const float* a;      // MODE 2: the activation (its sign gives the LeakyReLU branch)
    const float* da;     // MODE 2
    const float* mean;   // MODE 1, 2
    const float* rstd;   // MODE 2
    double* partial;     // [blocks][rows * C]
    long npix, per;
    int C;
};

template <int MODE>
__global__ __launch_bounds__(256) void ut_reduce_kernel(RedArgs r) {
    __shared__ double red[2][256];
    const int C = r.C, tid = threadIdx.x;
    const int c = tid % C, lanes = 256 / C, sub = tid / C;
    const long p0 = blockIdx.x * r.per, p1 = min(r.npix, p0 + r.per);
    double s0 = 0.0, s1 = 0.0;
    if (sub < lanes) {
        for (long p = p0 + sub; p < p1; p += lanes) {
            const long e = p * C + c;
            if constexpr (MODE == 0) {
                s0 += (double)r.z[e];
            } else if constexpr (MODE == 1) {
                const double d = (double)r.z[e] - (double)r.mean[c];
                s0 += d * d;
            } else {
                const float dq = r.da[e] * (r.a[e] > 0.0f ? 1.0f : kSlopeU);
                const float xh = (r.z[e] - r.mean[c]) * r.rstd[c];
                s0 += (double)dq;
                s1 += (double)dq * (double)xh;
            }
        }
    }
    red[0][tid] = s0;
    red[1][tid] = s1;
    __syncthreads();
    if (tid < C) {
        double t0 = 0.0, t1 = 0.0;
        for (int k = 0; k < lanes; ++k) {  // fixed order
            t0 += red[0][k * C + tid];
            t1 += red[1][k * C + tid];
        }
        const int rows = MODE == 2 ? 2 : 1;
        r.partial[(long)blockIdx.x * rows * C + tid] = t0;
        if (MODE == 2) r.partial[(long)blockIdx.x * rows * C + C + tid] = t1;
    }
}

// Sums the block partials of each channel in block order. MODE 0: mean;
// MODE 1: var -> rstd and the running statistics; MODE 2: dgamma, dbeta and
// the dz coefficients k1 = mean(dq), k2 = mean(dq xhat).
struct FinArgs {
    const double* partial;
    int blocks, C;
    long M;
    float* mean;       // MODE 0 out, MODE 1 in
    float* rstd;       // MODE 1 out
    float* run_mean;   // MODE 1: running statistics, updated in place
    float* run_var;
    const float* bmean;  // MODE 1: the batch mean (double precision source kept as float)
    float* dgamma;     // MODE 2 out
    float* dbeta;
    float* k1;         // MODE 2 out
    float* k2;
    double* dmean;     // MODE 0: the mean in double (for MODE 1)
};

template <int MODE>
__global__ void ut_finish_kernel(FinArgs f) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= f.C) return;
    const int rows = MODE == 2 ? 2 : 1;
    double s0 = 0.0, s1 = 0.0;
    for (int b = 0; b < f.blocks; ++b) {
        s0 += f.partial[(long)b * rows * f.C + c];
        if (MODE == 2) s1 += f.partial[(long)b * rows * f.C + f.C + c];
    }
    const double M = (double)f.M;
    if constexpr (MODE == 0) {
        f.mean[c] = (float)(s0 / M);
        f.dmean[c] = s0 / M;
    } else if constexpr (MODE == 1) {
        const double var = s0 / M;
        f.rstd[c] = (float)(1.0 / sqrt(var + kEpsU));
        f.run_mean[c] = (float)((1.0 - kMomentum) * (double)f.run_mean[c] + kMomentum * f.dmean[c]);
        f.run_var[c] = (float)((1.0 - kMomentum) * (double)f.run_var[c] + kMomentum * var * M / (M - 1.0));
    } else {
        f.dbeta[c] = (float)s0;
        f.dgamma[c] = (float)s1;
        f.k1[c] = (float)(s0 / M);
        f.k2[c] = (float)(s1 / M);
    }
}

// a = LeakyReLU(gamma (z - mean) rstd + beta), or LeakyReLU(z) without batch norm.
__global__ void ut_bn_act_kernel(const float* z, const float* mean, const float* rstd, const float* gamma,
                                 const float* beta, float* a, long count, int C) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        float q = z[e];
        if (gamma) q = fmaf(gamma[c], (q - mean[c]) * rstd[c], beta[c]);
        a[e] = q > 0.0f ? q : kSlopeU * q;
    }
}

// dz from da: batch norm: gamma rstd (dq - k1 - xhat k2); without: dq.
__global__ void ut_bn_bwd_kernel(const float* z, const float* a, const float* da, const float* mean,
                                 const float* rstd, const float* gamma, const float* k1, const float* k2, float* dz,
                                 long count, int C) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const float dq = da[e] * (a[e] > 0.0f ? 1.0f : kSlopeU);
        if (gamma) {
            const float xh = (z[e] - mean[c]) * rstd[c];
            dz[e] = gamma[c] * rstd[c] * (dq - k1[c] - xh * k2[c]);
        } else {
            dz[e] = dq;
        }
    }
}

// ------------------------------------------------------------------ pooling, upsampling
__global__ void ut_pool_kernel(const float* in, float* out, int n, int H, int W, int C) {
    const long total = (long)n * (H / 2) * (W / 2) * C;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const long q = e / C;
        const int x = (int)(q % (W / 2));
        const long r = q / (W / 2);
        const int y = (int)(r % (H / 2));
        const long m = r / (H / 2);
        const float* p = in + ((m * H + 2 * y) * W + 2 * x) * C + c;
        out[e] = fmaxf(fmaxf(p[0], p[C]), fmaxf(p[(long)W * C], p[(long)W * C + C]));
    }
}

// d_in (full resolution) += the pooled gradient at the first maximum of each window.
__global__ void ut_pool_bwd_kernel(const float* in, const float* dout, float* din, int n, int H, int W, int C) {
    const long total = (long)n * H * W * C;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const long q = e / C;
        const int x = (int)(q % W);
        const long r = q / W;
        const int y = (int)(r % H);
        const long m = r / H;
        const int y0 = y & ~1, x0 = x & ~1;
        const float* p = in + ((m * H + y0) * W + x0) * C + c;
        const float v[4] = {p[0], p[C], p[(long)W * C], p[(long)W * C + C]};
        int k = 0;
        float best = v[0];
#pragma unroll
        for (int i = 1; i < 4; ++i)
            if (v[i] > best) {
                best = v[i];
                k = i;
            }
        const int mine = 2 * (y - y0) + (x - x0);
        if (k == mine) din[e] += dout[((m * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c];
    }
}

// Bilinear 2x source coordinate of output index o (half-pixel centres,
// clamped): rows i0, i1 and the weight f of i1.
__device__ __forceinline__ void up_src(int o, int size, int& i0, int& i1, float& f) {
    const float s = fmaxf((o + 0.5f) * 0.5f - 0.5f, 0.0f);
    i0 = min((int)s, size - 1);
    i1 = min(i0 + 1, size - 1);
    f = s - (float)i0;
}

// out [n, 2h, 2w, Cl + Cs] = [upsample(low) | skip]
__global__ void ut_upcat_kernel(const float* low, const float* skip, float* out, int n, int h, int w, int Cl,
                                int Cs) {
    const int C = Cl + Cs, H = 2 * h, W = 2 * w;
    const long total = (long)n * H * W * C;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const long q = e / C;
        const int x = (int)(q % W);
        const long r = q / W;
        const int y = (int)(r % H);
        const long m = r / H;
        if (c >= Cl) {
            out[e] = skip[q * Cs + (c - Cl)];
            continue;
        }
        int r0, r1, c0, c1;
        float fr, fc;
        up_src(y, h, r0, r1, fr);
        up_src(x, w, c0, c1, fc);
        const float* b = low + m * h * w * Cl + c;
        const float top = b[((long)r0 * w + c0) * Cl] * (1.0f - fc) + b[((long)r0 * w + c1) * Cl] * fc;
        const float bot = b[((long)r1 * w + c0) * Cl] * (1.0f - fc) + b[((long)r1 * w + c1) * Cl] * fc;
        out[e] = top * (1.0f - fr) + bot * fr;
    }
}

// The adjoint of ut_upcat_kernel's upsampling part: dlow[m, i, j, c] = sum of
// dcat[m, o, q, c] times the weight with which output (o, q) read (i, j);
// only outputs o in [2i - 1, 2i + 2] (and likewise q) can read row i.
// dskip = dcat[..., Cl:].
__global__ void ut_upcat_bwd_kernel(const float* dcat, float* dlow, float* dskip, int n, int h, int w, int Cl,
                                    int Cs) {
    const int C = Cl + Cs, H = 2 * h, W = 2 * w;
    const long tl = (long)n * h * w * Cl;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tl; e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % Cl);
        const long q = e / Cl;
        const int j = (int)(q % w);
        const long r = q / w;
        const int i = (int)(r % h);
        const long m = r / h;
        float wr[4], wc[4];
        int orow[4], ocol[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int o = 2 * i - 1 + k, u = 2 * j - 1 + k;
            orow[k] = o;
            ocol[k] = u;
            wr[k] = 0.0f;
            wc[k] = 0.0f;
            if (o >= 0 && o < H) {
                int a0, a1;
                float f;
                up_src(o, h, a0, a1, f);
                wr[k] = (a0 == i ? 1.0f - f : 0.0f) + (a1 == i ? f : 0.0f);
            }
            if (u >= 0 && u < W) {
                int b0, b1;
                float f;
                up_src(u, w, b0, b1, f);
                wc[k] = (b0 == j ? 1.0f - f : 0.0f) + (b1 == j ? f : 0.0f);
            }
        }
        float s = 0.0f;
#pragma unroll
        for (int ka = 0; ka < 4; ++ka) {
            if (wr[ka] == 0.0f) continue;
            float row = 0.0f;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
                if (wc[kb] != 0.0f) row += wc[kb] * dcat[((m * H + orow[ka]) * W + ocol[kb]) * C + c];
            s += wr[ka] * row;
        }
        dlow[e] = s;
    }
    const long ts = (long)n * H * W * Cs;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < ts; e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % Cs);
        dskip[e] = dcat[(e / Cs) * C + Cl + c];
    }
}

// ------------------------------------------------------------------ output 1x1 convolution
// y = relu(d1 W^T + b) (3 outputs per pixel), and the pre-activation sign kept in y.
__global__ void ut_out_kernel(const float* d1, const float* w, const float* b, float* y, long npix) {
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < npix; p += (long)gridDim.x * blockDim.x) {
        float s[3] = {b[0], b[1], b[2]};
        const float* x = d1 + p * 64;
        for (int c = 0; c < 64; c += 4) {
            const float4 v = *(const float4*)(x + c);
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                const float* wr = w + o * 64 + c;
                s[o] = fmaf(wr[0], v.x, s[o]);
                s[o] = fmaf(wr[1], v.y, s[o]);
                s[o] = fmaf(wr[2], v.z, s[o]);
                s[o] = fmaf(wr[3], v.w, s[o]);
            }
        }
#pragma unroll
        for (int o = 0; o < 3; ++o) y[3 * p + o] = fmaxf(s[o], 0.0f);
    }
}

// g = dL/dy masked by y > 0 (in place), dd1 = g W; block partials of
// dW_out = sum g^T d1 (3 x 64) and db_out = sum g (3), per workgroup in double.
__global__ __launch_bounds__(256) void ut_out_bwd_kernel(const float* y, float* g, const float* d1,
                                                         const float* w, float* dd1, double* partial, long npix,
                                                         long per) {
    __shared__ double red[256];
    const long p0 = blockIdx.x * per, p1 = min(npix, p0 + per);
    // dd1 and the mask: one thread per pixel
    for (long p = p0 + threadIdx.x; p < p1; p += 256) {
        float gg[3];
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            gg[o] = y[3 * p + o] > 0.0f ? g[3 * p + o] : 0.0f;
            g[3 * p + o] = gg[o];
        }
        for (int c = 0; c < 64; ++c) dd1[p * 64 + c] = gg[0] * w[c] + gg[1] * w[64 + c] + gg[2] * w[128 + c];
    }
    __syncthreads();
    // 195 sums (3 x 64 weights, 3 biases): thread k < 195 accumulates entry k over the block's pixels
    const int k = threadIdx.x;
    double s = 0.0;
    if (k < 195) {
        for (long p = p0; p < p1; ++p) {
            const float gv = g[3 * p + (k < 192 ? k / 64 : k - 192)];
            s += (double)gv * (k < 192 ? (double)d1[p * 64 + (k % 64)] : 1.0);
        }
    }
    red[k] = s;
    __syncthreads();
    if (k < 195) partial[blockIdx.x * 195L + k] = red[k];
}

__global__ void ut_out_bwd_final_kernel(const double* partial, int blocks, float* dw, float* db) {
    const int k = threadIdx.x;
    if (k >= 195) return;
    double s = 0.0;
    for (int b = 0; b < blocks; ++b) s += partial[(long)b * 195 + k];
    if (k < 192) dw[k] = (float)s;
    else db[k - 192] = (float)s;
}

// ------------------------------------------------------------------ host side
__global__ void ut_pad_w_kernel(const float* w7, float* w8, int cout) {
    const long total = (long)cout * 9 * 8;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % 8);
        const long r = e / 8;  // co * 9 + t
        w8[e] = c < 7 ? w7[r * 7 + c] : 0.0f;
    }
}

__global__ void ut_fill_kernel(float* p, long count, float v) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) p[e] = v;
}

unsigned grid_for(long count, int per_thread = 1) {
    const long g = (count / per_thread + 255) / 256;
    return (unsigned)std::max(1L, std::min(g, 16384L));
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// Workspace layout of one training step (bytes from the start).
struct TrainLayout {
    size_t x8, z[14], a[14], p1, p2, p3, c3, c2, c1, y, mean[14], rstd[14], dmean, red, g, bufA, bufB, bufC, ds1,
        ds2, ds3, wt, w8, part, dparams, lossp, outp, colp, k1, k2, total;
    long P[4];  // pixels at H, H/2, H/4, H/8
};

constexpr int kRedBlocks = 256;   // per-channel reductions: workgroups
constexpr int kOutBlocks = 256;   // output-layer gradient: workgroups

// Weight-gradient schedule of a stride-1 3x3 layer (the generic FP32
// kernel's tiles; at most 256 chunks and 16 M floats of partial tiles).
struct WPlanU {
    int JB, PB, VEC, jtiles, ptiles, nchunks;
    long per_block;
    size_t partial_floats;
};
WPlanU wplan_u(int qc, int pc, long K) {
    WPlanU w;
    const int jblocks = (9 * qc + 15) / 16, pblocks = (pc + 15) / 16;
    w.JB = jblocks >= 4 ? 4 : 2;
    w.PB = (w.JB == 4 && pblocks <= 2) ? 2 : 4;
    w.VEC = (w.JB == 4 && w.PB == 4 && qc % 4 == 0 && pc % 4 == 0) ? 4 : 1;
    w.jtiles = (jblocks + w.JB - 1) / w.JB;
    w.ptiles = (pblocks + w.PB - 1) / w.PB;
    const long per_chunk = 4L * 9 * qc * pc;
    long want = std::max(1L, std::min(256L, 2048L / (w.jtiles * w.ptiles)));
    want = std::max(1L, std::min(want, (16L << 20) / per_chunk));
    long pb = (K + want - 1) / want;
    pb = std::max(64L, (pb + 15) / 16 * 16);
    w.per_block = pb;
    w.nchunks = (int)((K + pb - 1) / pb);
    w.partial_floats = (size_t)w.nchunks * per_chunk;
    return w;
}

TrainLayout train_layout(int n, int H, int W) {
    TrainLayout L;
    for (int k = 0; k < 4; ++k) L.P[k] = (long)n * (H >> k) * (W >> k);
    auto px = [&](int l) { return L.P[kDiv[l] == 1 ? 0 : kDiv[l] == 2 ? 1 : kDiv[l] == 4 ? 2 : 3]; };
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        const size_t o = cur;
        cur += al256(bytes);
        return o;
    };
    const size_t F = sizeof(float);
    L.x8 = take(L.P[0] * 8 * F);
    for (int l = 0; l < 14; ++l) {
        L.z[l] = take(px(l) * kU[l].cout * F);
        L.a[l] = take(px(l) * kU[l].cout * F);
        L.mean[l] = take(kU[l].cout * F);
        L.rstd[l] = take(kU[l].cout * F);
    }
    L.p1 = take(L.P[1] * 64 * F);
    L.p2 = take(L.P[2] * 128 * F);
    L.p3 = take(L.P[3] * 256 * F);
    L.c3 = take(L.P[2] * 512 * F);
    L.c2 = take(L.P[1] * 384 * F);
    L.c1 = take(L.P[0] * 192 * F);
    L.y = take(L.P[0] * 3 * F);
    L.dmean = take(256 * sizeof(double));
    L.red = take((size_t)kRedBlocks * 2 * 256 * sizeof(double));
    L.g = take(L.P[0] * 3 * F);
    size_t big = 0;  // largest per-layer gradient (output side or input side)
    for (int l = 0; l < 14; ++l) big = std::max(big, (size_t)px(l) * std::max(kU[l].cin, kU[l].cout));
    L.bufA = take(big * F);
    L.bufB = take(big * F);
    L.bufC = take(big * F);
    L.ds1 = take(L.P[0] * 64 * F);
    L.ds2 = take(L.P[1] * 128 * F);
    L.ds3 = take(L.P[2] * 256 * F);
    L.wt = take(512L * 9 * 256 * F);
    L.w8 = take(64L * 9 * 8 * F);
    size_t part = 0;
    for (int l = 0; l < 14; ++l) part = std::max(part, wplan_u(kU[l].cin, kU[l].cout, px(l)).partial_floats);
    L.part = take(part * F);
    L.dparams = take((size_t)nparams_u() * F);
    L.lossp = take(((L.P[0] * 3 + kLossPerBlock - 1) / kLossPerBlock) * sizeof(double));
    L.outp = take((size_t)kOutBlocks * 195 * sizeof(double));
    L.colp = take(384L * 256 * F);
    L.k1 = take(256 * F);
    L.k2 = take(256 * F);
    L.total = cur;
    return L;
}

drc_status conv_u(const float* in, const float* w, const float* bias, float* out, int n, int H, int W, int cin,
                  int cout, hipStream_t s) {
    ConvF a{in, w, bias, out, n, H, W, cin, cout};
    const long npix = (long)n * H * W;
    constexpr int NPW = 2;
    const int MT = cout % 64 == 0 ? 4 : (cout % 32 == 0 ? 2 : 1);
    dim3 grid((unsigned)((npix + 64 * NPW - 1) / (64 * NPW)), (unsigned)(cout / 16 / MT));
    if (MT == 4) hipLaunchKernelGGL((ut_conv_kernel<4, NPW>), grid, dim3(256), 0, s, a);
    else if (MT == 2) hipLaunchKernelGGL((ut_conv_kernel<2, NPW>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((ut_conv_kernel<1, NPW>), grid, dim3(256), 0, s, a);
    return check_launch("unet train: conv");
}

// Per-channel sums over npix pixels of a [npix][C] tensor (kRedBlocks partials).
template <int MODE>
void reduce_u(RedArgs r, hipStream_t s) {
    r.per = (r.npix + kRedBlocks - 1) / kRedBlocks;
    hipLaunchKernelGGL((ut_reduce_kernel<MODE>), dim3(kRedBlocks), dim3(256), 0, s, r);
}

}  // namespace

extern "C" drc_status drc_unet_train_workspace_size(int n, int H, int W, size_t* bytes) {
    if (!bytes) return drc_fail(DRC_ERR_INVALID_ARG, "unet train workspace: bytes is NULL");
    if (n < 2 || H < 8 || W < 8 || H % 8 || W % 8 || (long)n * H * W > (1L << 26))
        return drc_fail(DRC_ERR_SHAPE, "unet train: n = %d (>= 2), H = %d, W = %d (multiples of 8)", n, H, W);
    *bytes = train_layout(n, H, W).total;
    return DRC_OK;
}

extern "C" drc_status drc_unet_train_act_offsets(int n, int H, int W, int64_t offsets[14]) {
    if (!offsets) return drc_fail(DRC_ERR_INVALID_ARG, "unet train offsets: offsets is NULL");
    size_t need;
    const drc_status st = drc_unet_train_workspace_size(n, H, W, &need);
    if (st != DRC_OK) return st;
    const TrainLayout L = train_layout(n, H, W);
    for (int l = 0; l < 14; ++l) offsets[l] = (int64_t)L.a[l];
    return DRC_OK;
}

extern "C" drc_status drc_unet_train_step(float* d_params, float* d_m, float* d_v, int64_t t,
                                          const drc_adam_cfg* adam, const float* d_x, const float* d_target,
                                          float* d_loss, float* d_dparams, float* d_y, int n, int H, int W,
                                          void* d_ws, size_t ws_bytes, void* stream) {
    const char* who = "unet train";
    size_t need = 0;
    drc_status st = drc_unet_train_workspace_size(n, H, W, &need);
    if (st != DRC_OK) return st;
    if ((st = check_ptr(who, "d_params", d_params, 16, false)) != DRC_OK) return st;
    if ((st = check_ptr(who, "d_m", d_m, 16, false)) != DRC_OK) return st;
    if ((st = check_ptr(who, "d_v", d_v, 16, false)) != DRC_OK) return st;
    if ((st = check_ptr(who, "d_x", d_x, 4, false)) != DRC_OK) return st;
    if ((st = check_ptr(who, "d_target", d_target, 16, false)) != DRC_OK) return st;
    if ((st = check_ptr(who, "d_loss", d_loss, 4, false)) != DRC_OK) return st;
    if ((st = check_ptr(who, "d_dparams", d_dparams, 4, true)) != DRC_OK) return st;
    if ((st = check_ptr(who, "d_y", d_y, 16, true)) != DRC_OK) return st;
    if ((st = check_ptr(who, "d_ws", d_ws, 256, false)) != DRC_OK) return st;
    if (!adam) return drc_fail(DRC_ERR_INVALID_ARG, "%s: adam is NULL", who);
    if (!(adam->lr > 0) || !(adam->beta1 >= 0 && adam->beta1 < 1) || !(adam->beta2 >= 0 && adam->beta2 < 1) ||
        !(adam->eps >= 0))
        return drc_fail(DRC_ERR_INVALID_ARG, "%s: bad Adam hyper-parameters", who);
    if (t < 1) return drc_fail(DRC_ERR_INVALID_ARG, "%s: t = %lld (must be >= 1)", who, (long long)t);
    if (ws_bytes < need) return drc_fail(DRC_ERR_WORKSPACE, "%s: workspace %zu < %zu bytes", who, ws_bytes, need);

    hipStream_t s = (hipStream_t)stream;
    const TrainLayout L = train_layout(n, H, W);
    char* ws = (char*)d_ws;
    auto F = [&](size_t off) { return (float*)(ws + off); };
    auto hw = [&](int l, int& h, int& w) {
        h = H / kDiv[l];
        w = W / kDiv[l];
    };
    auto px = [&](int l) { return (long)n * (H / kDiv[l]) * (W / kDiv[l]); };
    float* dp = d_dparams ? d_dparams : F(L.dparams);
    float* y = d_y ? d_y : F(L.y);

    // ---------------- forward (batch statistics)
    hipLaunchKernelGGL(ut_pad_x_kernel, dim3(grid_for(L.P[0])), dim3(256), 0, s, d_x, F(L.x8), L.P[0]);
    hipLaunchKernelGGL(ut_pad_w_kernel, dim3(grid_for(64 * 72)), dim3(256), 0, s, d_params + woff_u(0), F(L.w8), 64);
    const float* in = F(L.x8);
    for (int l = 0; l < 14; ++l) {
        int h, w;
        hw(l, h, w);
        const int cin = l == 0 ? 8 : kU[l].cin, cout = kU[l].cout;
        const float* wt = l == 0 ? F(L.w8) : d_params + woff_u(l);
        const float* b = d_params + boff_u(l);
        float* z = F(L.z[l]);
        float* a = F(L.a[l]);
        if ((st = conv_u(in, wt, b, z, n, h, w, cin, cout, s)) != DRC_OK) return st;
        const long cnt = px(l) * cout;
        if (kU[l].bn) {
            float* gamma = d_params + boff_u(l) + cout;
            RedArgs r{};
            r.z = z;
            r.npix = px(l);
            r.C = cout;
            r.partial = (double*)(ws + L.red);
            reduce_u<0>(r, s);
            FinArgs f{};
            f.partial = r.partial;
            f.blocks = kRedBlocks;
            f.C = cout;
            f.M = px(l);
            f.mean = F(L.mean[l]);
            f.dmean = (double*)(ws + L.dmean);
            hipLaunchKernelGGL((ut_finish_kernel<0>), dim3(1), dim3(256), 0, s, f);
            r.mean = F(L.mean[l]);
            reduce_u<1>(r, s);
            f.rstd = F(L.rstd[l]);
            f.run_mean = gamma + 2 * cout;
            f.run_var = gamma + 3 * cout;
            hipLaunchKernelGGL((ut_finish_kernel<1>), dim3(1), dim3(256), 0, s, f);
            hipLaunchKernelGGL(ut_bn_act_kernel, dim3(grid_for(cnt)), dim3(256), 0, s, z, F(L.mean[l]), F(L.rstd[l]),
                               gamma, gamma + cout, a, cnt, cout);
        } else {
            hipLaunchKernelGGL(ut_bn_act_kernel, dim3(grid_for(cnt)), dim3(256), 0, s, z, nullptr, nullptr, nullptr,
                               nullptr, a, cnt, cout);
        }
        // the next layer's input
        in = a;
        if (l == 1 || l == 3 || l == 5) {
            const size_t po = l == 1 ? L.p1 : l == 3 ? L.p2 : L.p3;
            hipLaunchKernelGGL(ut_pool_kernel, dim3(grid_for(px(l) * cout / 4)), dim3(256), 0, s, a, F(po), n, h, w,
                               cout);
            in = F(po);
        } else if (l == 7 || l == 9 || l == 11) {
            // [upsample(a) | skip] at twice the resolution
            const size_t co = l == 7 ? L.c3 : l == 9 ? L.c2 : L.c1;
            const float* skip = F(L.a[l == 7 ? 5 : l == 9 ? 3 : 1]);
            const int cs = l == 7 ? 256 : l == 9 ? 128 : 64;
            hipLaunchKernelGGL(ut_upcat_kernel, dim3(grid_for(4 * px(l) * (cout + cs))), dim3(256), 0, s, a, skip,
                               F(co), n, h, w, cout, cs);
            in = F(co);
        }
        if ((st = check_launch("unet train: forward")) != DRC_OK) return st;
    }
    hipLaunchKernelGGL(ut_out_kernel, dim3(grid_for(L.P[0])), dim3(256), 0, s, F(L.a[13]), d_params + woff_u(14),
                       d_params + boff_u(14), y, L.P[0]);

    // ---------------- loss: mean |y - t|, g = sign(y - t) / M
    const long M = L.P[0] * 3;
    const int nparts = (int)((M + kLossPerBlock - 1) / kLossPerBlock);
    hipLaunchKernelGGL(l1_partial_kernel, dim3(nparts), dim3(256), 0, s, (const float*)y, d_target, M, kLossPerBlock,
                       (float)(1.0 / (double)M), F(L.g), (double*)(ws + L.lossp), nullptr, nullptr, 0, 0);
    hipLaunchKernelGGL(l1_final_kernel, dim3(1), dim3(256), 0, s, (const double*)(ws + L.lossp), nparts, M, d_loss);

    // ---------------- backward
    const long P = nparams_u();
    hipLaunchKernelGGL(ut_fill_kernel, dim3(grid_for(P)), dim3(256), 0, s, dp, P, 0.0f);  // running statistics: 0
    float* bufs[3] = {F(L.bufA), F(L.bufB), F(L.bufC)};
    float* da = bufs[0];
    {
        const long per = (L.P[0] + kOutBlocks - 1) / kOutBlocks;
        hipLaunchKernelGGL(ut_out_bwd_kernel, dim3(kOutBlocks), dim3(256), 0, s, (const float*)y, F(L.g),
                           (const float*)F(L.a[13]), (const float*)(d_params + woff_u(14)), da,
                           (double*)(ws + L.outp), L.P[0], per);
        hipLaunchKernelGGL(ut_out_bwd_final_kernel, dim3(1), dim3(256), 0, s, (const double*)(ws + L.outp), kOutBlocks,
                           dp + woff_u(14), dp + boff_u(14));
    }
    for (int l = 13; l >= 0; --l) {
        int h, w;
        hw(l, h, w);
        const int cin = kU[l].cin, cout = kU[l].cout;
        const long cnt = px(l) * cout;
        float* dz = da == bufs[0] ? bufs[1] : bufs[0];
        if (da != bufs[0] && da != bufs[1]) dz = bufs[0];
        float* gamma = d_params + boff_u(l) + cout;
        if (kU[l].bn) {
            RedArgs r{};
            r.z = F(L.z[l]);
            r.a = F(L.a[l]);
            r.da = da;
            r.mean = F(L.mean[l]);
            r.rstd = F(L.rstd[l]);
            r.npix = px(l);
            r.C = cout;
            r.partial = (double*)(ws + L.red);
            reduce_u<2>(r, s);
            FinArgs f{};
            f.partial = r.partial;
            f.blocks = kRedBlocks;
            f.C = cout;
            f.M = px(l);
            f.dgamma = dp + boff_u(l) + cout;
            f.dbeta = dp + boff_u(l) + 2 * cout;
            f.k1 = F(L.k1);
            f.k2 = F(L.k2);
            hipLaunchKernelGGL((ut_finish_kernel<2>), dim3(1), dim3(256), 0, s, f);
            hipLaunchKernelGGL(ut_bn_bwd_kernel, dim3(grid_for(cnt)), dim3(256), 0, s, (const float*)F(L.z[l]),
                               (const float*)F(L.a[l]), (const float*)da, (const float*)F(L.mean[l]),
                               (const float*)F(L.rstd[l]), (const float*)gamma, (const float*)F(L.k1),
                               (const float*)F(L.k2), dz, cnt, cout);
        } else {
            hipLaunchKernelGGL(ut_bn_bwd_kernel, dim3(grid_for(cnt)), dim3(256), 0, s, (const float*)F(L.z[l]),
                               (const float*)F(L.a[l]), (const float*)da, nullptr, nullptr, nullptr, nullptr, nullptr,
                               dz, cnt, cout);
        }
        // bias gradient: column sums of dz (384 fixed partial rows)
        hipLaunchKernelGGL((colsum_partial_kernel<float, 4>), dim3(384), dim3(256), 0, s, (const float*)dz, cnt, cout,
                           F(L.colp));
        hipLaunchKernelGGL(colsum_final_kernel, dim3(cout), dim3(256), 0, s, (const float*)F(L.colp), 384, cout, 1.0f,
                           dp + boff_u(l));
        // weight gradient: reduction over the layer's pixels of dz x its input (stride 1)
        const float* lin = l == 0 ? d_x
                         : l == 12 ? F(L.c1) : l == 10 ? F(L.c2) : l == 8 ? F(L.c3)
                         : l == 6 ? F(L.p3) : l == 4 ? F(L.p2) : l == 2 ? F(L.p1) : F(L.a[l - 1]);
        {
            const WPlanU wp = wplan_u(cin, cout, px(l));
            WgradArgs a{};
            a.p = dz;
            a.pc = cout;
            a.pc0 = cout;
            a.pld = cout;
            a.q = lin;
            a.q_raw = l == 0;
            a.qc = cin;
            a.qld = cin;
            a.nmaps = n;
            a.Hr = h;
            a.Wr = w;
            a.Hq = h;
            a.Wq = w;
            a.stride = 1;
            a.per_block = wp.per_block;
            a.jtiles = wp.jtiles;
            a.partial = F(L.part);
            dim3 grid(wp.nchunks, wp.jtiles * wp.ptiles);
            if (wp.VEC == 4) hipLaunchKernelGGL((wgrad_kernel<float, 4, 4, 4>), grid, dim3(256), 0, s, a);
            else if (wp.JB == 4 && wp.PB == 4) hipLaunchKernelGGL((wgrad_kernel<float, 4, 4, 1>), grid, dim3(256), 0, s, a);
            else return drc_fail(DRC_ERR_STATE, "%s: no weight-gradient tile for layer %d", who, l);
            const long count = 9L * cin * cout;
            hipLaunchKernelGGL(wgrad_final_kernel, dim3((int)((count + 63) / 64)), dim3(1024), 0, s,
                               (const float*)F(L.part), 4 * wp.nchunks, cin, cout, 0, 1.0f, dp + woff_u(l));
        }
        if ((st = check_launch("unet train: backward")) != DRC_OK) return st;
        if (l == 0) break;
        // data gradient: the same convolution with flipped, transposed weights
        float* dx = (dz == bufs[0] || da == bufs[0]) ? ((dz == bufs[1] || da == bufs[1]) ? bufs[2] : bufs[1])
                                                     : bufs[0];
        hipLaunchKernelGGL(ut_flip_kernel, dim3(grid_for(9L * cin * cout)), dim3(256), 0, s, d_params + woff_u(l),
                           F(L.wt), cin, cin, cout);
        if ((st = conv_u(dz, F(L.wt), nullptr, dx, n, h, w, cout, cin, s)) != DRC_OK) return st;
        // route the gradient of the layer's input
        if (l == 12 || l == 10 || l == 8) {
            // [upsample(low) | skip]: the adjoint upsampling gives the gradient of the
            // previous stage's output, the skip part seeds the encoder's gradient
            const int prev = l - 1, cl = kU[prev].cout, cs = cin - cl;
            int hp, wpv;
            hw(prev, hp, wpv);
            float* dlow = (dx == bufs[0]) ? bufs[1] : bufs[0];  // any buffer but dx (dz is dead)
            float* dskip = F(l == 12 ? L.ds1 : l == 10 ? L.ds2 : L.ds3);
            hipLaunchKernelGGL(ut_upcat_bwd_kernel, dim3(grid_for(px(prev) * cl)), dim3(256), 0, s, (const float*)dx,
                               dlow, dskip, n, hp, wpv, cl, cs);
            da = dlow;
        } else if (l == 6 || l == 4 || l == 2) {
            // pooled input: route to the first maximum, added to the skip gradient
            const int src = l - 1;  // the pooled stage output (5, 3, 1)
            int hs, wsz;
            hw(src, hs, wsz);
            float* ds = F(l == 6 ? L.ds3 : l == 4 ? L.ds2 : L.ds1);
            hipLaunchKernelGGL(ut_pool_bwd_kernel, dim3(grid_for(px(src) * kU[src].cout)), dim3(256), 0, s,
                               (const float*)F(L.a[src]), (const float*)dx, ds, n, hs, wsz, kU[src].cout);
            da = ds;
        } else {
            da = dx;
        }
        if ((st = check_launch("unet train: backward")) != DRC_OK) return st;
    }

    // ---------------- Adam on each layer's trainable segment (w, b, gamma, beta)
    float step_size, inv_sqrt_bc2;
    {
        const double bc1 = 1.0 - std::pow(adam->beta1, (double)t);
        const double bc2 = 1.0 - std::pow(adam->beta2, (double)t);
        step_size = (float)(adam->lr / bc1);
        inv_sqrt_bc2 = (float)(1.0 / std::sqrt(bc2));
    }
    for (int l = 0; l < kLayersU; ++l) {
        const long lo = woff_u(l), hi = boff_u(l) + kU[l].cout * (kU[l].bn ? 3 : 1);
        hipLaunchKernelGGL(adam_kernel, dim3(grid_for(hi - lo)), dim3(256), 0, s, d_params + lo, d_m + lo, d_v + lo,
                           (const float*)(dp + lo), hi - lo, (float)adam->beta1, (float)(1.0 - adam->beta1),
                           (float)adam->beta2, (float)(1.0 - adam->beta2), step_size, inv_sqrt_bc2, (float)adam->eps);
    }
    return check_launch("unet train: adam");
}
