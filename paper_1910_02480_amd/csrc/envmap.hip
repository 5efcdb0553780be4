// Sampling the predicted radiance map R as an environment map (Sec. 3: the
// indirect term is estimated with multiple importance sampling that
// alternates between R and the BRDF; Sec. 4.3: hemispherical lat-long
// projection with the normal along +Z).
//
// Per map the distribution is piecewise constant over the (u, v) unit
// square, pixel weight = max(0, luminance) * sin(row-centre polar angle):
// luminance times the pixel's solid angle. drc_envmap_build turns every map
// of a batch into a marginal CDF over rows and one conditional CDF over
// columns per row; drc_envmap_sample inverts them for given uniforms and
// drc_envmap_pdf evaluates the solid-angle density of given directions (the
// second density that MIS weights need).
//
// The build is one read of the map and one write of the tables: HBM-bound.
// One workgroup (4 waves) per map; a wave scans whole rows with wave-level
// shuffles (rows narrower than 64 columns are packed several to a wave, as
// segmented scans), keeps each row total in LDS, and wave 0 then scans the
// row totals into the marginal.
#include <hip/hip_runtime.h>

#include <cmath>

#include "drc_cae.h"
#include "internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxChunks = 16;  // columns per row <= 64 * kMaxChunks
constexpr int kMaxW = 64 * kMaxChunks;
constexpr int kMaxH = 4096;     // row totals and row sines held in LDS

constexpr float kHalfPi = 1.57079632679489662f;
constexpr float kTwoPi = 6.28318530717958648f;
constexpr float kPiSq = 9.86960440108935862f;
// ITU-R BT.709 relative luminance of linear R, G, B
constexpr float kLumR = 0.2126f, kLumG = 0.7152f, kLumB = 0.0722f;

struct BuildArgs {
    const float* y;  // [n, H, W, 3]
    float* cdf_u;    // [n, H, W]
    float* cdf_v;    // [n, H]
    float* total;    // [n]
    int H, W;
};

// Lane shifts through DPP (data-parallel primitives of the VALU, no LDS
// round trip): row_shr:d moves a value d lanes up within each 16-lane row
// (lanes below d read `fill`); row_bcast:15 / row_bcast:31 hand lane 15 of
// a row to the next row (rows 1 and 3) / lane 31 to rows 2 and 3.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}

// Inclusive prefix sum over segments of SEG lanes (a power of two <= 64),
// followed by a running maximum: the shift tree adds the terms of
// neighbouring lanes in different orders, so two prefixes of non-negative
// terms can come out one rounding step out of order; the maximum pass makes
// the sequence non-decreasing (exactly, as max does not round). Inputs are
// non-negative, so 0 is the identity of both passes.
template <int SEG, bool MAX>
__device__ __forceinline__ float seg_pass(float x, int ls) {
    auto op = [](float a, float b) { return MAX ? fmaxf(a, b) : a + b; };
    if constexpr (SEG > 1) { const float t = dpp<0x111, 0xf>(x); x = op(x, ls >= 1 ? t : 0.0f); }
    if constexpr (SEG > 2) { const float t = dpp<0x112, 0xf>(x); x = op(x, ls >= 2 ? t : 0.0f); }
    if constexpr (SEG > 4) { const float t = dpp<0x114, 0xf>(x); x = op(x, ls >= 4 ? t : 0.0f); }
    if constexpr (SEG > 8) { const float t = dpp<0x118, 0xf>(x); x = op(x, ls >= 8 ? t : 0.0f); }
    if constexpr (SEG > 16) x = op(x, dpp<0x142, 0xa>(x));
    if constexpr (SEG > 32) x = op(x, dpp<0x143, 0xc>(x));
    return x;
}

template <int SEG>
__device__ __forceinline__ float seg_scan(float x, int ls) {
    return seg_pass<SEG, true>(seg_pass<SEG, false>(x, ls), ls);
}

// SEG = lanes per row segment (next power of two >= W, at most 64); CH =
// 64-column chunks per row (W <= 64 CH); G = row groups a lane loads before
// it scans (all of a wave's loads of G row groups are in flight together:
// the kernel is bound by HBM latency otherwise).
template <int SEG, int CH, int G>
__global__ __launch_bounds__(kThreads) void envmap_build_kernel(BuildArgs a) {
    extern __shared__ float smem[];  // rowsum[H], then sin of the row centres [H]
    const int H = a.H, W = a.W;
    float* rowsum = smem;
    float* rowsin = smem + H;
    const int m = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ls = lane & (SEG - 1);
    constexpr int RPG = 64 / SEG;  // rows one wave scans side by side
    const float* ym = a.y + (size_t)m * H * W * 3;
    float* cu = a.cdf_u + (size_t)m * H * W;
    const float dtheta = kHalfPi / (float)H;
    for (int v = threadIdx.x; v < H; v += kThreads) rowsin[v] = sinf(((float)v + 0.5f) * dtheta);
    __syncthreads();

    for (int r0 = wave * RPG * G; r0 < H; r0 += 4 * RPG * G) {
        float rgb[G][CH][3];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int v = r0 + g * RPG + lane / SEG;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int u = c * 64 + ls;
                rgb[g][c][0] = rgb[g][c][1] = rgb[g][c][2] = 0.0f;
                if (v < H && u < W) {
                    const float* p = ym + ((size_t)v * W + u) * 3;
                    rgb[g][c][0] = p[0];
                    rgb[g][c][1] = p[1];
                    rgb[g][c][2] = p[2];
                }
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int v = r0 + g * RPG + lane / SEG;
            const bool row_ok = v < H;
            const float st = row_ok ? rowsin[v] : 0.0f;
            float pre[CH];
            float carry = 0.0f;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const float lum = kLumR * rgb[g][c][0] + kLumG * rgb[g][c][1] + kLumB * rgb[g][c][2];
                const float f = fmaxf(lum, 0.0f) * st;  // zero outside the map
                const float x = seg_scan<SEG>(f, ls) + carry;
                pre[c] = x;
                // the row prefix at the chunk's last column (W - 1 in the last
                // chunk): the largest value of the chunk, so every entry of the
                // row divided by the row total is at most 1 and the last is 1
                if (c * 64 < W) {
                    const int last = min(SEG, W - c * 64) - 1;
                    if constexpr (SEG == 64)  // one segment: a scalar read of the lane
                        carry = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), last));
                    else
                        carry = __shfl(x, (lane & ~(SEG - 1)) + last, 64);
                }
            }
            const float tot = carry;
            const float inv_w = 1.0f / (float)W;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int u = c * 64 + ls;
                if (row_ok && u < W)
                    cu[(size_t)v * W + u] = tot > 0.0f ? pre[c] / tot : (float)(u + 1) * inv_w;
            }
            if (row_ok && ls == 0) rowsum[v] = tot;
        }
    }
    __syncthreads();
    if (wave == 0) {
        float carry = 0.0f;
        for (int v0 = 0; v0 < H; v0 += 64) {
            const int v = v0 + lane;
            const float f = v < H ? rowsum[v] : 0.0f;
            const float x = seg_scan<64>(f, lane) + carry;
            if (v < H) rowsum[v] = x;
            carry = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), min(63, H - 1 - v0)));
        }
        const float tot = carry;
        float* cv = a.cdf_v + (size_t)m * H;
        for (int v = lane; v < H; v += 64)
            cv[v] = tot > 0.0f ? rowsum[v] / tot : (float)(v + 1) / (float)H;
        if (lane == 0) a.total[m] = tot;
    }
}

// First index k in [0, n) with cdf[k] > xi (n - 1 if none), and the
// probability of k and the position of xi inside it, in [0, 1].
__device__ __forceinline__ int invert_cdf(const float* cdf, int n, float xi, float& frac, float& p) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] <= xi) lo = mid + 1;
        else hi = mid;
    }
    const int k = lo < n ? lo : n - 1;
    const float prev = k > 0 ? cdf[k - 1] : 0.0f;
    p = cdf[k] - prev;
    frac = p > 0.0f ? fminf(fmaxf((xi - prev) / p, 0.0f), 1.0f) : 0.0f;
    return k;
}

struct SampleArgs {
    const float* cdf_u;
    const float* cdf_v;
    const float* xi;  // [n, S, 2]
    float* dir;       // [n, S, 3]
    float* pdf;       // [n, S]
    int32_t* pix;     // [n, S]
    long count;       // n * S
    int S, H, W;
};

__global__ __launch_bounds__(kThreads) void envmap_sample_kernel(SampleArgs a) {
    const float one_minus = 0x1.fffffep-1f;
    for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < a.count; i += (long)gridDim.x * kThreads) {
        const long m = i / a.S;
        const float x1 = fminf(fmaxf(a.xi[2 * i], 0.0f), one_minus);
        const float x2 = fminf(fmaxf(a.xi[2 * i + 1], 0.0f), one_minus);
        float fv, pv, fu, pu;
        const int v = invert_cdf(a.cdf_v + m * a.H, a.H, x1, fv, pv);
        const int u = invert_cdf(a.cdf_u + (m * a.H + v) * a.W, a.W, x2, fu, pu);
        const float theta = ((float)v + fv) / (float)a.H * kHalfPi;
        const float phi = ((float)u + fu) / (float)a.W * kTwoPi;
        float st, ct, sp, cp;
        sincosf(theta, &st, &ct);
        sincosf(phi, &sp, &cp);
        a.dir[3 * i] = st * cp;
        a.dir[3 * i + 1] = st * sp;
        a.dir[3 * i + 2] = ct;
        a.pdf[i] = st > 0.0f ? pv * pu * (float)a.H * (float)a.W / (kPiSq * st) : 0.0f;
        a.pix[i] = v * a.W + u;
    }
}

struct PdfArgs {
    const float* cdf_u;
    const float* cdf_v;
    const float* dir;  // [n, S, 3]
    float* pdf;        // [n, S]
    long count;
    int S, H, W;
};

__global__ __launch_bounds__(kThreads) void envmap_pdf_kernel(PdfArgs a) {
    for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < a.count; i += (long)gridDim.x * kThreads) {
        const long m = i / a.S;
        const float x = a.dir[3 * i], y = a.dir[3 * i + 1], z = a.dir[3 * i + 2];
        const float r = sqrtf(x * x + y * y);
        const float len = sqrtf(r * r + z * z);
        float out = 0.0f;
        if (z >= 0.0f && r > 0.0f) {
            const float theta = atan2f(r, z);
            float phi = atan2f(y, x);
            if (phi < 0.0f) phi += kTwoPi;
            const int v = min((int)(theta * (1.0f / kHalfPi) * (float)a.H), a.H - 1);
            const int u = min((int)(phi * (1.0f / kTwoPi) * (float)a.W), a.W - 1);
            const float* cv = a.cdf_v + m * a.H;
            const float* cu = a.cdf_u + (m * a.H + v) * a.W;
            const float pv = cv[v] - (v > 0 ? cv[v - 1] : 0.0f);
            const float pu = cu[u] - (u > 0 ? cu[u - 1] : 0.0f);
            out = pv * pu * (float)a.H * (float)a.W / (kPiSq * (r / len));
        }
        a.pdf[i] = out;
    }
}

drc_status shape_ok(const char* who, int n, int H, int W) {
    if (n < 0) return drc_fail(DRC_ERR_SHAPE, "%s: n = %d (must be >= 0)", who, n);
    if (H < 1 || H > kMaxH || W < 1 || W > kMaxW)
        return drc_fail(DRC_ERR_SHAPE, "%s: H = %d, W = %d (need 1 <= H <= %d, 1 <= W <= %d)", who, H, W,
                        kMaxH, kMaxW);
    return DRC_OK;
}

int grid_for(long count) {
    const long g = (count + kThreads - 1) / kThreads;
    return (int)(g < 16384 ? (g > 0 ? g : 1) : 16384);
}

}  // namespace

#define TRY(expr)                    \
    do {                             \
        drc_status s_ = (expr);      \
        if (s_ != DRC_OK) return s_; \
    } while (0)

extern "C" drc_status drc_envmap_build(const float* d_y, int n, int H, int W, float* d_cdf_u, float* d_cdf_v,
                                       float* d_total, void* stream) {
    TRY(shape_ok("envmap_build", n, H, W));
    if (n == 0) return DRC_OK;
    TRY(check_ptr("envmap_build", "d_y", d_y, 4, false));
    TRY(check_ptr("envmap_build", "d_cdf_u", d_cdf_u, 4, false));
    TRY(check_ptr("envmap_build", "d_cdf_v", d_cdf_v, 4, false));
    TRY(check_ptr("envmap_build", "d_total", d_total, 4, false));
    BuildArgs a{d_y, d_cdf_u, d_cdf_v, d_total, H, W};
    const dim3 grid(n), block(kThreads);
    const size_t lds = 2 * (size_t)H * sizeof(float);
    const hipStream_t s = (hipStream_t)stream;
    if (W <= 1) hipLaunchKernelGGL((envmap_build_kernel<1, 1, 4>), grid, block, lds, s, a);
    else if (W <= 2) hipLaunchKernelGGL((envmap_build_kernel<2, 1, 4>), grid, block, lds, s, a);
    else if (W <= 4) hipLaunchKernelGGL((envmap_build_kernel<4, 1, 4>), grid, block, lds, s, a);
    else if (W <= 8) hipLaunchKernelGGL((envmap_build_kernel<8, 1, 4>), grid, block, lds, s, a);
    else if (W <= 16) hipLaunchKernelGGL((envmap_build_kernel<16, 1, 4>), grid, block, lds, s, a);
    else if (W <= 32) hipLaunchKernelGGL((envmap_build_kernel<32, 1, 8>), grid, block, lds, s, a);
    else if (W <= 64) hipLaunchKernelGGL((envmap_build_kernel<64, 1, 8>), grid, block, lds, s, a);
    else if (W <= 128) hipLaunchKernelGGL((envmap_build_kernel<64, 2, 4>), grid, block, lds, s, a);
    else if (W <= 256) hipLaunchKernelGGL((envmap_build_kernel<64, 4, 2>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((envmap_build_kernel<64, kMaxChunks, 1>), grid, block, lds, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return drc_fail(DRC_ERR_HIP, "envmap_build: launch failed: %s", hipGetErrorString(e));
    return DRC_OK;
}

extern "C" drc_status drc_envmap_sample(const float* d_cdf_u, const float* d_cdf_v, int n, int H, int W, int S,
                                        const float* d_xi, float* d_dir, float* d_pdf, int32_t* d_pix,
                                        void* stream) {
    TRY(shape_ok("envmap_sample", n, H, W));
    if (S < 0) return drc_fail(DRC_ERR_SHAPE, "envmap_sample: S = %d (must be >= 0)", S);
    if (n == 0 || S == 0) return DRC_OK;
    TRY(check_ptr("envmap_sample", "d_cdf_u", d_cdf_u, 4, false));
    TRY(check_ptr("envmap_sample", "d_cdf_v", d_cdf_v, 4, false));
    TRY(check_ptr("envmap_sample", "d_xi", d_xi, 4, false));
    TRY(check_ptr("envmap_sample", "d_dir", d_dir, 4, false));
    TRY(check_ptr("envmap_sample", "d_pdf", d_pdf, 4, false));
    TRY(check_ptr("envmap_sample", "d_pix", d_pix, 4, false));
    SampleArgs a{d_cdf_u, d_cdf_v, d_xi, d_dir, d_pdf, d_pix, (long)n * S, S, H, W};
    hipLaunchKernelGGL(envmap_sample_kernel, dim3(grid_for(a.count)), dim3(kThreads), 0, (hipStream_t)stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return drc_fail(DRC_ERR_HIP, "envmap_sample: launch failed: %s", hipGetErrorString(e));
    return DRC_OK;
}

extern "C" drc_status drc_envmap_pdf(const float* d_cdf_u, const float* d_cdf_v, int n, int H, int W, int S,
                                     const float* d_dir, float* d_pdf, void* stream) {
    TRY(shape_ok("envmap_pdf", n, H, W));
    if (S < 0) return drc_fail(DRC_ERR_SHAPE, "envmap_pdf: S = %d (must be >= 0)", S);
    if (n == 0 || S == 0) return DRC_OK;
    TRY(check_ptr("envmap_pdf", "d_cdf_u", d_cdf_u, 4, false));
    TRY(check_ptr("envmap_pdf", "d_cdf_v", d_cdf_v, 4, false));
    TRY(check_ptr("envmap_pdf", "d_dir", d_dir, 4, false));
    TRY(check_ptr("envmap_pdf", "d_pdf", d_pdf, 4, false));
    PdfArgs a{d_cdf_u, d_cdf_v, d_dir, d_pdf, (long)n * S, S, H, W};
    hipLaunchKernelGGL(envmap_pdf_kernel, dim3(grid_for(a.count)), dim3(kThreads), 0, (hipStream_t)stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return drc_fail(DRC_ERR_HIP, "envmap_pdf: launch failed: %s", hipGetErrorString(e));
    return DRC_OK;
}
