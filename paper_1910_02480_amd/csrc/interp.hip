// Interpolation between cache points (Sec. 4.2, Eqs. 4-6): for each image
// pixel, the probabilities of sampling the radiance maps of the cache points
// around it.
//
// Cache points sit on a regular grid of spacing r pixels: point (gy, gx) on
// pixel (gx r, gy r). A pixel's candidates are the four corners of its grid
// cell inside the image (the only points with a non-zero position weight).
// Weight of a candidate: w = w_p w_n + w_p + eps with the position weight
// w_p = max(0, 1 - dist / r) (dist in pixels) and the normal weight
// w_n = max(0, dot of the unit normals), as the text describes them; the
// weights are normalised to probabilities, and when they all vanish the
// present corners are equally likely.
//
// Per pixel: a 12-byte normal read, four cache normals read through the
// caches (each is shared by about r^2 pixels), and one 16-byte store each
// of indices and probabilities: HBM-bound.
#include <hip/hip_runtime.h>

#include <cmath>

#include "drc_cae.h"
#include "internal.h"

namespace {

constexpr int kThreads = 256;

struct InterpArgs {
    const float* normals;        // [Hi, Wi, 3]
    const float* cache_normals;  // [Gy, Gx, 3]
    int4* idx;                   // [Hi, Wi] x 4
    float4* prob;                // [Hi, Wi] x 4
    long pixels;
    int Wi, r, Gx, Gy;
    float eps;
};

__device__ __forceinline__ void pixel_weights(const InterpArgs& a, long i, int x, int y, float nx, float ny,
                                              float nz) {
    const float nn = nx * nx + ny * ny + nz * nz;
    const int gx0 = x / a.r, gy0 = y / a.r;
    int id[4];
    float w[4];
    float tot = 0.0f;
    int present = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int gx = gx0 + (k & 1), gy = gy0 + (k >> 1);
        id[k] = -1;
        w[k] = 0.0f;
        if (gx < a.Gx && gy < a.Gy) {
            const int c = gy * a.Gx + gx;
            const float cx = a.cache_normals[3 * c], cy = a.cache_normals[3 * c + 1],
                        cz = a.cache_normals[3 * c + 2];
            const float cc = cx * cx + cy * cy + cz * cz;
            const float dx = (float)(x - gx * a.r), dy = (float)(y - gy * a.r);
            const float dist = sqrtf(dx * dx + dy * dy);
            const float wp = fmaxf(0.0f, 1.0f - dist / (float)a.r);
            const float den = sqrtf(nn * cc);
            const float wn = den > 0.0f ? fmaxf(0.0f, (nx * cx + ny * cy + nz * cz) / den) : 0.0f;
            id[k] = c;
            w[k] = wp * wn + wp + a.eps;
            tot += w[k];
            ++present;
        }
    }
    float p[4];
    const float uni = 1.0f / (float)present;
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = id[k] < 0 ? 0.0f : (tot > 0.0f ? w[k] / tot : uni);
    a.idx[i] = make_int4(id[0], id[1], id[2], id[3]);
    a.prob[i] = make_float4(p[0], p[1], p[2], p[3]);
}

// One pixel per thread: a wave's index and probability stores are 1 KB
// contiguous each. (Four consecutive pixels per thread spread them 64 bytes
// apart and ran at half the bandwidth; four pixels a grid apart per thread
// ran 15 % slower than this.)
__global__ __launch_bounds__(kThreads) void interp_weights_kernel(InterpArgs a) {
    for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < a.pixels; i += (long)gridDim.x * kThreads) {
        const int y = (int)(i / a.Wi), x = (int)(i - (long)y * a.Wi);
        pixel_weights(a, i, x, y, a.normals[3 * i], a.normals[3 * i + 1], a.normals[3 * i + 2]);
    }
}

}  // namespace

extern "C" drc_status drc_interp_weights(const float* d_normals, int Hi, int Wi, int r,
                                         const float* d_cache_normals, float eps, int32_t* d_idx,
                                         float* d_prob, void* stream) {
    if (Hi < 1 || Wi < 1 || (long)Hi * Wi > 0x7fffffffL)
        return drc_fail(DRC_ERR_SHAPE, "interp_weights: image %d x %d", Hi, Wi);
    if (r < 1 || r > 4096) return drc_fail(DRC_ERR_SHAPE, "interp_weights: grid spacing r = %d", r);
    if (!(eps >= 0.0f) || !std::isfinite(eps))
        return drc_fail(DRC_ERR_INVALID_ARG, "interp_weights: eps must be finite and >= 0");
    drc_status st;
    if ((st = check_ptr("interp_weights", "d_normals", d_normals, 4, false)) != DRC_OK) return st;
    if ((st = check_ptr("interp_weights", "d_cache_normals", d_cache_normals, 4, false)) != DRC_OK) return st;
    if ((st = check_ptr("interp_weights", "d_idx", d_idx, 16, false)) != DRC_OK) return st;
    if ((st = check_ptr("interp_weights", "d_prob", d_prob, 16, false)) != DRC_OK) return st;
    InterpArgs a{d_normals, d_cache_normals, (int4*)d_idx, (float4*)d_prob, (long)Hi * Wi,
                 Wi, r, (Wi - 1) / r + 1, (Hi - 1) / r + 1, eps};
    const long g = (a.pixels + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(interp_weights_kernel, dim3((unsigned)(g < 65536 ? g : 65536)), dim3(kThreads), 0,
                       (hipStream_t)stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return drc_fail(DRC_ERR_HIP, "interp_weights: launch failed: %s", hipGetErrorString(e));
    return DRC_OK;
}
