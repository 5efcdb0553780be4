// Training-data augmentation (Sec. 5: the data loader rotates and flips the
// training maps), read as the symmetries of a hemispherical lat-long map
// (normal along +Z, Sec. 4.3): azimuth rotations by whole columns and mirror
// images through a plane containing the normal. A map transformed by
// phi -> s phi + alpha (s = -1 when flipped, alpha = 2 pi k / W) moves the
// value of column u to column (u + k) mod W, or (k - 1 - u) mod W when
// flipped; the normals' (Nx, Ny) are reflected (Ny -> -Ny) when flipped and
// then rotated by alpha, everything else keeps its value; the target map
// moves with its input.
//
// One thread per output pixel gathers its source pixel (the same row of the
// same map): 40 bytes read and 40 written per pixel with a target, HBM-bound.
#include <hip/hip_runtime.h>

#include <cmath>

#include "drc_cae.h"
#include "common.h"
#include "internal.h"

namespace {

constexpr int kThreads = 256;

struct AugArgs {
    const float* x;   // [n, H, W, 7]
    const float* t;   // [n, H, W, 3] or null
    const int32_t* roll;
    const int32_t* flip;
    float* xo;
    float* to;
    long pixels;      // n * H * W
    int H, W;
};

__global__ __launch_bounds__(kThreads) void augment_kernel(AugArgs a) {
    for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < a.pixels; i += (long)gridDim.x * kThreads) {
        const long row = i / a.W;                 // (map, row) index
        const int u = (int)(i - row * a.W);
        const long m = row / a.H;
        const drc::AugMap am = drc::aug_map(a.roll, a.flip, m, a.W);
        const long j = row * a.W + drc::aug_src_col(am, u, a.W);
        const float* p = a.x + 7 * j;
        float v[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) v[c] = p[c];
        drc::aug_normal(am, v[3], v[4]);
        float* q = a.xo + 7 * i;
#pragma unroll
        for (int c = 0; c < 7; ++c) q[c] = v[c];
        if (a.t) {
#pragma unroll
            for (int c = 0; c < 3; ++c) a.to[3 * i + c] = a.t[3 * j + c];
        }
    }
}

}  // namespace

extern "C" drc_status drc_augment(const float* d_x, const float* d_t, int n, int H, int W, const int32_t* d_roll,
                                  const int32_t* d_flip, float* d_x_out, float* d_t_out, void* stream) {
    if (n < 0 || H < 1 || W < 1 || (long)n * H * W > (1L << 40))
        return drc_fail(DRC_ERR_SHAPE, "augment: n = %d, H = %d, W = %d", n, H, W);
    if (n == 0) return DRC_OK;
    drc_status st;
    if ((st = check_ptr("augment", "d_x", d_x, 4, false)) != DRC_OK) return st;
    if ((st = check_ptr("augment", "d_roll", d_roll, 4, false)) != DRC_OK) return st;
    if ((st = check_ptr("augment", "d_flip", d_flip, 4, false)) != DRC_OK) return st;
    if ((st = check_ptr("augment", "d_x_out", d_x_out, 4, false)) != DRC_OK) return st;
    if ((st = check_ptr("augment", "d_t", d_t, 4, true)) != DRC_OK) return st;
    if ((st = check_ptr("augment", "d_t_out", d_t_out, 4, d_t == nullptr)) != DRC_OK) return st;
    if (d_t == nullptr && d_t_out != nullptr)
        return drc_fail(DRC_ERR_INVALID_ARG, "augment: d_t_out given without d_t");
    const size_t xb = (size_t)n * H * W * 7 * sizeof(float), tb = (size_t)n * H * W * 3 * sizeof(float);
    const char *x0 = (const char*)d_x, *x1 = (const char*)d_x_out;
    if (x0 < x1 + xb && x1 < x0 + xb) return drc_fail(DRC_ERR_INVALID_ARG, "augment: d_x and d_x_out overlap");
    if (d_t) {
        const char *t0 = (const char*)d_t, *t1 = (const char*)d_t_out;
        if (t0 < t1 + tb && t1 < t0 + tb) return drc_fail(DRC_ERR_INVALID_ARG, "augment: d_t and d_t_out overlap");
    }
    AugArgs a{d_x, d_t, d_roll, d_flip, d_x_out, d_t_out, (long)n * H * W, H, W};
    const long g = (a.pixels + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(augment_kernel, dim3((unsigned)(g < 65536 ? g : 65536)), dim3(kThreads), 0,
                       (hipStream_t)stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return drc_fail(DRC_ERR_HIP, "augment: launch failed: %s", hipGetErrorString(e));
    return DRC_OK;
}
