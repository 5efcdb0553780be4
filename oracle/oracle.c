/*
 * FP64 reference oracle for the Deep Radiance Caching convolutional
 * autoencoder (Jiang & Kainz, "Deep Radiance Caching", Sec. 4.3 and 5).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can check and time the HIP kernels. It shares no
 * code, header, table or helper with them.
 *
 * Everything is computed from the plain definitions with direct nested loops
 * in double precision. Inputs arrive as float64 arrays (the FP32 generator
 * values widened exactly). Tensors are NHWC, contiguous.
 *
 * Definitions (Sec. 4.3: 3x3 (de)convolutions, skip connections, L1 loss;
 * Sec. 5: Adam as shipped with PyTorch):
 *   conv_s2  : y[n,p,q,co] = b[co] + sum_{kh,kw,ci} W[co][kh][kw][ci]
 *                                   * x[n, 2p+kh-1, 2q+kw-1, ci]
 *              (cross-correlation, zero padding 1, stride 2, output H/2)
 *   tconv_s2 : y[n,p,q,co] = b[co] + sum over (i,kh) with p = 2i+kh-1 and
 *              (j,kw) with q = 2j+kw-1 of W[co][kh][kw][ci] * x[n,i,j,ci]
 *              (transposed convolution, padding 1, output padding 1,
 *               output 2H)
 *   circular : the same two layers with the width periodic (a lat-long map
 *              of a hemisphere wraps around in azimuth, Sec. 4.3): column
 *              indices are taken mod the width instead of being dropped,
 *              conv reads x[.., (2q+kw-1) mod W, ..] and tconv adds into
 *              column (2j+kw-1) mod 2W; rows keep zero padding
 *   network  : h1 = relu(conv(x)), h2 = relu(conv(h1)), h3 = relu(conv(h2)),
 *              u3 = relu(tconv(h3)), u2 = relu(tconv([u3|h2])),
 *              y  = tconv([u2|h1])  (linear unless final_relu)
 *   loss     : L = (1/M) sum |y - t|, dL/dy = sign(y - t)/M, sign(0) = 0
 *   adam     : PyTorch's Adam, bias-corrected, no weight decay.
 *
 * Parity: each operator is pinned in the test suite against library
 * routines (PyTorch float64 conv2d / conv_transpose2d and autograd, SciPy
 * correlate2d, torch.optim.Adam), closed forms (adjointness, delta kernels,
 * homogeneity, Adam's first step) and central finite differences. The
 * network as a whole has no worked example in the paper: parity against the
 * paper itself is unpinned beyond those operator-level pins.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Network shape: 7 -> 32 -> 64 -> 128 -> 64 (+64 skip) -> 32 (+32 skip) -> 3 */
/* ------------------------------------------------------------------ */
enum { L_E1 = 0, L_E2, L_E3, L_D3, L_D2, L_D1, NUM_LAYERS };
static const long LAYER_CIN[NUM_LAYERS] = {7, 32, 64, 128, 128, 64};
static const long LAYER_COUT[NUM_LAYERS] = {32, 64, 128, 64, 32, 3};

/* Offset of layer k's weight in the flat parameter vector; its bias follows
 * the weight (W[co][kh][kw][ci] then b[co]). */
static long layer_offset(int k)
{
    long off = 0;
    for (int i = 0; i < k; ++i)
        off += LAYER_COUT[i] * 9 * LAYER_CIN[i] + LAYER_COUT[i];
    return off;
}

long orc_num_params(void) { return layer_offset(NUM_LAYERS); }

long orc_layer_offset(int k) { return layer_offset(k); }

/* ------------------------------------------------------------------ */
/* Column rules. Zero padding: a column outside [0, w) contributes      */
/* nothing (-1). Circular padding along the width: columns mod w.       */
/* ------------------------------------------------------------------ */
static long conv_col(long j, long w, int circ)
{
    if (circ) return ((j % w) + w) % w;
    return (j < 0 || j >= w) ? -1 : j;
}

/* ------------------------------------------------------------------ */
/* Strided 3x3 convolution (stride 2, padding 1: zero, or circular in   */
/* the width when circ).                                                */
/* ------------------------------------------------------------------ */
static void conv_s2(const double *x, long n, long h, long w, long cin,
                    const double *wt, const double *b, long cout, double *y, int circ)
{
    const long ho = h / 2, wo = w / 2;
#pragma omp parallel for collapse(2) schedule(static)
    for (long m = 0; m < n; ++m)
        for (long p = 0; p < ho; ++p)
            for (long q = 0; q < wo; ++q)
                for (long co = 0; co < cout; ++co) {
                    double s = b ? b[co] : 0.0;
                    for (long kh = 0; kh < 3; ++kh) {
                        const long i = 2 * p + kh - 1;
                        if (i < 0 || i >= h) continue;
                        for (long kw = 0; kw < 3; ++kw) {
                            const long j = conv_col(2 * q + kw - 1, w, circ);
                            if (j < 0) continue;
                            const double *xp = x + ((m * h + i) * w + j) * cin;
                            const double *wp = wt + ((co * 3 + kh) * 3 + kw) * cin;
                            for (long ci = 0; ci < cin; ++ci) s += wp[ci] * xp[ci];
                        }
                    }
                    y[((m * ho + p) * wo + q) * cout + co] = s;
                }
}

void orc_conv_s2(const double *x, long n, long h, long w, long cin,
                 const double *wt, const double *b, long cout, double *y)
{
    conv_s2(x, n, h, w, cin, wt, b, cout, y, 0);
}

void orc_conv_s2_pad(const double *x, long n, long h, long w, long cin,
                     const double *wt, const double *b, long cout, double *y, int circ)
{
    conv_s2(x, n, h, w, cin, wt, b, cout, y, circ);
}

/* Input index i feeding output p through kernel row k, for the transposed
 * convolution's relation p = 2 i + k - 1; -1 when no such i exists. With
 * circ (columns only) the relation holds mod 2 h_in. */
static long tconv_src_c(long p, long k, long h_in, int circ)
{
    long t = p + 1 - k;
    if (circ) t = ((t % (2 * h_in)) + 2 * h_in) % (2 * h_in);
    if (t < 0 || (t & 1)) return -1;
    const long i = t / 2;
    return i < h_in ? i : -1;
}

static long tconv_src(long p, long k, long h_in) { return tconv_src_c(p, k, h_in, 0); }

/* ------------------------------------------------------------------ */
/* Transposed 3x3 convolution (stride 2, padding 1, output padding 1;  */
/* circular in the width when circ).                                   */
/* ------------------------------------------------------------------ */
static void tconv_s2(const double *x, long n, long h, long w, long cin,
                     const double *wt, const double *b, long cout, double *y, int circ)
{
    const long ho = 2 * h, wo = 2 * w;
#pragma omp parallel for collapse(2) schedule(static)
    for (long m = 0; m < n; ++m)
        for (long p = 0; p < ho; ++p)
            for (long q = 0; q < wo; ++q)
                for (long co = 0; co < cout; ++co) {
                    double s = b ? b[co] : 0.0;
                    for (long kh = 0; kh < 3; ++kh) {
                        const long i = tconv_src(p, kh, h);
                        if (i < 0) continue;
                        for (long kw = 0; kw < 3; ++kw) {
                            const long j = tconv_src_c(q, kw, w, circ);
                            if (j < 0) continue;
                            const double *xp = x + ((m * h + i) * w + j) * cin;
                            const double *wp = wt + ((co * 3 + kh) * 3 + kw) * cin;
                            for (long ci = 0; ci < cin; ++ci) s += wp[ci] * xp[ci];
                        }
                    }
                    y[((m * ho + p) * wo + q) * cout + co] = s;
                }
}

void orc_tconv_s2(const double *x, long n, long h, long w, long cin,
                  const double *wt, const double *b, long cout, double *y)
{
    tconv_s2(x, n, h, w, cin, wt, b, cout, y, 0);
}

void orc_tconv_s2_pad(const double *x, long n, long h, long w, long cin,
                      const double *wt, const double *b, long cout, double *y, int circ)
{
    tconv_s2(x, n, h, w, cin, wt, b, cout, y, circ);
}

/* ------------------------------------------------------------------ */
/* Reverse-mode derivatives of the two layers: the forward loops read   */
/* backwards. g is dL/d(layer output before activation).               */
/* ------------------------------------------------------------------ */
static void conv_s2_bwd(const double *x, long n, long h, long w, long cin,
                        const double *wt, long cout, const double *g,
                        double *dw, double *db, double *dx, int circ)
{
    const long ho = h / 2, wo = w / 2;
#pragma omp parallel for schedule(static)
    for (long co = 0; co < cout; ++co) {
        double *dwc = dw + co * 9 * cin;
        for (long k = 0; k < 9 * cin; ++k) dwc[k] = 0.0;
        double sb = 0.0;
        for (long m = 0; m < n; ++m)
            for (long p = 0; p < ho; ++p)
                for (long q = 0; q < wo; ++q) {
                    const double gv = g[((m * ho + p) * wo + q) * cout + co];
                    sb += gv;
                    for (long kh = 0; kh < 3; ++kh) {
                        const long i = 2 * p + kh - 1;
                        if (i < 0 || i >= h) continue;
                        for (long kw = 0; kw < 3; ++kw) {
                            const long j = conv_col(2 * q + kw - 1, w, circ);
                            if (j < 0) continue;
                            const double *xp = x + ((m * h + i) * w + j) * cin;
                            double *dwp = dwc + (kh * 3 + kw) * cin;
                            for (long ci = 0; ci < cin; ++ci) dwp[ci] += gv * xp[ci];
                        }
                    }
                }
        if (db) db[co] = sb;
    }
    if (!dx) return;
#pragma omp parallel for schedule(static)
    for (long m = 0; m < n; ++m) {
        double *dxm = dx + m * h * w * cin;
        for (long k = 0; k < h * w * cin; ++k) dxm[k] = 0.0;
        for (long p = 0; p < ho; ++p)
            for (long q = 0; q < wo; ++q)
                for (long co = 0; co < cout; ++co) {
                    const double gv = g[((m * ho + p) * wo + q) * cout + co];
                    for (long kh = 0; kh < 3; ++kh) {
                        const long i = 2 * p + kh - 1;
                        if (i < 0 || i >= h) continue;
                        for (long kw = 0; kw < 3; ++kw) {
                            const long j = conv_col(2 * q + kw - 1, w, circ);
                            if (j < 0) continue;
                            double *dxp = dxm + (i * w + j) * cin;
                            const double *wp = wt + ((co * 3 + kh) * 3 + kw) * cin;
                            for (long ci = 0; ci < cin; ++ci) dxp[ci] += wp[ci] * gv;
                        }
                    }
                }
    }
}

void orc_conv_s2_bwd(const double *x, long n, long h, long w, long cin,
                     const double *wt, long cout, const double *g,
                     double *dw, double *db, double *dx)
{
    conv_s2_bwd(x, n, h, w, cin, wt, cout, g, dw, db, dx, 0);
}

void orc_conv_s2_bwd_pad(const double *x, long n, long h, long w, long cin,
                         const double *wt, long cout, const double *g,
                         double *dw, double *db, double *dx, int circ)
{
    conv_s2_bwd(x, n, h, w, cin, wt, cout, g, dw, db, dx, circ);
}

static void tconv_s2_bwd(const double *x, long n, long h, long w, long cin,
                         const double *wt, long cout, const double *g,
                         double *dw, double *db, double *dx, int circ)
{
    const long ho = 2 * h, wo = 2 * w;
#pragma omp parallel for schedule(static)
    for (long co = 0; co < cout; ++co) {
        double *dwc = dw + co * 9 * cin;
        for (long k = 0; k < 9 * cin; ++k) dwc[k] = 0.0;
        double sb = 0.0;
        for (long m = 0; m < n; ++m)
            for (long p = 0; p < ho; ++p)
                for (long q = 0; q < wo; ++q) {
                    const double gv = g[((m * ho + p) * wo + q) * cout + co];
                    sb += gv;
                    for (long kh = 0; kh < 3; ++kh) {
                        const long i = tconv_src(p, kh, h);
                        if (i < 0) continue;
                        for (long kw = 0; kw < 3; ++kw) {
                            const long j = tconv_src_c(q, kw, w, circ);
                            if (j < 0) continue;
                            const double *xp = x + ((m * h + i) * w + j) * cin;
                            double *dwp = dwc + (kh * 3 + kw) * cin;
                            for (long ci = 0; ci < cin; ++ci) dwp[ci] += gv * xp[ci];
                        }
                    }
                }
        if (db) db[co] = sb;
    }
    if (!dx) return;
#pragma omp parallel for schedule(static)
    for (long m = 0; m < n; ++m) {
        double *dxm = dx + m * h * w * cin;
        for (long k = 0; k < h * w * cin; ++k) dxm[k] = 0.0;
        for (long p = 0; p < ho; ++p)
            for (long q = 0; q < wo; ++q)
                for (long co = 0; co < cout; ++co) {
                    const double gv = g[((m * ho + p) * wo + q) * cout + co];
                    for (long kh = 0; kh < 3; ++kh) {
                        const long i = tconv_src(p, kh, h);
                        if (i < 0) continue;
                        for (long kw = 0; kw < 3; ++kw) {
                            const long j = tconv_src_c(q, kw, w, circ);
                            if (j < 0) continue;
                            double *dxp = dxm + (i * w + j) * cin;
                            const double *wp = wt + ((co * 3 + kh) * 3 + kw) * cin;
                            for (long ci = 0; ci < cin; ++ci) dxp[ci] += wp[ci] * gv;
                        }
                    }
                }
    }
}

void orc_tconv_s2_bwd(const double *x, long n, long h, long w, long cin,
                      const double *wt, long cout, const double *g,
                      double *dw, double *db, double *dx)
{
    tconv_s2_bwd(x, n, h, w, cin, wt, cout, g, dw, db, dx, 0);
}

void orc_tconv_s2_bwd_pad(const double *x, long n, long h, long w, long cin,
                          const double *wt, long cout, const double *g,
                          double *dw, double *db, double *dx, int circ)
{
    tconv_s2_bwd(x, n, h, w, cin, wt, cout, g, dw, db, dx, circ);
}

/* ------------------------------------------------------------------ */
/* Small helpers: concatenation along channels, ReLU with optional mask */
/* ------------------------------------------------------------------ */
static void concat_ch(const double *a, long ca, const double *b, long cb,
                      long pixels, double *out)
{
    for (long k = 0; k < pixels; ++k) {
        memcpy(out + k * (ca + cb), a + k * ca, (size_t)ca * sizeof(double));
        memcpy(out + k * (ca + cb) + ca, b + k * cb, (size_t)cb * sizeof(double));
    }
}

static void split_ch(const double *in, long ca, long cb, long pixels,
                     double *a, double *b)
{
    for (long k = 0; k < pixels; ++k) {
        memcpy(a + k * ca, in + k * (ca + cb), (size_t)ca * sizeof(double));
        memcpy(b + k * cb, in + k * (ca + cb) + ca, (size_t)cb * sizeof(double));
    }
}

/* a = relu(z) in place. With a mask, the activation is kept exactly where
 * mask != 0 (so an external mask decides the branch of the kink); without
 * one the rule is z > 0, i.e. relu(0) = 0 and relu'(0) = 0. */
static void relu_inplace(double *z, long count, const uint8_t *mask)
{
    for (long k = 0; k < count; ++k) {
        const int on = mask ? (mask[k] != 0) : (z[k] > 0.0);
        if (!on) z[k] = 0.0;
    }
}

/* Multiply a gradient by the derivative of relu at the stored activation:
 * 1 where the unit was on, 0 elsewhere. */
static void relu_grad(double *g, const double *act, long count, const uint8_t *mask)
{
    for (long k = 0; k < count; ++k) {
        const int on = mask ? (mask[k] != 0) : (act[k] > 0.0);
        if (!on) g[k] = 0.0;
    }
}

/* ------------------------------------------------------------------ */
/* Whole network, forward.                                             */
/* masks: NULL, or an array of 6 pointers (h1,h2,h3,u3,u2,y), each NULL */
/* or a uint8 mask that replaces the z > 0 rule for that activation.    */
/* ------------------------------------------------------------------ */
static void forward_impl(const double *params, const double *x, long n, long h, long w,
                         int final_relu, const uint8_t *const *masks,
                         double *h1, double *h2, double *h3, double *u3, double *u2,
                         double *y, int circ)
{
    const double *W[NUM_LAYERS], *B[NUM_LAYERS];
    for (int k = 0; k < NUM_LAYERS; ++k) {
        W[k] = params + layer_offset(k);
        B[k] = W[k] + LAYER_COUT[k] * 9 * LAYER_CIN[k];
    }
    const long p1 = n * (h / 2) * (w / 2), p2 = n * (h / 4) * (w / 4),
               p3 = n * (h / 8) * (w / 8), p0 = n * h * w;
    const uint8_t *mk[6] = {0, 0, 0, 0, 0, 0};
    if (masks)
        for (int k = 0; k < 6; ++k) mk[k] = masks[k];

    conv_s2(x, n, h, w, 7, W[L_E1], B[L_E1], 32, h1, circ);
    relu_inplace(h1, p1 * 32, mk[0]);
    conv_s2(h1, n, h / 2, w / 2, 32, W[L_E2], B[L_E2], 64, h2, circ);
    relu_inplace(h2, p2 * 64, mk[1]);
    conv_s2(h2, n, h / 4, w / 4, 64, W[L_E3], B[L_E3], 128, h3, circ);
    relu_inplace(h3, p3 * 128, mk[2]);

    tconv_s2(h3, n, h / 8, w / 8, 128, W[L_D3], B[L_D3], 64, u3, circ);
    relu_inplace(u3, p2 * 64, mk[3]);
    double *c3 = calloc((size_t)(p2 * 128), sizeof(double));
    concat_ch(u3, 64, h2, 64, p2, c3);
    tconv_s2(c3, n, h / 4, w / 4, 128, W[L_D2], B[L_D2], 32, u2, circ);
    relu_inplace(u2, p1 * 32, mk[4]);
    free(c3);
    double *c2 = calloc((size_t)(p1 * 64), sizeof(double));
    concat_ch(u2, 32, h1, 32, p1, c2);
    tconv_s2(c2, n, h / 2, w / 2, 64, W[L_D1], B[L_D1], 3, y, circ);
    if (final_relu) relu_inplace(y, p0 * 3, mk[5]);
    free(c2);
}

void orc_forward(const double *params, const double *x, long n, long h, long w,
                 int final_relu, const uint8_t *const *masks,
                 double *h1, double *h2, double *h3, double *u3, double *u2,
                 double *y)
{
    forward_impl(params, x, n, h, w, final_relu, masks, h1, h2, h3, u3, u2, y, 0);
}

void orc_forward_pad(const double *params, const double *x, long n, long h, long w,
                     int final_relu, const uint8_t *const *masks,
                     double *h1, double *h2, double *h3, double *u3, double *u2,
                     double *y, int circ)
{
    forward_impl(params, x, n, h, w, final_relu, masks, h1, h2, h3, u3, u2, y, circ);
}

/* ------------------------------------------------------------------ */
/* L1 loss, mean over all M = N*H*W*3 outputs (Sec. 6.1's mean form).  */
/* Returns L and writes dL/dy = sign(y - t) / M with sign(0) = 0.       */
/* ------------------------------------------------------------------ */
double orc_l1(const double *y, const double *t, long count, double *dy)
{
    double s = 0.0;
    for (long k = 0; k < count; ++k) {
        const double d = y[k] - t[k];
        s += fabs(d);
        if (dy) dy[k] = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) / (double)count;
    }
    return s / (double)count;
}

/* ------------------------------------------------------------------ */
/* Whole network, backward. Takes the stored activations of a forward   */
/* pass (and the same optional masks), dL/dy, and writes dL/dparams in  */
/* the flat parameter layout. dx (dL/dx) is written when non-NULL.      */
/* ------------------------------------------------------------------ */
static void backward_impl(const double *params, const double *x, long n, long h, long w,
                          int final_relu, const uint8_t *const *masks,
                          const double *h1, const double *h2, const double *h3,
                          const double *u3, const double *u2, const double *y,
                          const double *dy, double *dparams, double *dx, int circ)
{
    const double *W[NUM_LAYERS];
    double *dW[NUM_LAYERS], *dB[NUM_LAYERS];
    for (int k = 0; k < NUM_LAYERS; ++k) {
        W[k] = params + layer_offset(k);
        dW[k] = dparams + layer_offset(k);
        dB[k] = dW[k] + LAYER_COUT[k] * 9 * LAYER_CIN[k];
    }
    const long p1 = n * (h / 2) * (w / 2), p2 = n * (h / 4) * (w / 4),
               p3 = n * (h / 8) * (w / 8), p0 = n * h * w;
    const uint8_t *mk[6] = {0, 0, 0, 0, 0, 0};
    if (masks)
        for (int k = 0; k < 6; ++k) mk[k] = masks[k];

    /* D1: y = tconv(c2) */
    double *gy = malloc(sizeof(double) * p0 * 3);
    memcpy(gy, dy, sizeof(double) * p0 * 3);
    if (final_relu) relu_grad(gy, y, p0 * 3, mk[5]);
    double *c2 = calloc((size_t)(p1 * 64), sizeof(double));
    concat_ch(u2, 32, h1, 32, p1, c2);
    double *dc2 = malloc(sizeof(double) * p1 * 64);
    tconv_s2_bwd(c2, n, h / 2, w / 2, 64, W[L_D1], 3, gy, dW[L_D1], dB[L_D1], dc2, circ);
    free(c2);
    free(gy);
    double *du2 = malloc(sizeof(double) * p1 * 32);
    double *dh1 = malloc(sizeof(double) * p1 * 32); /* skip part of dc2 */
    split_ch(dc2, 32, 32, p1, du2, dh1);
    free(dc2);

    /* D2: u2 = relu(tconv(c3)) */
    relu_grad(du2, u2, p1 * 32, mk[4]);
    double *c3 = calloc((size_t)(p2 * 128), sizeof(double));
    concat_ch(u3, 64, h2, 64, p2, c3);
    double *dc3 = malloc(sizeof(double) * p2 * 128);
    tconv_s2_bwd(c3, n, h / 4, w / 4, 128, W[L_D2], 32, du2, dW[L_D2], dB[L_D2], dc3, circ);
    free(c3);
    free(du2);
    double *du3 = malloc(sizeof(double) * p2 * 64);
    double *dh2 = malloc(sizeof(double) * p2 * 64); /* skip part of dc3 */
    split_ch(dc3, 64, 64, p2, du3, dh2);
    free(dc3);

    /* D3: u3 = relu(tconv(h3)) */
    relu_grad(du3, u3, p2 * 64, mk[3]);
    double *dh3 = malloc(sizeof(double) * p3 * 128);
    tconv_s2_bwd(h3, n, h / 8, w / 8, 128, W[L_D3], 64, du3, dW[L_D3], dB[L_D3], dh3, circ);
    free(du3);

    /* E3: h3 = relu(conv(h2)); dh2 gets the encoder path added to the skip */
    relu_grad(dh3, h3, p3 * 128, mk[2]);
    double *dh2e = malloc(sizeof(double) * p2 * 64);
    conv_s2_bwd(h2, n, h / 4, w / 4, 64, W[L_E3], 128, dh3, dW[L_E3], dB[L_E3], dh2e, circ);
    free(dh3);
    for (long k = 0; k < p2 * 64; ++k) dh2[k] += dh2e[k];
    free(dh2e);

    /* E2: h2 = relu(conv(h1)) */
    relu_grad(dh2, h2, p2 * 64, mk[1]);
    double *dh1e = malloc(sizeof(double) * p1 * 32);
    conv_s2_bwd(h1, n, h / 2, w / 2, 32, W[L_E2], 64, dh2, dW[L_E2], dB[L_E2], dh1e, circ);
    free(dh2);
    for (long k = 0; k < p1 * 32; ++k) dh1[k] += dh1e[k];
    free(dh1e);

    /* E1: h1 = relu(conv(x)) */
    relu_grad(dh1, h1, p1 * 32, mk[0]);
    conv_s2_bwd(x, n, h, w, 7, W[L_E1], 32, dh1, dW[L_E1], dB[L_E1], dx, circ);
    free(dh1);
}

void orc_backward(const double *params, const double *x, long n, long h, long w,
                  int final_relu, const uint8_t *const *masks,
                  const double *h1, const double *h2, const double *h3,
                  const double *u3, const double *u2, const double *y,
                  const double *dy, double *dparams, double *dx)
{
    backward_impl(params, x, n, h, w, final_relu, masks, h1, h2, h3, u3, u2, y, dy, dparams, dx, 0);
}

void orc_backward_pad(const double *params, const double *x, long n, long h, long w,
                      int final_relu, const uint8_t *const *masks,
                      const double *h1, const double *h2, const double *h3,
                      const double *u3, const double *u2, const double *y,
                      const double *dy, double *dparams, double *dx, int circ)
{
    backward_impl(params, x, n, h, w, final_relu, masks, h1, h2, h3, u3, u2, y, dy, dparams, dx, circ);
}

/* ------------------------------------------------------------------ */
/* Adam as in PyTorch (Sec. 5 names PyTorch's Adam): t counts from 1.   */
/* ------------------------------------------------------------------ */
void orc_adam(double *theta, double *m, double *v, const double *g, long count,
              long t, double lr, double beta1, double beta2, double eps)
{
    const double bc1 = 1.0 - pow(beta1, (double)t);
    const double bc2 = 1.0 - pow(beta2, (double)t);
    for (long k = 0; k < count; ++k) {
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
        const double mhat = m[k] / bc1;
        const double vhat = v[k] / bc2;
        theta[k] -= lr * mhat / (sqrt(vhat) + eps);
    }
}
