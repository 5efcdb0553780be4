/*
 * drc_cae.h - C ABI of the MI355X (gfx950) radiance-cache autoencoder.
 *
 * The library runs the data-parallel hot path of Deep Radiance Caching
 * (Jiang & Kainz, arXiv 1910.02480): the convolutional autoencoder that
 * turns each cache point's noisy hemispherical map (radiance, normals and
 * distance, Sec. 4.3) into a clean radiance map R (Eq. 2), batched over many
 * cache points, plus the training step of that network (L1 loss, Sec. 4.3;
 * PyTorch's Adam, Sec. 5).
 *
 * Network (fully convolutional; one set of weights for every map size):
 *   h1 = relu(conv(x; W1,b1))            7 -> 32,  H/2
 *   h2 = relu(conv(h1; W2,b2))          32 -> 64,  H/4
 *   h3 = relu(conv(h2; W3,b3))          64 -> 128, H/8
 *   u3 = relu(tconv(h3; W4,b4))        128 -> 64,  H/4
 *   u2 = relu(tconv([u3|h2]; W5,b5))   128 -> 32,  H/2
 *   y  =      tconv([u2|h1]; W6,b6)     64 -> 3,   H     (linear by default)
 * conv  = 3x3 cross-correlation, stride 2, zero padding 1;
 * tconv = 3x3 transposed convolution, stride 2, padding 1, output padding 1
 *         (y[p] gathers x[i] through kernel row k where p = 2i + k - 1);
 * [a|b] = channel concatenation, decoder channels first (the skip
 *         connections of the paper's U-Net-like design, Sec. 4.3).
 *
 * Conventions shared by every call:
 * - Tensors are NHWC, contiguous, float32 at the boundary. x has 7 channels
 *   in the order R, G, B, Nx, Ny, Nz, D (Sec. 4.3); y has R, G, B.
 * - Maps are H x W with H and W multiples of 8 (three halvings) and >= 8.
 * - Parameters are one flat float32 vector: layers E1 E2 E3 D3 D2 D1, each
 *   W[co][kh][kw][ci] followed by b[co]; 206 819 values. Gradients, Adam's
 *   m and v use the same layout.
 * - All pointers named d_* are device pointers on the handle's device,
 *   16-byte aligned (256-byte aligned for workspaces). The caller owns every
 *   device buffer; the library owns only its handle, its packed low-precision
 *   weight copies and its plans.
 * - Calls only enqueue work on the given stream (hipStream_t passed as
 *   void*; NULL = the default stream). They never synchronise the device and,
 *   except the create calls, never allocate device memory.
 * - Errors: arguments are validated on the host before anything is
 *   enqueued; a failing call returns a status and enqueues nothing.
 *   Asynchronous device faults surface as DRC_ERR_HIP from a later call.
 *   drc_last_error() gives a thread-local text for the last failure.
 * - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef DRC_CAE_H
#define DRC_CAE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DRC_OK = 0,
    DRC_ERR_INVALID_ARG = 1, /* null / misaligned pointer, bad enum value */
    DRC_ERR_SHAPE = 2,       /* n < 1, H or W not a multiple of 8, ... */
    DRC_ERR_UNSUPPORTED = 3, /* a configuration this build does not implement */
    DRC_ERR_WORKSPACE = 4,   /* workspace smaller than required */
    DRC_ERR_HIP = 5,         /* a HIP runtime call failed */
    DRC_ERR_STATE = 6        /* call order: e.g. forward before set_params */
} drc_status;

typedef enum { DRC_F32 = 0, DRC_BF16 = 1, DRC_FP8_E4M3 = 2 } drc_dtype;

/* Network description. Only in_ch = 7, out_ch = 3, widths = {32, 64, 128}
 * are implemented; other values return DRC_ERR_UNSUPPORTED. compute selects
 * the arithmetic of the layer GEMMs:
 *   DRC_F32      float32 operands, float32 MFMA accumulation;
 *   DRC_BF16     bfloat16 operands and stored activations (round to nearest
 *                even), float32 accumulation, bias and activation;
 *   DRC_FP8_E4M3 OCP e4m3 operands with per-tensor scales (inference only),
 *                float32 accumulation; see drc_cae_calibrate_fp8.
 * final_relu = 1 applies relu to y (the paper's output stage has a ReLU,
 * Sec. 4.3); the default 0 keeps the output linear. Training calls require
 * final_relu = 0.
 * pad_w selects the padding of every layer along the width (azimuth):
 *   DRC_PAD_ZERO     (default) zero padding 1, as along the height;
 *   DRC_PAD_CIRCULAR the width is periodic, since a lat-long map of the
 *                    hemisphere (Sec. 4.3) wraps around in azimuth: the
 *                    convolution reads column (2q + kw - 1) mod W and the
 *                    transposed convolution adds into column (2j + kw - 1)
 *                    mod 2W; rows keep zero padding. Forward, backward and
 *                    step run layer by layer (the whole-network kernels are
 *                    zero-padding only). */
typedef enum { DRC_PAD_ZERO = 0, DRC_PAD_CIRCULAR = 1 } drc_pad;

typedef struct {
    int in_ch;
    int out_ch;
    int widths[3];
    int compute; /* drc_dtype */
    int final_relu;
    int pad_w;   /* drc_pad */
} drc_cae_desc;

/* Adam hyper-parameters (PyTorch's Adam, Sec. 5: lr = 6e-5). Doubles, as
 * PyTorch keeps them: 1 - beta1, 1 - beta2, lr / (1 - beta1^t) and
 * 1 / sqrt(1 - beta2^t) are formed in double precision and rounded once to
 * float32 for the update. */
typedef struct {
    double lr;
    double beta1;
    double beta2;
    double eps;
} drc_adam_cfg;

/* One map of a mixed-resolution frame: an h x w map whose input starts at
 * element x_off of the packed input (7 channels per pixel) and whose output
 * starts at element y_off of the packed output (3 channels per pixel). */
typedef struct {
    int h, w;
    int64_t x_off, y_off;
} drc_map_desc;

typedef struct drc_cae drc_cae;
typedef struct drc_plan drc_plan;

/* Default description: 7 -> 3 channels, widths 32/64/128, given compute. */
drc_cae_desc drc_cae_default_desc(int compute);

/* Create a handle on the current HIP device. Allocates the handle's packed
 * weight buffers (a few MB). *out is NULL on failure. */
drc_status drc_cae_create(const drc_cae_desc* desc, drc_cae** out);
void drc_cae_destroy(drc_cae* h);

/* Number of float32 values in the flat parameter vector (206 819). */
size_t drc_cae_num_params(const drc_cae* h);

/* Convert the float32 master parameters d_params into the handle's packed
 * weights (forward and transposed backward packs, in the compute type) and
 * bias copy: the network's learnable parameters (the weights and biases of
 * the six layers of Sec. 4.3, kept in float32 as the Adam state of Sec. 5).
 * Must be called before forward/backward; drc_cae_step repacks by itself
 * after its update. For FP8 handles the weight scales are computed here
 * (448 / max |W| per layer) and the call synchronises the stream to read
 * them. d_params: 206 819 floats, device, 4-byte aligned, read only.
 * Errors: DRC_ERR_INVALID_ARG for a NULL handle or a NULL / misaligned
 * d_params; DRC_ERR_HIP if the packing launch fails. The packs are
 * replaced in place: work already enqueued on another stream that still
 * reads them must be complete first. */
drc_status drc_cae_set_params(drc_cae* h, const float* d_params, void* stream);

/* Activation recompute policy for training (default 0).
 * 0: forward saves every activation (h1 h2 h3 u3 u2) in d_saved;
 * 1: forward saves only the skip tensors h1 and h2; backward recomputes
 *    h3, u3 and u2 from h2 into its workspace. Gradients are bitwise equal
 *    either way. */
drc_status drc_cae_set_recompute(drc_cae* h, int on);

/* Bytes of the d_saved buffer for an n x H x W batch under the current
 * policy, and the byte offsets of h1 h2 h3 u3 u2 inside it (each NHWC in
 * the compute type: float32, bfloat16 bits, or e4m3 bytes holding value *
 * scale); offsets of activations not saved under the policy are -1. */
drc_status drc_cae_saved_size(const drc_cae* h, int n, int H, int W, size_t* bytes,
                              int64_t offsets[5]);

/* Forward path of BF16 and FP8 handles on 32x32 and 64x64 maps (default 1).
 * 1: one kernel runs the whole network per map with its activations in LDS
 * (HBM traffic is the FP32 input and output, and for BF16 the activations
 * a saving forward must keep); the recompute of a BF16 training backward
 * (h2 -> h3, u3, u2) and its data gradients run the same way.
 * 0: one kernel per layer with activations in HBM. Both give bitwise equal
 * outputs and saved activations (same packs, K order and rounding). FP32
 * and other sizes always run layer by layer, and so do handles with
 * pad_w = DRC_PAD_CIRCULAR (created with 0). Errors: DRC_ERR_INVALID_ARG
 * for a NULL handle or on not in {0, 1}; DRC_ERR_UNSUPPORTED for on = 1 on
 * a circular-padding handle. */
drc_status drc_cae_set_fused(drc_cae* h, int on);

enum { DRC_WS_FORWARD = 1, DRC_WS_BACKWARD = 2, DRC_WS_STEP = 4, DRC_WS_CALIBRATE = 8, DRC_WS_AUTOTUNE = 16 };

/* Workspace bytes needed by the calls named in flags (an OR of DRC_WS_*)
 * for an n x H x W batch. */
drc_status drc_cae_workspace_size(const drc_cae* h, int n, int H, int W, int flags,
                                  size_t* bytes);

/* Forward pass (Sec. 4.3, Eq. 2's R): d_x [n,H,W,7] -> d_y [n,H,W,3].
 * d_saved may be NULL (inference) or a buffer of drc_cae_saved_size bytes
 * that receives the activations for a later drc_cae_backward; it must stay
 * untouched until then. d_ws: drc_cae_workspace_size(DRC_WS_FORWARD)
 * bytes (may be NULL when that size is 0).
 * Errors (nothing is enqueued): DRC_ERR_INVALID_ARG for a NULL handle,
 * NULL d_x / d_y / d_ws, d_x or d_y not 16-byte aligned, or d_saved /
 * d_ws not 256-byte aligned; DRC_ERR_SHAPE for n < 1, H or W not a
 * multiple of 8 (>= 8), or n*H*W > 2^28; DRC_ERR_WORKSPACE when ws_bytes
 * is below the required size; DRC_ERR_STATE before drc_cae_set_params
 * (FP8: before drc_cae_calibrate_fp8) or when the current device is not
 * the handle's. */
drc_status drc_cae_forward(drc_cae* h, const float* d_x, float* d_y, int n, int H, int W,
                           void* d_saved, void* d_ws, size_t ws_bytes, void* stream);

/* Backward pass of the network of Sec. 4.3 (the gradient that training
 * with the L1 loss of Sec. 4.3 and Adam, Sec. 5, needs): given d_dy =
 * dL/dy [n,H,W,3] and the d_saved of the forward pass on d_x, writes
 * dL/dparams (flat layout) to d_dparams and, when d_dx is not NULL, dL/dx
 * [n,H,W,7]. ReLU derivatives use the rule relu'(z) = [z > 0] evaluated on
 * the stored activations; a transposed convolution's data gradient is the
 * matching stride-2 convolution with channel-transposed weights and vice
 * versa; the skip concatenations split their gradient and add it to h1,
 * h2. Float32 and bfloat16 handles only. d_saved is read only (with the
 * recompute policy on, h3, u3 and u2 are recomputed into d_ws). d_ws:
 * drc_cae_workspace_size(DRC_WS_BACKWARD) bytes.
 * Errors (nothing is enqueued): DRC_ERR_INVALID_ARG for a NULL handle or
 * NULL / misaligned d_x, d_dy, d_dparams (16 bytes), d_saved, d_ws (256
 * bytes), or misaligned d_dx; DRC_ERR_SHAPE as drc_cae_forward;
 * DRC_ERR_WORKSPACE for a short workspace; DRC_ERR_STATE before
 * drc_cae_set_params or on another device; DRC_ERR_UNSUPPORTED for FP8
 * handles and for final_relu = 1. */
drc_status drc_cae_backward(drc_cae* h, const float* d_x, const float* d_dy, const void* d_saved,
                            float* d_dparams, float* d_dx, int n, int H, int W, void* d_ws,
                            size_t ws_bytes, void* stream);

/* One training step (Sec. 4.3 L1 loss, Sec. 5 Adam): forward on d_x, mean
 * L1 loss against d_target [n,H,W,3] written to d_loss (one float, device),
 * backward (recompute policy of the handle), Adam update of d_params with
 * moments d_m, d_v at step count t (>= 1), then repack of the weights.
 * dL/dy = sign(y - t) / (n H W 3) with sign(0) = 0. d_dparams may be NULL;
 * when given it receives the gradient used by the update. d_params, d_m,
 * d_v are updated in place (206 819 floats each). d_ws:
 * drc_cae_workspace_size(DRC_WS_STEP) bytes.
 * The step packs d_params itself when the handle was not packed from
 * that buffer, so drc_cae_set_params is optional here.
 * Errors (nothing is enqueued): DRC_ERR_INVALID_ARG for a NULL handle or
 * adam, bad Adam hyper-parameters (lr <= 0, betas outside [0, 1),
 * eps < 0), t < 1, or a NULL / misaligned buffer (16 bytes; d_loss 4,
 * d_ws 256); DRC_ERR_SHAPE and DRC_ERR_WORKSPACE as drc_cae_backward;
 * DRC_ERR_STATE on another device; DRC_ERR_UNSUPPORTED for FP8 handles
 * and for final_relu = 1. */
drc_status drc_cae_step(drc_cae* h, float* d_params, float* d_m, float* d_v, int64_t t,
                        const drc_adam_cfg* adam, const float* d_x, const float* d_target,
                        float* d_loss, float* d_dparams, int n, int H, int W, void* d_ws,
                        size_t ws_bytes, void* stream);

/* The training step on augmented maps (Sec. 5: the data loader rotates and
 * flips the training maps; see drc_augment for the transformation): the
 * result (loss, gradient, parameters, moments) is that of drc_cae_step on
 * the maps drc_augment(d_x, d_target, d_roll, d_flip) would write, bit for
 * bit, but no augmented copy is made: the first layer's input loaders (the
 * forward's staging of x and the E1 weight gradient's) and the loss read
 * x and the target through the rotation / mirror. d_roll, d_flip: int32
 * [n] on the device. Implemented for the whole-network BF16 path (32x32
 * and 64x64 maps, drc_cae_set_fused on, zero padding): other handles get
 * DRC_ERR_UNSUPPORTED (use drc_augment and drc_cae_step). Other errors as
 * drc_cae_step, and DRC_ERR_INVALID_ARG for a NULL or misaligned d_roll /
 * d_flip. */
drc_status drc_cae_step_aug(drc_cae* h, float* d_params, float* d_m, float* d_v, int64_t t,
                            const drc_adam_cfg* adam, const float* d_x, const float* d_target,
                            const int32_t* d_roll, const int32_t* d_flip, float* d_loss, float* d_dparams,
                            int n, int H, int W, void* d_ws, size_t ws_bytes, void* stream);

/* The training step of drc_cae_step recorded once as a HIP graph and
 * replayed, for training loops whose steps are short enough that launching
 * the step's kernels one by one costs a noticeable share of the step (the
 * paper trains with small batches, Sec. 5). create checks its arguments as
 * drc_cae_step does (same buffers, layout and errors; t is given per launch)
 * and records the step on the given non-null stream (it allocates the
 * graph). launch replays it on that stream for step count t (>= 1): every
 * buffer, pointer and shape is the one given to create, and the results are
 * bitwise those of drc_cae_step(..., t, ...) on the same state. If a call
 * has changed the handle since the recording (set_params from another
 * buffer, set_fused, set_recompute does not count), launch records the step
 * again first. Errors: create as drc_cae_step, DRC_ERR_INVALID_ARG for a
 * NULL out or the null stream, DRC_ERR_HIP if the recording fails; launch:
 * DRC_ERR_INVALID_ARG for NULL or t < 1, DRC_ERR_STATE on another device.
 * captures reports how often the step was recorded. The graph must be
 * destroyed before its handle. */
typedef struct drc_step_graph drc_step_graph;
drc_status drc_cae_step_graph_create(drc_cae* h, float* d_params, float* d_m, float* d_v, const drc_adam_cfg* adam,
                                     const float* d_x, const float* d_target, float* d_loss, float* d_dparams, int n,
                                     int H, int W, void* d_ws, size_t ws_bytes, void* stream, drc_step_graph** out);
drc_status drc_cae_step_graph_launch(drc_step_graph* g, int64_t t);
drc_status drc_cae_step_graph_captures(const drc_step_graph* g, int64_t* count);
void drc_cae_step_graph_destroy(drc_step_graph* g);

/* FP8 handles: static per-tensor activation scales (448 / max |value|) from
 * a float32 forward over the calibration batch d_x. Must follow set_params.
 * The scales of x, [u2|h1], [u3|h2] and h3 are kept in the handle. This is
 * the precision form of the network of Sec. 4.3 (the paper evaluates it in
 * float32; e4m3 with per-tensor scales is this library's inference
 * variant). d_ws: drc_cae_workspace_size(DRC_WS_CALIBRATE) bytes.
 * Synchronises the stream (the scales are read back to the host).
 * Errors: DRC_ERR_INVALID_ARG for a NULL handle or NULL / misaligned d_x,
 * d_ws; DRC_ERR_STATE for a handle that is not FP8 or before
 * drc_cae_set_params; DRC_ERR_SHAPE and DRC_ERR_WORKSPACE as
 * drc_cae_forward. */
drc_status drc_cae_calibrate_fp8(drc_cae* h, const float* d_x, int n, int H, int W, void* d_ws,
                                 size_t ws_bytes, void* stream);

/* Copy the FP8 scales to host memory: out[0..5] weight scales E1..D1,
 * out[6..9] activation scales x, [u2|h1], [u3|h2], h3. Synchronises the
 * stream. */
drc_status drc_cae_get_fp8_scales(const drc_cae* h, float out[10], void* stream);

/* Mixed-resolution frames (many maps of different sizes, one pass). The
 * network is fully convolutional, so the weights of the 32x32 maps of
 * Sec. 4.3 serve any size; larger maps keep more detail (Sec. 6.3) and
 * fixed 32x32 maps are a limitation the paper names (Sec. 7).
 * plan_create sorts the maps into resolution classes, builds per-layer work
 * lists (tile shapes per resolution from the tuning cache file, NULL =
 * built-in defaults) and uploads them (it allocates the plan's device
 * tables). maps[m]: h, w multiples of 8 (>= 8), at most 4 distinct sizes;
 * x_off, y_off >= 0 element offsets (a map whose x_off is not a multiple
 * of 4 floats runs through the layer kernels). Errors: DRC_ERR_SHAPE for
 * count < 1 or a bad size, DRC_ERR_INVALID_ARG for a negative offset or a
 * NULL handle / out, DRC_ERR_UNSUPPORTED for more than 4 sizes.
 * plan_workspace_size gives the bytes of d_ws for plan_launch.
 * plan_launch runs the whole frame on the given stream: on a non-null
 * stream as one captured HIP graph, recorded on the first launch for a
 * given (workspace, stream, x, y) and after any call that changes the
 * handle (set_params, calibrate_fp8, set_fused, set_tile, autotune), and
 * replayed otherwise; on the null stream directly. When the frame's BF16
 * 128x128 classes run through the banded kernel and every other class
 * through the whole-network kernel, their chain runs on one of the
 * handle's internal streams, forked from and joined back to the given
 * stream (inside the graph when captured), so the launch is still ordered
 * on the given stream as a whole; one handle's launches must not overlap
 * (a handle is not thread-safe). Errors:
 * DRC_ERR_INVALID_ARG for NULL / misaligned pointers, DRC_ERR_WORKSPACE,
 * DRC_ERR_STATE before set_params (FP8: calibrate_fp8). plan_destroy frees
 * the plan and its graph; the handle must outlive its plans. */
drc_status drc_cae_plan_create(drc_cae* h, const drc_map_desc* maps, int count,
                               const char* tune_cache, drc_plan** out);
drc_status drc_cae_plan_workspace_size(const drc_plan* p, size_t* bytes);
drc_status drc_cae_plan_launch(drc_plan* p, const float* d_x_packed, float* d_y_packed, void* d_ws,
                               size_t ws_bytes, void* stream);
void drc_cae_plan_destroy(drc_plan* p);
/* Number of times plan_launch has recorded the plan's graph (introspection:
 * a replay does not record). Errors: DRC_ERR_INVALID_ARG for NULL. */
drc_status drc_cae_plan_captures(const drc_plan* p, int64_t* count);

/* Forward pass that allocates nothing and takes no workspace, for callers
 * that cannot allocate device memory (code under HIP graph capture, serving
 * loops or harnesses that forbid hipMalloc): the same computation, kernels
 * and results as drc_cae_forward(h, d_x, d_y, n, H, W, NULL, ws, ...) (no
 * saved activations), with the layer path's intermediate activations in a
 * scratch array the library keeps in device memory, one per device, of
 * drc_cae_static_scratch_bytes() bytes (64 MiB; held from the first
 * drc_cae_create on that device until the process ends). The BF16
 * whole-network route of 32x32 and 64x64 maps needs no scratch; other
 * batches need drc_cae_workspace_size(DRC_WS_FORWARD) bytes of it.
 * Every call on a device shares that device's array and leaves its contents
 * behind (nothing in it has to start at zero): calls that may overlap on
 * one device, on different streams or from different threads, race and
 * must be ordered by the caller. Errors: as drc_cae_forward, plus
 * DRC_ERR_WORKSPACE when the batch needs more scratch than the array holds
 * (split the batch, or call drc_cae_forward with a workspace). */
size_t drc_cae_static_scratch_bytes(void);
drc_status drc_cae_forward_static(drc_cae* h, const float* d_x, float* d_y, int n, int H, int W, void* stream);

/* Sampling the predicted map R as an environment map (Sec. 3: the indirect
 * term alternates samples drawn from R, as from an environment map with
 * perfect visibility, with samples from the BRDF, combined by multiple
 * importance sampling; Sec. 4.3: R is a hemispherical latitude-longitude
 * map with the surface normal along +Z).
 *
 * Map geometry: row v (0 = at the normal) spans polar angles
 * [v, v + 1] * (pi / 2) / H, column u spans azimuths [u, u + 1] * 2 pi / W.
 * Directions are in the map's frame: (sin t cos p, sin t sin p, cos t).
 * Distribution: piecewise constant over the (u, v) unit square, pixel weight
 * max(0, 0.2126 R + 0.7152 G + 0.0722 B) * sin(row-centre polar angle)
 * (luminance of BT.709 primaries times the pixel's solid angle).
 * The tables are inclusive CDFs: cdf_v[m][v] = P(row <= v) and
 * cdf_u[m][v][u] = P(column <= u | row v), non-decreasing, last entry 1. A
 * row (or map) of zero total weight gets the uniform CDF (k + 1) / count,
 * and total[m] = 0 marks a map that fell back entirely.
 * Shapes: 0 <= n (n = 0 does nothing), 1 <= H <= 4096, 1 <= W <= 1024. All
 * arrays are float32 (pix int32), contiguous, device, 4-byte aligned, owned
 * by the caller. Inputs must be finite.
 *
 * build: d_y [n, H, W, 3] (e.g. drc_cae_forward's output) -> d_cdf_u
 *   [n, H, W], d_cdf_v [n, H], d_total [n] (sum of the pixel weights). */
drc_status drc_envmap_build(const float* d_y, int n, int H, int W, float* d_cdf_u, float* d_cdf_v,
                            float* d_total, void* stream);

/* S samples per map by inversion of the tables: d_xi [n, S, 2] uniforms in
 * [0, 1) (values outside are clamped; xi[0] picks the row, xi[1] the
 * column, and each places the sample linearly inside its pixel). Outputs:
 * d_dir [n, S, 3] unit directions, d_pdf [n, S] their density with respect
 * to solid angle (p(u, v) / (pi^2 sin t); 0 where sin t = 0), d_pix [n, S]
 * the pixel v * W + u. */
drc_status drc_envmap_sample(const float* d_cdf_u, const float* d_cdf_v, int n, int H, int W, int S,
                             const float* d_xi, float* d_dir, float* d_pdf, int32_t* d_pix, void* stream);

/* Solid-angle density of S directions per map, d_dir [n, S, 3] in the map's
 * frame (any non-zero length), under that map's distribution -> d_pdf
 * [n, S]; 0 below the horizon (z < 0) and along the normal. */
drc_status drc_envmap_pdf(const float* d_cdf_u, const float* d_cdf_v, int n, int H, int W, int S,
                          const float* d_dir, float* d_pdf, void* stream);

/* Interpolation between cache points (Sec. 4.2, Eqs. 4-6): for each pixel
 * of an Hi x Wi image, the probabilities of sampling the radiance maps of
 * the cache points around it. Cache points lie on a grid of spacing r
 * pixels, point (gy, gx) on pixel (gx r, gy r), Gy = (Hi - 1) / r + 1 rows
 * and Gx = (Wi - 1) / r + 1 columns, numbered gy * Gx + gx. The candidates
 * of pixel (x, y) are the corners k = 0..3 of its grid cell,
 * (x / r + (k & 1), y / r + (k >> 1)), that lie inside the grid; each gets
 * w = w_p w_n + w_p + eps with w_p = max(0, 1 - dist / r) (dist in pixels)
 * and w_n = max(0, dot of the unit normals; 0 for a zero normal). The
 * printed Eqs. 5 and 6 contradict the text around them; the text's reading
 * is taken (weight falls with distance and rises with normal agreement).
 * The weights are normalised to probabilities; if all vanish (eps = 0), the
 * present corners are equally likely. Absent corners get index -1 and
 * probability 0.
 * d_normals [Hi, Wi, 3] pixel normals (primary hits) and d_cache_normals
 * [Gy, Gx, 3], float32, any lengths, 4-byte aligned; outputs d_idx
 * [Hi, Wi, 4] int32 and d_prob [Hi, Wi, 4] float32, 16-byte aligned. eps
 * finite and >= 0; 1 <= r <= 4096; Hi * Wi < 2^31. */
drc_status drc_interp_weights(const float* d_normals, int Hi, int Wi, int r, const float* d_cache_normals,
                              float eps, int32_t* d_idx, float* d_prob, void* stream);

/* Training-data augmentation (Sec. 5: the data loader rotates and flips the
 * training maps), read as the symmetries of the hemispherical lat-long map
 * (normal along +Z, Sec. 4.3): map m is turned by d_roll[m] columns about the
 * normal (any integer, taken mod W) and, if d_flip[m] != 0, mirrored through
 * a plane containing the normal. The value of column u goes to column
 * (u + k) mod W, or (k - 1 - u) mod W when flipped (k = roll mod W); the
 * normal channels (Nx, Ny) are reflected (Ny -> -Ny) when flipped and then
 * rotated by 2 pi k / W; R, G, B, Nz, D and the target values are copied.
 * d_x [n, H, W, 7] -> d_x_out, and d_t [n, H, W, 3] -> d_t_out (both NULL to
 * leave targets out). float32, d_roll and d_flip int32 [n], all on the
 * device, 4-byte aligned; outputs must not overlap inputs. n = 0 does
 * nothing; H, W >= 1. */
drc_status drc_augment(const float* d_x, const float* d_t, int n, int H, int W, const int32_t* d_roll,
                       const int32_t* d_flip, float* d_x_out, float* d_t_out, void* stream);

/* The paper's own network (Sec. 4.3 and Sec. 5), inference form, BF16
 * activations with FP32 accumulation: a U-Net-like autoencoder with two 3x3
 * convolutions (stride 1, zero padding 1) per stage, each followed by batch
 * normalisation (running statistics, eps 1e-5) and LeakyReLU (slope 0.01);
 * 2x2 max-pool between encoder stages; decoder stages upsample 2x
 * bilinearly (half-pixel centres, edges clamped), concatenate
 * [upsampled | skip] and apply two 3x3 convolutions (the output stage
 * without batch norm); a final 1x1 convolution to 3 channels with ReLU.
 * Widths 64-128-256 with a 256-channel bottleneck (three 2x2 poolings;
 * 4.83 M weights, the 20 MB model of Sec. 5). Layer order and shapes
 * (cin -> cout): enc1a 7->64, enc1b 64->64, enc2a 64->128, enc2b 128->128,
 * enc3a 128->256, enc3b 256->256, mid_a 256->256, mid_b 256->256,
 * dec3a 512->256, dec3b 256->256, dec2a 384->128, dec2b 128->128,
 * dec1a 192->64, dec1b 64->64 (no batch norm for dec1a/dec1b), out 64->3
 * (1x1). Parameters: one flat float32 vector, per layer W[co][kh][kw][ci]
 * (the 1x1: W[co][ci]), b[co], then for batch-normalised layers gamma, beta,
 * running mean, running var (each [co]). Maps NHWC float32, x with the 7
 * channels of drc_cae_forward, y with 3; H and W multiples of 8.
 * create allocates the handle's packed weights; the other calls only
 * enqueue work on the stream (no allocation, no synchronisation). */
typedef struct drc_unet drc_unet;
drc_status drc_unet_create(drc_unet** out);
void drc_unet_destroy(drc_unet* u);
size_t drc_unet_num_params(void);
drc_status drc_unet_set_params(drc_unet* u, const float* d_params, void* stream);
drc_status drc_unet_workspace_size(int n, int H, int W, size_t* bytes);
drc_status drc_unet_forward(drc_unet* u, const float* d_x, float* d_y, int n, int H, int W, void* d_ws,
                            size_t ws_bytes, void* stream);

/* The same network's training step (Sec. 5: trained with Adam; Sec. 4.3:
 * L1 loss), FP32 throughout: a forward with batch statistics (each batch-
 * normalised layer normalises with the mean and biased variance of its
 * convolution output over the batch's n x H x W pixels, and updates its
 * running mean and variance in d_params in place with momentum 0.1, the
 * variance unbiased, as PyTorch's BatchNorm2d in training mode), the mean L1
 * loss against d_target [n,H,W,3] written to d_loss (one float), the
 * gradient of every trainable parameter (all W and b, gamma and beta; the
 * running-statistics entries get 0) written to d_dparams when it is not
 * NULL (flat layout of d_params), and Adam (PyTorch's form, drc_adam_cfg,
 * step count t >= 1) on the trainable entries; d_m and d_v have the flat
 * layout too (their running-statistics entries are left alone). d_y, when
 * not NULL, receives the forward's output [n,H,W,3]. Max-pool gradients go
 * to the first maximum of each 2x2 window (row-major), as PyTorch's.
 * Workspace: drc_unet_train_workspace_size bytes, 256-byte aligned. No
 * handle: the weights are read from d_params in place. Errors (nothing is
 * enqueued): DRC_ERR_SHAPE for n < 2 or H, W not multiples of 8 (>= 8);
 * DRC_ERR_INVALID_ARG for NULL or misaligned buffers (16 bytes; d_x, d_loss
 * and d_dparams 4), a NULL adam, bad Adam hyper-parameters or t < 1;
 * DRC_ERR_WORKSPACE for a short workspace. */
drc_status drc_unet_train_workspace_size(int n, int H, int W, size_t* bytes);
/* Where a training step leaves the activations of the 14 3x3 layers in its
 * workspace (byte offsets; float32 NHWC [n, H/d, W/d, cout] with d the
 * layer's stage divisor), for inspection: the tests read the branch
 * decisions of the GPU forward (LeakyReLU signs, max-pool choices) from
 * them. Errors as drc_unet_train_workspace_size; DRC_ERR_INVALID_ARG for a
 * NULL offsets. */
drc_status drc_unet_train_act_offsets(int n, int H, int W, int64_t offsets[14]);
drc_status drc_unet_train_step(float* d_params, float* d_m, float* d_v, int64_t t, const drc_adam_cfg* adam,
                               const float* d_x, const float* d_target, float* d_loss, float* d_dparams,
                               float* d_y, int n, int H, int W, void* d_ws, size_t ws_bytes, void* stream);

/* Tile-shape tuning: time each implemented tile shape of every layer for
 * an n x H x W forward batch on the given stream and write the fastest to
 * the JSON cache file path (keyed by arch, precision, layer and
 * resolution). Synchronises the stream. */
drc_status drc_cae_autotune(drc_cae* h, int n, int H, int W, const float* d_x, void* d_ws,
                            size_t ws_bytes, const char* tune_cache, void* stream);

/* Tile shape (pixel blocks of 16 per wave) the forward uses for layer
 * 0..5 (E1..D1) at resolution H; 0 = built-in default. */
drc_status drc_cae_set_tile(drc_cae* h, int layer, int H, int npw);

/* Weight-gradient schedule (host only; enqueues nothing, needs no GPU):
 * for layer 0..5 (E1..D1) of an n x H x W backward in compute type
 * DRC_F32 or DRC_BF16, info[0] = kernel (0: float32 MFMA with register
 * prefetch, 1: BF16 with LDS-staged operands, 2: BF16 with LDS transpose
 * reads), info[1] = reduction rows per strip (BF16) or 0, info[2] = strips
 * per workgroup chunk (BF16) or reduction pixels per chunk (float32),
 * info[3] = chunks (workgroups per tile column). Each chunk sums its strips
 * in order into one partial tile; the partial tiles are then summed in a
 * fixed order. Errors: DRC_ERR_INVALID_ARG (NULL info, bad layer or
 * compute), DRC_ERR_UNSUPPORTED (FP8), DRC_ERR_SHAPE. */
drc_status drc_cae_wgrad_schedule(int compute, int layer, int n, int H, int W, int64_t info[4]);

/* Kernel timing (profiling hook). enable = 1 creates a pool of HIP events
 * and records one event pair on the call's stream around each group of
 * kernel launches (per layer and direction); enable = 0 stops. Reading
 * waits for the recorded events, adds their elapsed times per slot
 * (ms[24], calls[24]) and clears the record. Slots: 0..5 forward GEMM of
 * E1..D1, 6..11 backward-data GEMM of E1..D1, 12..17 weight gradient of
 * E1..D1, 18 gradient sums (the bias gradients; in BF16 also the
 * fixed-order sums of every layer's weight-gradient partial tiles and of the
 * loss, run as one launch at the end of the backward), 19 L1 loss, 20 Adam
 * and repack. */
drc_status drc_cae_profile(drc_cae* h, int enable);
drc_status drc_cae_profile_read(drc_cae* h, double ms[24], int64_t calls[24]);

const char* drc_status_string(drc_status s);
const char* drc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DRC_CAE_H */
