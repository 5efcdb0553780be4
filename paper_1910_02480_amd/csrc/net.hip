// Launch sequences of the autoencoder: forward (Sec. 4.3), backward, the
// training step (L1 loss, Sec. 4.3; Adam, Sec. 5) and FP8 calibration.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "drc_cae.h"
#include "common.h"
#include "conv_layer.h"
#include "aux_kernels.h"
#include "internal.h"

using namespace drc;

#define TRY(expr)                    \
    do {                             \
        drc_status s_ = (expr);      \
        if (s_ != DRC_OK) return s_; \
    } while (0)

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return drc_fail(DRC_ERR_HIP, "%s:%d %s: %s", __FILE__, __LINE__, #expr,           \
                            hipGetErrorString(e_));                                           \
    } while (0)

// ------------------------------------------------------------------ tile shapes
// MFMA accumulator blocks (16 rows) a wave holds per 16-pixel block.
// Mirrors GemmCfg: row blocks are split over WM waves when the weight pack
// does not fit the 160 KB LDS budget (one workgroup per CU above 80 KB).
static int acc_blocks(int prec, int layer, bool backward) {
    const GemmGeom g = gemm_geom(layer, backward, prec);
    const int rb = g.rows_pad / 16;
    const long lds = (long)g.nblk * g.rows_pad * (g.kstride * prec_esize(prec) + 16);
    const int wm = (lds <= 160 * 1024 || g.mode == M_TCONV_MERGED) ? 1 : (rb % 4 == 0 ? 4 : (rb % 2 == 0 ? 2 : 1));
    return (g.mode == M_TCONV_PAIRS ? 4 * rb : rb) / wm;
}

bool npw_supported(int prec, int layer, bool backward, int npw) {
    if (npw != 1 && npw != 2 && npw != 4 && npw != 8) return false;
    if (backward && prec == P_FP8) return false;
    return acc_blocks(prec, layer, backward) * npw <= 16;
}

int default_npw(int prec, int layer, bool backward) {
    const int mt = acc_blocks(prec, layer, backward);
    int npw = mt >= 8 ? 2 : 4;
    if (mt * npw > 16) npw = std::max(1, 16 / mt);
    // FP8 operands are 32 bytes per lane: halve the tile to stay out of scratch
    return prec == P_FP8 ? std::max(1, npw / 2) : npw;
}

// Layer-GEMM launches, instantiated per precision in gemm_*.hip.
template <int P>
drc_status run_gemm(int layer, bool bwd, LayerArgs& a, int npw, int num_cu, hipStream_t s);
extern template drc_status run_gemm<P_F32>(int, bool, LayerArgs&, int, int, hipStream_t);
extern template drc_status run_gemm<P_BF16>(int, bool, LayerArgs&, int, int, hipStream_t);
extern template drc_status run_gemm<P_FP8>(int, bool, LayerArgs&, int, int, hipStream_t);
// BF16 E1 and D1 with their inputs staged in LDS by bands of rows (layer_bands.hip)
namespace drc {
bool e1_band_fits(int Hin, int Win);
drc_status e1_band_forward(const LayerArgs& a, int prec, int num_cu, hipStream_t s);
bool d1_band_fits(int Hin, int Win);
drc_status d1_band_forward(const LayerArgs& a, int prec, int num_cu, int per_cu, hipStream_t s);
}  // namespace drc

static Seg seg_none() {
    Seg s;
    memset(&s, 0, sizeof s);
    s.qscale = 1.0f;
    return s;
}
static Seg seg_out(void* dst, int c, int relu, float qscale) {
    Seg s = seg_none();
    s.dst = dst;
    s.c = c;
    s.ld = c;
    s.relu = relu;
    s.qscale = qscale;
    return s;
}

// Geometry of layer l's forward (or backward-data) GEMM for n maps of H x W.
ClassGeom class_geom(int l, int n, int H, int W, bool bwd, int circ) {
    ClassGeom G;
    memset(&G, 0, sizeof G);
    int hin, win, hout, wout;
    layer_io(l, H, W, &hin, &win, &hout, &wout);
    if (bwd) {  // the data gradient runs from the layer output back to its input
        std::swap(hin, hout);
        std::swap(win, wout);
    }
    const bool gemm_tconv = kLayers[l].tconv != bwd;
    G.nmaps = n;
    G.Hin = hin;
    G.Win = win;
    G.Hout = hout;
    G.Wout = wout;
    G.Hg = gemm_tconv ? hin : hout;
    G.Wg = gemm_tconv ? win : wout;
    G.seg0 = seg_none();
    G.seg1 = seg_none();
    G.circ = circ;
    return G;
}

static LayerArgs layer_args(const void* wpack, int kstride) {
    LayerArgs a;
    memset(&a, 0, sizeof a);
    a.nclass = 1;
    a.wpack = wpack;
    a.kstride = kstride;
    a.acc_scale = 1.0f;
    a.raw_qscale = 1.0f;
    return a;
}

// Halves the pixel blocks per wave until the launch has at least two work
// items per compute unit (small batches), keeping every CU busy.
static int fit_npw(int npw, long npix, int num_cu) {
    while (npw > 1 && (npix + 64L * npw - 1) / (64L * npw) < 2L * num_cu) npw >>= 1;
    return npw;
}

static long gemm_pixels(const LayerArgs& a) {
    long p = 0;
    for (int c = 0; c < a.nclass; ++c) p += (long)a.cls[c].nmaps * a.cls[c].Hg * a.cls[c].Wg;
    return p;
}

int pick_npw(const drc_cae* h, int l, int H, int prec, bool bwd) {
    if (!bwd) {
        auto it = h->tile.find({l, H});
        if (it != h->tile.end()) return it->second;
    }
    return default_npw(prec, l, bwd);
}

// ------------------------------------------------------------------ forward
// FP8 scale slots: 0..5 weights, 6 x, 7 [u2|h1], 8 [u3|h2], 9 h3.
static const int kInScale[6] = {6, 7, 8, 9, 8, 7};
static const int kOutScale[6] = {7, 8, 9, 8, 7, -1};

// Tensors of forward layer l for one class of maps.
static void fwd_tensors(int l, const FwdBufs& b, int final_relu, float qout, ClassGeom& G) {
    switch (l) {
        case 0:
            G.s0 = {b.x, 8, 7};
            G.in_off = b.x_off;
            G.seg0 = seg_out(b.h1, 32, 1, qout);
            break;
        case 1:
            G.s0 = {b.h1, 32, 32};
            G.seg0 = seg_out(b.h2, 64, 1, qout);
            break;
        case 2:
            G.s0 = {b.h2, 64, 64};
            G.seg0 = seg_out(b.h3, 128, 1, qout);
            break;
        case 3:
            G.s0 = {b.h3, 128, 128};
            G.seg0 = seg_out(b.u3, 64, 1, qout);
            break;
        case 4:
            G.s0 = {b.u3, 64, 64};
            G.s1 = {b.h2, 64, 64};
            G.seg0 = seg_out(b.u2, 32, 1, qout);
            break;
        case 5:
            G.s0 = {b.u2, 32, 32};
            G.s1 = {b.h1, 32, 32};
            G.seg0 = seg_out(b.y, 3, final_relu, 1.0f);
            G.out_off = b.y_off;
            break;
    }
}

// Runs layers [l0, l1] of the forward pass in precision P with packs, over
// nclass classes of maps (one launch per layer covers all classes).
template <int P>
drc_status forward_classes(drc_cae* h, void* const* packs, const FwdClass* fc, int nclass, int l0, int l1,
                           hipStream_t s, int d1_per_cu) {
    if (nclass < 1 || nclass > kMaxClasses) return drc_fail(DRC_ERR_INVALID_ARG, "forward: %d classes", nclass);
    const float* sc = h->host_scales;
    for (int l = l0; l <= l1; ++l) {
        const GemmGeom g = gemm_geom(l, false, P);
        LayerArgs a = layer_args(packs[l], g.kstride);
        a.bias = h->bias + bias_slot(l);
        float qout = 1.0f;
        if (P == P_FP8) {
            a.acc_scale = 1.0f / (sc[kInScale[l]] * sc[l]);
            if (kOutScale[l] >= 0) qout = sc[kOutScale[l]];
        }
        if (l == 0) {
            a.raw_c = 7;
            a.raw_qscale = P == P_FP8 ? sc[6] : 1.0f;
        }
        a.nclass = nclass;
        int npw = 0;
        // BF16 and FP8 E1 and D1: input rows staged in LDS by bands
        bool band = P != P_F32 && (l == 0 || l == 5) && h->desc.pad_w == DRC_PAD_ZERO;
        for (int c = 0; c < nclass; ++c) {
            a.cls[c] = class_geom(l, fc[c].n, fc[c].H, fc[c].W, false, h->desc.pad_w);
            fwd_tensors(l, fc[c].b, h->desc.final_relu, qout, a.cls[c]);
            a.cls[c].tile_px = fc[c].tile_px[l];
            if (a.cls[c].tile_px <= 0) {
                auto it = h->tile_px.find({l, fc[c].H});
                if (it != h->tile_px.end()) a.cls[c].tile_px = it->second;
            }
            band = band && (l == 0 ? fc[c].x_al16 && e1_band_fits(fc[c].H, fc[c].W)
                                   : d1_band_fits(fc[c].H / 2, fc[c].W / 2));
        }
        if (band) {
            const long tok = prof_begin(h, PROF_FWD + l, s);
            TRY(l == 0 ? e1_band_forward(a, P, h->num_cu, s) : d1_band_forward(a, P, h->num_cu, d1_per_cu, s));
            prof_end(h, tok, s);
            continue;
        }
        if (fc[0].npw[l] > 0) {
            npw = fc[0].npw[l];
        } else if (h->tile.count({l, fc[0].H})) {
            npw = pick_npw(h, l, fc[0].H, P, false);
        } else {
            npw = default_npw(P, l, false);
            bool fixed_px = false;
            for (int c = 0; c < nclass; ++c) fixed_px |= a.cls[c].tile_px > 0;
            if (!fixed_px) npw = fit_npw(npw, gemm_pixels(a), h->num_cu);
        }
        const long tok = prof_begin(h, PROF_FWD + l, s);
        TRY(run_gemm<P>(l, false, a, npw, h->num_cu, s));
        prof_end(h, tok, s);
    }
    return DRC_OK;
}
template drc_status forward_classes<P_F32>(drc_cae*, void* const*, const FwdClass*, int, int, int, hipStream_t,
                                            int);
template drc_status forward_classes<P_BF16>(drc_cae*, void* const*, const FwdClass*, int, int, int, hipStream_t,
                                            int);
template drc_status forward_classes<P_FP8>(drc_cae*, void* const*, const FwdClass*, int, int, int, hipStream_t,
                                            int);

template <int P>
static drc_status forward_seq(drc_cae* h, void* const* packs, const FwdBufs& b, int n, int H, int W,
                              int l0, int l1, hipStream_t s) {
    FwdClass fc;
    memset(&fc, 0, sizeof fc);
    fc.b = b;
    fc.n = n;
    fc.H = H;
    fc.W = W;
    fc.x_al16 = b.x_off == nullptr && (uintptr_t)b.x % 16 == 0;  // packed maps of H * W * 7 floats
    return forward_classes<P>(h, packs, &fc, 1, l0, l1, s);
}

drc_status forward_dispatch(drc_cae* h, const FwdBufs& b, int n, int H, int W, int l0, int l1,
                            hipStream_t s) {
    switch (h->prec) {
        case P_F32: return forward_seq<P_F32>(h, h->wf, b, n, H, W, l0, l1, s);
        case P_BF16: return forward_seq<P_BF16>(h, h->wf, b, n, H, W, l0, l1, s);
        case P_FP8: return forward_seq<P_FP8>(h, h->wf, b, n, H, W, l0, l1, s);
    }
    return drc_fail(DRC_ERR_STATE, "bad precision");
}

static drc_status check_ready(const drc_cae* h, const char* who) {
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "%s: handle is NULL", who);
    if (!h->params_set) return drc_fail(DRC_ERR_STATE, "%s: call drc_cae_set_params first", who);
    if (h->prec == P_FP8 && !h->calibrated)
        return drc_fail(DRC_ERR_STATE, "%s: FP8 handle needs drc_cae_calibrate_fp8 first", who);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->device)
        return drc_fail(DRC_ERR_STATE, "%s: current device %d is not the handle's device %d", who, dev,
                        h->device);
    return DRC_OK;
}

extern "C" drc_status drc_cae_forward(drc_cae* h, const float* d_x, float* d_y, int n, int H, int W,
                                      void* d_saved, void* d_ws, size_t ws_bytes, void* stream) {
    TRY(check_ready(h, "forward"));
    TRY(check_shape("forward", n, H, W));
    TRY(check_ptr("forward", "d_x", d_x, 16, false));
    TRY(check_ptr("forward", "d_y", d_y, 16, false));
    TRY(check_ptr("forward", "d_saved", d_saved, 256, true));
    TRY(check_ptr("forward", "d_ws", d_ws, 256, false));
    size_t need = 0;
    TRY(drc_cae_workspace_size(h, n, H, W, DRC_WS_FORWARD, &need));
    if (ws_bytes < need)
        return drc_fail(DRC_ERR_WORKSPACE, "forward: workspace %zu < %zu bytes", ws_bytes, need);
    if (h->fused && h->prec == P_FP8 && fused_forward_size(H, W) && !d_saved)
        return fused_fp8_forward(h, d_x, d_y, n, H, W, nullptr, nullptr, (hipStream_t)stream);
    if (h->fused && h->prec == P_BF16 && fused_forward_size(H, W)) {
        char* save[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
        if (d_saved) {
            size_t sb;
            int64_t off[5];
            TRY(drc_cae_saved_size(h, n, H, W, &sb, off));
            for (int k = 0; k < 5; ++k)
                if (off[k] >= 0) save[k] = (char*)d_saved + off[k];
        }
        return fused_forward(h, d_x, d_y, n, H, W, nullptr, nullptr, d_ws, ws_bytes, (hipStream_t)stream, save);
    }
    ActSizes a = act_sizes(h->prec, n, H, W);
    char* ws = (char*)d_ws;
    void* act[5];
    size_t cur = 0;
    for (int k = 0; k < 5; ++k) {
        act[k] = ws + cur;
        cur += a.bytes[k];
    }
    if (d_saved) {
        size_t sb;
        int64_t off[5];
        TRY(drc_cae_saved_size(h, n, H, W, &sb, off));
        for (int k = 0; k < 5; ++k)
            if (off[k] >= 0) act[k] = (char*)d_saved + off[k];
    }
    FwdBufs b{d_x, d_y, act[0], act[1], act[2], act[3], act[4], nullptr, nullptr};
    if (h->fused && h->prec == P_BF16 && !d_saved && fused_tail_size(H, W) && h->desc.pad_w == DRC_PAD_ZERO) {
        // E1-D2 in the banded kernel (h3 and u3 stay on chip), D1 through its layer kernel
        TRY(fused_tail(h, n, H, W, d_x, nullptr, b.h1, b.h2, b.u2, (hipStream_t)stream));
        return forward_dispatch(h, b, n, H, W, 5, 5, (hipStream_t)stream);
    }
    return forward_dispatch(h, b, n, H, W, 0, 5, (hipStream_t)stream);
}

// ------------------------------------------------------------------ backward
template <typename T>
static drc_status bias_grad(const void* g, bool g_raw, int C, long npix, float* partial, float* out,
                            float scale, hipStream_t s) {
    int nb;
    long per;
    colsum_split(npix, &nb, &per);
    const long nelem = npix * C;
    if (g_raw || sizeof(T) == 4)
        hipLaunchKernelGGL((colsum_partial_kernel<float, 4>), dim3(nb), dim3(256), 0, s, (const float*)g, nelem, C,
                           partial);
    else
        hipLaunchKernelGGL((colsum_partial_kernel<T, 8>), dim3(nb), dim3(256), 0, s, (const T*)g, nelem, C,
                           partial);
    hipLaunchKernelGGL(colsum_final_kernel, dim3(C), dim3(256), 0, s, (const float*)partial, nb, C, scale, out);
    return check_launch("bias_grad");
}

// Weight gradient of layer l. g: gradient at the layer output (pre-
// activation; float32 when g_raw), s0/s1: the layer input (a concatenation
// for D2 and D1; float32 x with a_raw_c channels for E1).
// All deferred gradient sums of a backward pass in one launch (GradFinal):
// workgroups [0, nbw) take 64 weight-gradient outputs each, exactly as
// wgrad_final_kernel (16 waves add chunk rows w, w + 16, ... in order, then
// the wave sums in order); the rest take four bias slots each, one 256-thread
// group per slot, exactly as bias_final_kernel (strided row sums, then a
// halving tree).
struct GradFinalArgs {
    GradFinal::Wjob w[6];
    int wblock0[7];  // first workgroup of each weight job, then the first bias workgroup
    const float* bpart;
    int bnrows, bslots;
    float bscale;
    float* bdparams;
    long boff[6];
    int bs0[7];
    int lblock;  // the loss workgroup (-1: none)
    const double* lpart;
    int lnparts;
    long lcount;
    float* loss;
};
static __global__ __launch_bounds__(1024) void grad_final_kernel(const GradFinalArgs a) {
    __shared__ float red[1024];
    __shared__ double lred[256];
    const int b = blockIdx.x;
    if (b == a.lblock) {  // threads 0..255 as l1_final_kernel's 256-thread workgroup
        const int t = threadIdx.x;
        if (t < 256) {
            double s = 0.0;
            for (int i = t; i < a.lnparts; i += 256) s += a.lpart[i];
            lred[t] = s;
        }
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) lred[t] += lred[t + o];
            __syncthreads();
        }
        if (t == 0) a.loss[0] = (float)(lred[0] / (double)a.lcount);
        return;
    }
    if (b < a.wblock0[6]) {
        int j = 0;
#pragma unroll
        for (int k = 1; k < 6; ++k)
            if (b >= a.wblock0[k]) j = k;
        const GradFinal::Wjob& J = a.w[j];
        const long count = 9L * J.qc * J.pc;
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const long e = (b - a.wblock0[j]) * 64L + lane;
        float s = 0.0f;
        if (e < count) {
            int k = wv;
            for (; k + 48 < J.nchunks; k += 64) {
                const float a0 = J.partial[(long)k * count + e], a1 = J.partial[(long)(k + 16) * count + e];
                const float a2 = J.partial[(long)(k + 32) * count + e], a3 = J.partial[(long)(k + 48) * count + e];
                s += a0; s += a1; s += a2; s += a3;
            }
            for (; k < J.nchunks; k += 16) s += J.partial[(long)k * count + e];
        }
        red[wv * 64 + lane] = s;
        __syncthreads();
        if (wv == 0 && e < count) {
            float v = 0.0f;
#pragma unroll
            for (int w = 0; w < 16; ++w) v += red[w * 64 + lane];
            const int cp = (int)(e % J.pc);
            const int jj = (int)(e / J.pc);
            const int t = jj / J.qc, c = jj - t * J.qc;
            const int co = J.q_is_cout ? c : cp, ci = J.q_is_cout ? cp : c;
            const int cin = J.q_is_cout ? J.pc : J.qc;
            J.dw[((long)co * 9 + t) * cin + ci] = v * J.scale;
        }
        return;
    }
    // bias slots 4 (b - first) .. + 3
    const int q = threadIdx.x >> 8, t = threadIdx.x & 255;
    const int c = 4 * (b - a.wblock0[6]) + q;
    float s = 0.0f;
    if (c < a.bslots)
        for (int r = t; r < a.bnrows; r += 256) s += a.bpart[(long)r * a.bslots + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (t == 0 && c < a.bslots) {
        int l = 0;
#pragma unroll
        for (int k = 1; k < 6; ++k)
            if (c >= a.bs0[k]) l = k;
        a.bdparams[a.boff[l] + (c - a.bs0[l])] = red[threadIdx.x] * a.bscale;
    }
}

drc_status grad_final_launch(const GradFinal& g, hipStream_t s) {
    GradFinalArgs a;
    memset(&a, 0, sizeof a);
    int blocks = 0;
    for (int k = 0; k < 6; ++k) {
        a.wblock0[k] = blocks;
        if (k < g.nw) {
            a.w[k] = g.w[k];
            blocks += (int)((9L * g.w[k].qc * g.w[k].pc + 63) / 64);
        }
    }
    a.wblock0[6] = blocks;
    if (g.bpart) {
        a.bpart = g.bpart;
        a.bnrows = g.bnrows;
        a.bslots = g.bslots;
        a.bscale = g.bscale;
        a.bdparams = g.bdparams;
        for (int l = 0; l < 6; ++l) a.boff[l] = g.boff[l];
        for (int l = 0; l < 7; ++l) a.bs0[l] = g.bs0[l];
        blocks += (g.bslots + 3) / 4;
    }
    a.lblock = -1;
    if (g.loss) {
        a.lblock = blocks++;
        a.lpart = g.lpart;
        a.lnparts = g.lnparts;
        a.lcount = g.lcount;
        a.loss = g.loss;
    }
    if (blocks == 0) return DRC_OK;
    hipLaunchKernelGGL(grad_final_kernel, dim3(blocks), dim3(1024), 0, s, a);
    return check_launch("gradient sums");
}

template <typename T>
static drc_status weight_grad(int l, int n, int H, int W, const void* g, bool g_raw, Src s0, Src s1,
                              int a_raw_c, float* partial, float* out, float scale, int circ, hipStream_t s,
                              const int32_t* roll = nullptr, const int32_t* flip = nullptr,
                              GradFinal* defer = nullptr) {
    // the fixed-order sum of the partial tiles: now, or recorded for grad_final_launch
    auto final_sum = [&](int nchunks, const WgradPlan& wp) -> drc_status {
        const long count = 9L * wp.qc * wp.pc;
        if (defer) {
            if (defer->nw >= 6) return drc_fail(DRC_ERR_STATE, "weight_grad: more than six deferred sums");
            defer->w[defer->nw++] = GradFinal::Wjob{partial, nchunks, wp.qc, wp.pc, (int)kLayers[l].tconv, scale, out};
            return check_launch("weight_grad");
        }
        hipLaunchKernelGGL(wgrad_final_kernel, dim3((int)((count + 63) / 64)), dim3(1024), 0, s,
                           (const float*)partial, nchunks, wp.qc, wp.pc, (int)kLayers[l].tconv, scale, out);
        return check_launch("weight_grad");
    };
    const LayerDef& L = kLayers[l];
    const WgradPlan wp = wgrad_plan(l, n, H, W, sizeof(T) == 2 ? P_BF16 : P_F32);
    int hin, win, hout, wout;
    layer_io(l, H, W, &hin, &win, &hout, &wout);
    // an augmented x is read by the transposed-read kernel's float32 staging only
    if (roll && !(l == 0 && wp.tr && wp.QR == 7))
        return drc_fail(DRC_ERR_UNSUPPORTED, "weight_grad: no augmented loader for layer %d's plan", l);
    if (wp.tr) {
        WgradTArgs b;
        memset(&b, 0, sizeof b);
        if (!L.tconv) {
            b.p = g; b.pc = L.cout; b.pc0 = L.cout; b.pld = L.cout;
            b.q = s0.p; b.qld = s0.ld; b.Hq = hin; b.Wq = win;
        } else {
            b.p = s0.p; b.p2 = s1.p; b.pc = L.cin; b.pc0 = s0.c; b.pld = s0.ld; b.p2ld = s1.ld;
            b.q = g; b.qld = L.cout; b.Hq = hout; b.Wq = wout;
        }
        b.Hr = wp.Hr;
        b.Wr = wp.Wr;
        b.circ = circ;
        b.R = wp.R;
        b.strips_per_map = wp.strips_per_map;
        b.total_strips = wp.total_strips;
        b.strips_per_chunk = wp.strips_per_chunk;
        b.partial = partial;
        b.qc = wp.qc;
        b.roll = roll;
        b.flip = flip;
        const bool raw = wp.QR > 0;
        if (raw != (l == 0 ? a_raw_c > 0 : (l == 5 ? g_raw : false)))
            return drc_fail(DRC_ERR_STATE, "weight_grad: operand type does not fit the plan of layer %d", l);
        dim3 grid(wp.bchunks, wp.bptiles);
        const int kind = wp.NW * 10000 + wp.QCP * 100 + wp.JBW * 10 + wp.BPB;
        if (b.Wq != 2 * b.Wr || b.Hq != 2 * b.Hr)
            return drc_fail(DRC_ERR_STATE, "weight_grad: transpose-read plan does not fit layer %d", l);
        const dim3 block(64 * wp.NW);
        // float32 gathered operand: staged as whole 16-byte chunks of dense
        // rows (x and dy are dense and 16-byte aligned at the boundary)
        if (raw && (b.qld != wp.QR || (uintptr_t)b.q % 16 != 0 || (b.Wq * wp.QR) % 4 != 0 ||
                    (2L * wp.R + 1) * b.Wq * wp.QR / 4 > 64L * wp.NW * (wp.QR == 7 ? kWgradTGRaw7 : kWgradTGRaw3)))
            return drc_fail(DRC_ERR_STATE, "weight_grad: float32 operand of layer %d is not staged densely", l);
        if (kind == 43254 && !raw)
            hipLaunchKernelGGL((wgrad_tr_kernel<4, 5, 4, 32, kWgradTG, kWgradTP, 0>), grid, block, wp.lds, s, b);
        else if (kind == 83238 && !raw)
            hipLaunchKernelGGL((wgrad_tr_kernel<8, 3, 8, 32, kWgradTG8, kWgradTP8, 0>), grid, block, wp.lds, s, b);
        else if (kind == 46494 && !raw)
            hipLaunchKernelGGL((wgrad_tr_kernel<4, 9, 4, 64, kWgradTG, kWgradTP, 0>), grid, block, wp.lds, s, b);
        else if (kind == 40822 && wp.QR == 7)
            hipLaunchKernelGGL((wgrad_tr_kernel<4, 2, 2, 8, kWgradTGRaw7, kWgradTP, 7>), grid, block, wp.lds, s, b);
        else if (kind == 40414 && wp.QR == 3)
            hipLaunchKernelGGL((wgrad_tr_kernel<4, 1, 4, 4, kWgradTGRaw3, kWgradTP, 3>), grid, block, wp.lds, s, b);
        else
            return drc_fail(DRC_ERR_STATE, "weight_grad: no transpose-read kernel for layer %d", l);
        return final_sum(wp.bchunks, wp);
    }
    if (wp.bf16) {
        WgradBArgs b;
        memset(&b, 0, sizeof b);
        if (!L.tconv) {
            b.p = g; b.pc = L.cout; b.pc0 = L.cout; b.pld = L.cout;
            b.q = s0.p; b.q_raw = a_raw_c > 0; b.qc = L.cin; b.qld = s0.ld; b.Hq = hin; b.Wq = win;
        } else {
            b.p = s0.p; b.p2 = s1.p; b.pc = L.cin; b.pc0 = s0.c; b.pld = s0.ld; b.p2ld = s1.ld;
            b.q = g; b.q_raw = g_raw; b.qc = L.cout; b.qld = L.cout; b.Hq = hout; b.Wq = wout;
        }
        b.nmaps = n;
        b.Hr = wp.Hr;
        b.Wr = wp.Wr;
        b.circ = circ;
        b.R = wp.R;
        b.strips_per_map = wp.strips_per_map;
        b.total_strips = wp.total_strips;
        b.strips_per_chunk = wp.strips_per_chunk;
        b.qcs = wp.qcs;
        b.partial = partial;
        dim3 grid(wp.bchunks, wp.bptiles);
        if (wp.JBW == 1 && wp.BPB == 2)
            hipLaunchKernelGGL((wgrad_bf16_kernel<1, 2, 8>), grid, dim3(256), wp.lds, s, b);
        else if (wp.JBW == 1)
            hipLaunchKernelGGL((wgrad_bf16_kernel<1, 4, 8>), grid, dim3(256), wp.lds, s, b);
        else if (wp.JBW == 5)
            hipLaunchKernelGGL((wgrad_bf16_kernel<5, 4, 32>), grid, dim3(256), wp.lds, s, b);
        else
            hipLaunchKernelGGL((wgrad_bf16_kernel<9, 4, 64>), grid, dim3(256), wp.lds, s, b);
        return final_sum(wp.bchunks, wp);
    }
    WgradArgs a;
    memset(&a, 0, sizeof a);
    if (!L.tconv) {  // plain = output gradient, gathered = layer input
        a.p = g;
        a.p_raw = g_raw;
        a.pc = L.cout;
        a.pc0 = L.cout;
        a.pld = L.cout;
        a.q = s0.p;
        a.q_raw = a_raw_c > 0;
        a.qc = L.cin;
        a.qld = s0.ld;
        a.Hq = hin;
        a.Wq = win;
    } else {         // plain = layer input (maybe a concatenation), gathered = output gradient
        a.p = s0.p;
        a.p2 = s1.p;
        a.p_raw = 0;
        a.pc = L.cin;
        a.pc0 = s0.c;
        a.pld = s0.ld;
        a.p2ld = s1.ld;
        a.q = g;
        a.q_raw = g_raw;
        a.qc = L.cout;
        a.qld = L.cout;
        a.Hq = hout;
        a.Wq = wout;
    }
    a.nmaps = n;
    a.Hr = wp.Hr;
    a.Wr = wp.Wr;
    a.circ = circ;
    a.stride = 2;
    a.per_block = wp.per_block;
    a.jtiles = wp.jtiles;
    a.partial = partial;
    dim3 grid(wp.nchunks, wp.jtiles * wp.ptiles);
    if (wp.VEC == 4)
        hipLaunchKernelGGL((wgrad_kernel<T, 4, 4, 4>), grid, dim3(256), 0, s, a);
    else if (wp.JB == 4 && wp.PB == 4)
        hipLaunchKernelGGL((wgrad_kernel<T, 4, 4, 1>), grid, dim3(256), 0, s, a);
    else if (wp.JB == 4)
        hipLaunchKernelGGL((wgrad_kernel<T, 4, 2, 1>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((wgrad_kernel<T, 2, 4, 1>), grid, dim3(256), 0, s, a);
    return final_sum(4 * wp.nchunks, wp);
}

struct BwdBufs {
    const float* x;
    const float* dy;
    const void *h1, *h2, *h3, *u3, *u2;
    float* dparams;
    float* dx;
    char* ws;
    BwdLayout L;
    const int32_t* roll = nullptr;  // x is read augmented (AugMap) by E1's weight gradient
    const int32_t* flip = nullptr;
    // a training step's L1 loss partials, summed into *loss by the backward
    // (with its other fixed-order sums when those are deferred)
    const double* lpart = nullptr;
    int lnparts = 0;
    long lcount = 0;
    float* loss = nullptr;
};

template <int P>
static drc_status backward_seq(drc_cae* h, const BwdBufs& b, int n, int H, int W, float gscale,
                               hipStream_t s) {
    typedef typename Traits<P>::T T;
    char* ws = b.ws;
    const BwdLayout& L = b.L;
    void* dz_u2 = ws + L.dz_u2;
    void* dh1s = ws + L.dh1s;
    void* dz_u3 = ws + L.dz_u3;
    void* dh2s = ws + L.dh2s;
    void* dz_h3 = ws + L.dz_h3;
    void* dz_h2 = ws + L.dz_h2;
    void* dz_h1 = ws + L.dz_h1;
    float* bpart = (float*)(ws + L.bpart);
    // FP32: the weight gradients run on the handle's side streams, each
    // forked after the data gradient it reads and joined before the call
    // returns (each layer has its own partial tiles); 4096 maps of 64x64:
    // forward + backward 9 % faster. BF16 keeps them on the stream: there
    // the large-LDS weight-gradient kernels do not share CUs and the forks
    // made the 256-map training step 7 % slower.
    constexpr bool kFork = P == P_F32;
    const int circ = h->desc.pad_w;  // circular width: every gather wraps columns
    auto wgrad_on = [&](int l, auto&& launch) -> drc_status {
        hipStream_t ss = kFork ? h->side[l % drc_cae::kSide] : s;
        if (kFork) {
            HIPCHK(hipEventRecord(h->ev_fork[l], s));
            HIPCHK(hipStreamWaitEvent(ss, h->ev_fork[l], 0));
        }
        const long tok = prof_begin(h, PROF_WGRAD + l, ss);
        TRY(launch((float*)(ws + L.wpart[l]), ss));
        prof_end(h, tok, ss);
        return DRC_OK;
    };
    ActSizes as = act_sizes(P, n, H, W);
    float* dp = b.dparams;
    // on one stream, the fixed-order gradient sums (weights, and the biases
    // of the data-gradient chain) run as one launch after the last weight
    // gradient instead of one small launch each
    GradFinal gf;
    GradFinal* dfr = kFork ? nullptr : &gf;
    if (b.loss) {
        if (dfr) {
            gf.lpart = b.lpart;
            gf.lnparts = b.lnparts;
            gf.lcount = b.lcount;
            gf.loss = b.loss;
        } else {
            const long ltok = prof_begin(h, PROF_LOSS, s);
            hipLaunchKernelGGL(l1_final_kernel, dim3(1), dim3(256), 0, s, b.lpart, b.lnparts, b.lcount, b.loss);
            prof_end(h, ltok, s);
            TRY(check_launch("step/l1 final"));
        }
    }
    // BF16 32x32 / 64x64: all data gradients of D1..E2 in one kernel first
    const bool fdg = P == P_BF16 && h->fused && fused_forward_size(H, W);
    if (fdg)
        TRY(fused_dgrad(h, n, H, W, b.dy, b.u2, b.u3, b.h3, b.h2, b.h1, dz_u2, dh1s, dz_u3, dz_h3, dz_h2, dz_h1,
                        bpart, L.bpart_bytes, dp, gscale, s, dfr));

    // D1: y = tconv([u2|h1]); its data gradient is a stride-2 conv of dy.
    {
        const GemmGeom g = gemm_geom(5, true, P);
        LayerArgs a = layer_args(h->wb[5], g.kstride);
        ClassGeom& G = a.cls[0];
        G = class_geom(5, n, H, W, true, circ);
        G.s0 = {b.dy, g.cin_eff, 3};
        a.raw_c = 3;
        G.seg0 = seg_out(dz_u2, 32, 0, 1.0f);
        G.seg0.mask = b.u2;
        G.seg0.ldm = 32;
        G.seg1 = seg_out(dh1s, 32, 0, 1.0f);
        if (!fdg) { const long tok = prof_begin(h, PROF_BWD + 5, s);
        TRY(run_gemm<P>(5, true, a, fit_npw(default_npw(P, 5, true), gemm_pixels(a), h->num_cu), h->num_cu, s));
        prof_end(h, tok, s); }
        TRY(wgrad_on(5, [&](float* wpart, hipStream_t ss) {
            return weight_grad<T>(5, n, H, W, b.dy, true, Src{b.u2, 32, 32}, Src{b.h1, 32, 32}, 0, wpart,
                                  dp + layer_w_offset(5), gscale, circ, ss, nullptr, nullptr, dfr);
        }));
        if (!fdg) { const long tok = prof_begin(h, PROF_BIAS, s);
        TRY(bias_grad<T>(b.dy, true, 3, as.p0, bpart, dp + layer_b_offset(5), gscale, s));
        prof_end(h, tok, s); }
    }
    // D2: u2 = relu(tconv([u3|h2]))
    {
        const GemmGeom g = gemm_geom(4, true, P);
        LayerArgs a = layer_args(h->wb[4], g.kstride);
        ClassGeom& G = a.cls[0];
        G = class_geom(4, n, H, W, true, circ);
        G.s0 = {dz_u2, 32, 32};
        G.seg0 = seg_out(dz_u3, 64, 0, 1.0f);
        G.seg0.mask = b.u3;
        G.seg0.ldm = 64;
        G.seg1 = seg_out(dh2s, 64, 0, 1.0f);
        if (!fdg) { const long tok = prof_begin(h, PROF_BWD + 4, s);
        TRY(run_gemm<P>(4, true, a, fit_npw(default_npw(P, 4, true), gemm_pixels(a), h->num_cu), h->num_cu, s));
        prof_end(h, tok, s); }
        TRY(wgrad_on(4, [&](float* wpart, hipStream_t ss) {
            return weight_grad<T>(4, n, H, W, dz_u2, false, Src{b.u3, 64, 64}, Src{b.h2, 64, 64}, 0, wpart,
                                  dp + layer_w_offset(4), gscale, circ, ss, nullptr, nullptr, dfr);
        }));
        if (!fdg) { const long tok = prof_begin(h, PROF_BIAS, s);
        TRY(bias_grad<T>(dz_u2, false, 32, as.p1, bpart, dp + layer_b_offset(4), gscale, s));
        prof_end(h, tok, s); }
    }
    // D3: u3 = relu(tconv(h3))
    {
        const GemmGeom g = gemm_geom(3, true, P);
        LayerArgs a = layer_args(h->wb[3], g.kstride);
        ClassGeom& G = a.cls[0];
        G = class_geom(3, n, H, W, true, circ);
        G.s0 = {dz_u3, 64, 64};
        G.seg0 = seg_out(dz_h3, 128, 0, 1.0f);
        G.seg0.mask = b.h3;
        G.seg0.ldm = 128;
        if (!fdg) { const long tok = prof_begin(h, PROF_BWD + 3, s);
        TRY(run_gemm<P>(3, true, a, fit_npw(default_npw(P, 3, true), gemm_pixels(a), h->num_cu), h->num_cu, s));
        prof_end(h, tok, s); }
        TRY(wgrad_on(3, [&](float* wpart, hipStream_t ss) {
            return weight_grad<T>(3, n, H, W, dz_u3, false, Src{b.h3, 128, 128}, Src{nullptr, 0, 0}, 0, wpart,
                                  dp + layer_w_offset(3), gscale, circ, ss, nullptr, nullptr, dfr);
        }));
        if (!fdg) { const long tok = prof_begin(h, PROF_BIAS, s);
        TRY(bias_grad<T>(dz_u3, false, 64, as.p2, bpart, dp + layer_b_offset(3), gscale, s));
        prof_end(h, tok, s); }
    }
    // E3: h3 = relu(conv(h2)); dh2 = skip part + encoder part
    {
        const GemmGeom g = gemm_geom(2, true, P);
        LayerArgs a = layer_args(h->wb[2], g.kstride);
        ClassGeom& G = a.cls[0];
        G = class_geom(2, n, H, W, true, circ);
        G.s0 = {dz_h3, 128, 128};
        G.seg0 = seg_out(dz_h2, 64, 0, 1.0f);
        G.seg0.add = dh2s;
        G.seg0.lda = 64;
        G.seg0.mask = b.h2;
        G.seg0.ldm = 64;
        if (!fdg) { const long tok = prof_begin(h, PROF_BWD + 2, s);
        TRY(run_gemm<P>(2, true, a, fit_npw(default_npw(P, 2, true), gemm_pixels(a), h->num_cu), h->num_cu, s));
        prof_end(h, tok, s); }
        TRY(wgrad_on(2, [&](float* wpart, hipStream_t ss) {
            return weight_grad<T>(2, n, H, W, dz_h3, false, Src{b.h2, 64, 64}, Src{nullptr, 0, 0}, 0, wpart,
                                  dp + layer_w_offset(2), gscale, circ, ss, nullptr, nullptr, dfr);
        }));
        if (!fdg) { const long tok = prof_begin(h, PROF_BIAS, s);
        TRY(bias_grad<T>(dz_h3, false, 128, as.p3, bpart, dp + layer_b_offset(2), gscale, s));
        prof_end(h, tok, s); }
    }
    // E2: h2 = relu(conv(h1))
    {
        const GemmGeom g = gemm_geom(1, true, P);
        LayerArgs a = layer_args(h->wb[1], g.kstride);
        ClassGeom& G = a.cls[0];
        G = class_geom(1, n, H, W, true, circ);
        G.s0 = {dz_h2, 64, 64};
        G.seg0 = seg_out(dz_h1, 32, 0, 1.0f);
        G.seg0.add = dh1s;
        G.seg0.lda = 32;
        G.seg0.mask = b.h1;
        G.seg0.ldm = 32;
        if (!fdg) { const long tok = prof_begin(h, PROF_BWD + 1, s);
        TRY(run_gemm<P>(1, true, a, fit_npw(default_npw(P, 1, true), gemm_pixels(a), h->num_cu), h->num_cu, s));
        prof_end(h, tok, s); }
        TRY(wgrad_on(1, [&](float* wpart, hipStream_t ss) {
            return weight_grad<T>(1, n, H, W, dz_h2, false, Src{b.h1, 32, 32}, Src{nullptr, 0, 0}, 0, wpart,
                                  dp + layer_w_offset(1), gscale, circ, ss, nullptr, nullptr, dfr);
        }));
        if (!fdg) { const long tok = prof_begin(h, PROF_BIAS, s);
        TRY(bias_grad<T>(dz_h2, false, 64, as.p2, bpart, dp + layer_b_offset(1), gscale, s));
        prof_end(h, tok, s); }
    }
    // E1: h1 = relu(conv(x))
    {
        TRY(wgrad_on(0, [&](float* wpart, hipStream_t ss) {
            return weight_grad<T>(0, n, H, W, dz_h1, false, Src{b.x, 7, 7}, Src{nullptr, 0, 0}, 7, wpart,
                                  dp + layer_w_offset(0), gscale, circ, ss, b.roll, b.flip, dfr);
        }));
        if (!fdg) { const long tok = prof_begin(h, PROF_BIAS, s);
        TRY(bias_grad<T>(dz_h1, false, 32, as.p1, bpart, dp + layer_b_offset(0), gscale, s));
        prof_end(h, tok, s); }
        if (b.dx) {
            const GemmGeom g = gemm_geom(0, true, P);
            LayerArgs a = layer_args(h->wb[0], g.kstride);
            ClassGeom& G = a.cls[0];
            G = class_geom(0, n, H, W, true, circ);
            G.s0 = {dz_h1, 32, 32};
            a.acc_scale = gscale;
            G.seg0 = seg_out(b.dx, 7, 0, 1.0f);
            { const long tok = prof_begin(h, PROF_BWD + 0, s);
            TRY(run_gemm<P>(0, true, a, fit_npw(default_npw(P, 0, true), gemm_pixels(a), h->num_cu), h->num_cu, s));
            prof_end(h, tok, s); }
        }
    }
    if (dfr) {
        const long tok = prof_begin(h, PROF_BIAS, s);
        TRY(grad_final_launch(gf, s));
        prof_end(h, tok, s);
    }
    // join the side streams
    for (int k = 0; k < drc_cae::kSide && kFork; ++k) {
        HIPCHK(hipEventRecord(h->ev_join[k], h->side[k]));
        HIPCHK(hipStreamWaitEvent(s, h->ev_join[k], 0));
    }
    return DRC_OK;
}

// Recompute h3, u3 and u2 from the saved h2 (layers E3, D3, D2).
static drc_status recompute_acts(drc_cae* h, BwdBufs& b, int n, int H, int W, hipStream_t s) {
    FwdBufs f{nullptr, nullptr, const_cast<void*>(b.h1), const_cast<void*>(b.h2), b.ws + b.L.recomp[0],
              b.ws + b.L.recomp[1], b.ws + b.L.recomp[2], nullptr, nullptr};
    if (h->fused && h->prec == P_BF16 && fused_forward_size(H, W))
        TRY(fused_recompute(h, n, H, W, b.h2, f.h3, f.u3, f.u2, s));
    else
        TRY(forward_dispatch(h, f, n, H, W, 2, 4, s));
    b.h3 = f.h3;
    b.u3 = f.u3;
    b.u2 = f.u2;
    return DRC_OK;
}

static drc_status backward_dispatch(drc_cae* h, BwdBufs& b, int n, int H, int W, float gscale,
                                    hipStream_t s) {
    if (h->prec == P_F32) return backward_seq<P_F32>(h, b, n, H, W, gscale, s);
    if (h->prec == P_BF16) return backward_seq<P_BF16>(h, b, n, H, W, gscale, s);
    return drc_fail(DRC_ERR_UNSUPPORTED, "backward: FP8 handles are inference only");
}

extern "C" drc_status drc_cae_backward(drc_cae* h, const float* d_x, const float* d_dy,
                                       const void* d_saved, float* d_dparams, float* d_dx, int n, int H,
                                       int W, void* d_ws, size_t ws_bytes, void* stream) {
    TRY(check_ready(h, "backward"));
    if (h->prec == P_FP8) return drc_fail(DRC_ERR_UNSUPPORTED, "backward: FP8 handles are inference only");
    if (h->desc.final_relu) return drc_fail(DRC_ERR_UNSUPPORTED, "backward: final_relu = 1 is inference only");
    TRY(check_shape("backward", n, H, W));
    TRY(check_ptr("backward", "d_x", d_x, 16, false));
    TRY(check_ptr("backward", "d_dy", d_dy, 16, false));
    TRY(check_ptr("backward", "d_saved", d_saved, 256, false));
    TRY(check_ptr("backward", "d_dparams", d_dparams, 16, false));
    TRY(check_ptr("backward", "d_dx", d_dx, 16, true));
    TRY(check_ptr("backward", "d_ws", d_ws, 256, false));
    size_t need = 0;
    TRY(drc_cae_workspace_size(h, n, H, W, DRC_WS_BACKWARD, &need));
    if (ws_bytes < need)
        return drc_fail(DRC_ERR_WORKSPACE, "backward: workspace %zu < %zu bytes", ws_bytes, need);
    size_t sb;
    int64_t off[5];
    TRY(drc_cae_saved_size(h, n, H, W, &sb, off));
    BwdBufs b;
    b.x = d_x;
    b.dy = d_dy;
    const char* sv = (const char*)d_saved;
    b.h1 = sv + off[0];
    b.h2 = sv + off[1];
    b.h3 = off[2] >= 0 ? sv + off[2] : nullptr;
    b.u3 = off[3] >= 0 ? sv + off[3] : nullptr;
    b.u2 = off[4] >= 0 ? sv + off[4] : nullptr;
    b.dparams = d_dparams;
    b.dx = d_dx;
    b.ws = (char*)d_ws;
    b.L = bwd_layout(h->prec, n, H, W, true);
    hipStream_t s = (hipStream_t)stream;
    if (h->recompute) TRY(recompute_acts(h, b, n, H, W, s));
    return backward_dispatch(h, b, n, H, W, 1.0f, s);
}

// ------------------------------------------------------------------ training step
// Host-side checks of a training step (nothing is enqueued).
static drc_status check_step(drc_cae* h, const float* d_params, const float* d_m, const float* d_v,
                             const drc_adam_cfg* adam, const float* d_x, const float* d_target, const float* d_loss,
                             const float* d_dparams, int n, int H, int W, const void* d_ws, size_t ws_bytes,
                             const char* who) {
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "%s: handle is NULL", who);
    if (h->prec == P_FP8) return drc_fail(DRC_ERR_UNSUPPORTED, "%s: FP8 handles are inference only", who);
    if (h->desc.final_relu) return drc_fail(DRC_ERR_UNSUPPORTED, "%s: final_relu = 1 is inference only", who);
    TRY(check_shape(who, n, H, W));
    TRY(check_ptr(who, "d_params", d_params, 16, false));
    TRY(check_ptr(who, "d_m", d_m, 16, false));
    TRY(check_ptr(who, "d_v", d_v, 16, false));
    TRY(check_ptr(who, "d_x", d_x, 16, false));
    TRY(check_ptr(who, "d_target", d_target, 16, false));
    TRY(check_ptr(who, "d_loss", d_loss, 4, false));
    TRY(check_ptr(who, "d_dparams", d_dparams, 16, true));
    TRY(check_ptr(who, "d_ws", d_ws, 256, false));
    if (!adam) return drc_fail(DRC_ERR_INVALID_ARG, "%s: adam is NULL", who);
    if (!(adam->lr > 0) || !(adam->beta1 >= 0 && adam->beta1 < 1) || !(adam->beta2 >= 0 && adam->beta2 < 1) ||
        !(adam->eps >= 0))
        return drc_fail(DRC_ERR_INVALID_ARG, "%s: bad Adam hyper-parameters", who);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->device)
        return drc_fail(DRC_ERR_STATE, "%s: current device is not the handle's device", who);
    const StepLayout S = step_layout(h->prec, n, H, W, h->recompute);
    if (ws_bytes < S.total)
        return drc_fail(DRC_ERR_WORKSPACE, "%s: workspace %zu < %zu bytes", who, ws_bytes, S.total);
    return DRC_OK;
}

// Adam's step-dependent factors, formed in double precision as PyTorch does
// and rounded once to float32: lr / (1 - beta1^t) and 1 / sqrt(1 - beta2^t).
static void adam_factors(const drc_adam_cfg* adam, int64_t t, float* step_size, float* inv_sqrt_bc2) {
    const double bc1 = 1.0 - std::pow(adam->beta1, (double)t);
    const double bc2 = 1.0 - std::pow(adam->beta2, (double)t);
    *step_size = (float)(adam->lr / bc1);
    *inv_sqrt_bc2 = (float)(1.0 / std::sqrt(bc2));
}

// Enqueue one training step (arguments already checked).
static drc_status step_enqueue(drc_cae* h, float* d_params, float* d_m, float* d_v, int64_t t,
                               const drc_adam_cfg* adam, const float* d_x, const float* d_target, float* d_loss,
                               float* d_dparams, int n, int H, int W, void* d_ws, void* stream,
                               const int32_t* roll = nullptr, const int32_t* flip = nullptr) {
    const StepLayout S = step_layout(h->prec, n, H, W, h->recompute);
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_ws;

    if (!h->params_set || h->packed_from != d_params) TRY(drc_cae_set_params(h, d_params, stream));

    // forward: skip tensors in the saved region, the rest in scratch (recompute) or saved
    ActSizes a = act_sizes(h->prec, n, H, W);
    int64_t off[5];
    size_t sb;
    TRY(drc_cae_saved_size(h, n, H, W, &sb, off));
    void* act[5];
    size_t scur = S.fwd_scratch;
    for (int k = 0; k < 5; ++k) {
        if (off[k] >= 0) {
            act[k] = ws + S.saved + off[k];
        } else {
            act[k] = ws + scur;
            scur += a.bytes[k];
        }
    }
    float* y = (float*)(ws + S.y);
    float* dy = (float*)(ws + S.dy);
    FwdBufs fb{d_x, y, act[0], act[1], act[2], act[3], act[4], nullptr, nullptr};
    if (h->fused && h->prec == P_BF16 && fused_forward_size(H, W)) {
        // one kernel; it writes the activations the backward reads
        char* save[5];
        for (int k = 0; k < 5; ++k) save[k] = off[k] >= 0 ? (char*)act[k] : nullptr;
        TRY(fused_forward(h, d_x, y, n, H, W, nullptr, nullptr, nullptr, 0, s, save, roll, flip));
    } else {
        if (roll) return drc_fail(DRC_ERR_UNSUPPORTED, "step_aug: the layer path has no augmented loaders");
        TRY(forward_dispatch(h, fb, n, H, W, 0, 5, s));
    }

    // L1 loss (mean) and dL/dy; dy is stored as sign(y - t) and the 1/M
    // factor is applied once, to the parameter gradients.
    const long M = a.p0 * 3;
    const int nparts = (int)((M + kLossPerBlock - 1) / kLossPerBlock);
    const long ltok = prof_begin(h, PROF_LOSS, s);
    hipLaunchKernelGGL(l1_partial_kernel, dim3(nparts), dim3(256), 0, s, (const float*)y, d_target, M, kLossPerBlock,
                       1.0f, dy, (double*)(ws + S.loss_part), roll, flip, H, W);
    prof_end(h, ltok, s);
    TRY(check_launch("step/l1"));

    BwdBufs b;
    b.x = d_x;
    b.dy = dy;
    b.h1 = act[0];
    b.h2 = act[1];
    b.h3 = act[2];
    b.u3 = act[3];
    b.u2 = act[4];
    b.dparams = d_dparams ? d_dparams : (float*)(ws + S.dparams);
    b.dx = nullptr;
    b.ws = ws + S.bwd;
    b.L = bwd_layout(h->prec, n, H, W, h->recompute != 0);
    b.roll = roll;
    b.flip = flip;
    b.lpart = (const double*)(ws + S.loss_part);  // the loss: summed by the backward
    b.lnparts = nparts;
    b.lcount = M;
    b.loss = d_loss;
    if (h->recompute) TRY(recompute_acts(h, b, n, H, W, s));
    TRY(backward_dispatch(h, b, n, H, W, (float)(1.0 / (double)M), s));

    // Adam (PyTorch form), then repack the weights from the new masters.
    float step_size, inv_sqrt_bc2;
    adam_factors(adam, t, &step_size, &inv_sqrt_bc2);
    const long P = (long)drc_cae_num_params(h);
    const long atok = prof_begin(h, PROF_ADAM, s);
    hipLaunchKernelGGL(adam_kernel, dim3((int)((P + 255) / 256)), dim3(256), 0, s, d_params, d_m, d_v,
                       (const float*)b.dparams, P, (float)adam->beta1, (float)(1.0 - adam->beta1),
                       (float)adam->beta2, (float)(1.0 - adam->beta2), step_size, inv_sqrt_bc2,
                       (float)adam->eps);
    TRY(check_launch("step/adam"));
    const drc_status st = drc_cae_set_params(h, d_params, stream);
    prof_end(h, atok, s);
    return st;
}

extern "C" drc_status drc_cae_step(drc_cae* h, float* d_params, float* d_m, float* d_v, int64_t t,
                                   const drc_adam_cfg* adam, const float* d_x, const float* d_target,
                                   float* d_loss, float* d_dparams, int n, int H, int W, void* d_ws,
                                   size_t ws_bytes, void* stream) {
    TRY(check_step(h, d_params, d_m, d_v, adam, d_x, d_target, d_loss, d_dparams, n, H, W, d_ws, ws_bytes,
                   "step"));
    if (t < 1) return drc_fail(DRC_ERR_INVALID_ARG, "step: t = %lld (must be >= 1)", (long long)t);
    return step_enqueue(h, d_params, d_m, d_v, t, adam, d_x, d_target, d_loss, d_dparams, n, H, W, d_ws, stream);
}

extern "C" drc_status drc_cae_step_aug(drc_cae* h, float* d_params, float* d_m, float* d_v, int64_t t,
                                       const drc_adam_cfg* adam, const float* d_x, const float* d_target,
                                       const int32_t* d_roll, const int32_t* d_flip, float* d_loss,
                                       float* d_dparams, int n, int H, int W, void* d_ws, size_t ws_bytes,
                                       void* stream) {
    TRY(check_step(h, d_params, d_m, d_v, adam, d_x, d_target, d_loss, d_dparams, n, H, W, d_ws, ws_bytes,
                   "step_aug"));
    if (t < 1) return drc_fail(DRC_ERR_INVALID_ARG, "step_aug: t = %lld (must be >= 1)", (long long)t);
    TRY(check_ptr("step_aug", "d_roll", d_roll, 4, false));
    TRY(check_ptr("step_aug", "d_flip", d_flip, 4, false));
    if (!(h->fused && h->prec == P_BF16 && fused_forward_size(H, W)))
        return drc_fail(DRC_ERR_UNSUPPORTED,
                        "step_aug: augmented loaders exist in the whole-network BF16 path (32x32, 64x64) only; "
                        "use drc_augment and drc_cae_step");
    return step_enqueue(h, d_params, d_m, d_v, t, adam, d_x, d_target, d_loss, d_dparams, n, H, W, d_ws, stream,
                        d_roll, d_flip);
}

// ------------------------------------------------------------------ captured training step
// One training step recorded once as a HIP graph and replayed per step. The
// only argument that changes from step to step, the step count t, enters
// through Adam's two bias-correction factors: the replay rewrites the
// arguments of the graph's Adam kernel node (same values as drc_cae_step
// computes), so a replayed step is the eager step bit for bit.
struct drc_step_graph {
    drc_cae* h = nullptr;
    float *params = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr, *dparams = nullptr;
    const float *x = nullptr, *target = nullptr;
    drc_adam_cfg adam{};
    int n = 0, H = 0, W = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t adam_node = nullptr;
    hipKernelNodeParams adam_params{};
    // the Adam node's arguments, in adam_kernel's parameter order, owned here
    struct {
        float* theta;
        float* m;
        float* v;
        const float* g;
        long count;
        float b1, omb1, b2, omb2, step_size, inv_sqrt_bc2, eps;
    } adam_args{};
    void* adam_argv[12] = {};
    unsigned long gen = 0;  // handle generation the graph was recorded at
    long captures = 0;
};

static void step_graph_release(drc_step_graph* g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->exec = nullptr;
    g->graph = nullptr;
    g->adam_node = nullptr;
}

// Record the step on g->stream and find the Adam kernel node.
static drc_status step_graph_record(drc_step_graph* g) {
    step_graph_release(g);
    drc_cae* h = g->h;
    const bool prof = h->prof;
    h->prof = false;  // no timing events inside the graph
    HIPCHK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
    const drc_status st = step_enqueue(h, g->params, g->m, g->v, 1, &g->adam, g->x, g->target, g->loss,
                                       g->dparams, g->n, g->H, g->W, g->ws, g->stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(g->stream, &graph);
    h->prof = prof;
    if (st != DRC_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return drc_fail(DRC_ERR_HIP, "step_graph: capture failed: %s", hipGetErrorString(e));
    g->graph = graph;
    size_t nn = 0;
    HIPCHK(hipGraphGetNodes(graph, nullptr, &nn));
    std::vector<hipGraphNode_t> nodes(nn);
    HIPCHK(hipGraphGetNodes(graph, nodes.data(), &nn));
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        if (hipGraphNodeGetType(nd, &ty) != hipSuccess || ty != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp;
        if (hipGraphKernelNodeGetParams(nd, &kp) != hipSuccess) continue;
        if (kp.func == reinterpret_cast<void*>(&adam_kernel)) {
            if (g->adam_node) return drc_fail(DRC_ERR_HIP, "step_graph: two Adam nodes in the recorded step");
            if (!kp.kernelParams) return drc_fail(DRC_ERR_HIP, "step_graph: Adam node without arguments");
            g->adam_node = nd;
            auto& A = g->adam_args;
            void** in = kp.kernelParams;
            A.theta = *(float**)in[0];
            A.m = *(float**)in[1];
            A.v = *(float**)in[2];
            A.g = *(const float**)in[3];
            A.count = *(long*)in[4];
            float* fl[7] = {&A.b1, &A.omb1, &A.b2, &A.omb2, &A.step_size, &A.inv_sqrt_bc2, &A.eps};
            for (int i = 0; i < 7; ++i) *fl[i] = *(float*)in[5 + i];
            void* argv[12] = {&A.theta, &A.m, &A.v, &A.g, &A.count, &A.b1, &A.omb1, &A.b2, &A.omb2,
                              &A.step_size, &A.inv_sqrt_bc2, &A.eps};
            memcpy(g->adam_argv, argv, sizeof argv);
            g->adam_params = kp;
            g->adam_params.kernelParams = g->adam_argv;
            g->adam_params.extra = nullptr;
        }
    }
    if (!g->adam_node) return drc_fail(DRC_ERR_HIP, "step_graph: the recorded step has no Adam node");
    if (g->adam_args.theta != g->params || g->adam_args.m != g->m || g->adam_args.v != g->v)
        return drc_fail(DRC_ERR_HIP, "step_graph: unexpected Adam node arguments");
    HIPCHK(hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0));
    g->gen = h->gen;
    g->captures++;
    return DRC_OK;
}

extern "C" drc_status drc_cae_step_graph_create(drc_cae* h, float* d_params, float* d_m, float* d_v,
                                                const drc_adam_cfg* adam, const float* d_x, const float* d_target,
                                                float* d_loss, float* d_dparams, int n, int H, int W, void* d_ws,
                                                size_t ws_bytes, void* stream, drc_step_graph** out) {
    if (!out) return drc_fail(DRC_ERR_INVALID_ARG, "step_graph_create: out is NULL");
    *out = nullptr;
    TRY(check_step(h, d_params, d_m, d_v, adam, d_x, d_target, d_loss, d_dparams, n, H, W, d_ws, ws_bytes,
                   "step_graph_create"));
    if (!stream) return drc_fail(DRC_ERR_INVALID_ARG, "step_graph_create: the null stream cannot be captured");
    drc_step_graph* g = new drc_step_graph();
    g->h = h;
    g->params = d_params;
    g->m = d_m;
    g->v = d_v;
    g->adam = *adam;
    g->x = d_x;
    g->target = d_target;
    g->loss = d_loss;
    g->dparams = d_dparams;
    g->n = n;
    g->H = H;
    g->W = W;
    g->ws = d_ws;
    g->ws_bytes = ws_bytes;
    g->stream = (hipStream_t)stream;
    const drc_status st = step_graph_record(g);
    if (st != DRC_OK) {
        drc_cae_step_graph_destroy(g);
        return st;
    }
    *out = g;
    return DRC_OK;
}

extern "C" drc_status drc_cae_step_graph_launch(drc_step_graph* g, int64_t t) {
    if (!g) return drc_fail(DRC_ERR_INVALID_ARG, "step_graph_launch: graph is NULL");
    if (t < 1) return drc_fail(DRC_ERR_INVALID_ARG, "step_graph_launch: t = %lld (must be >= 1)", (long long)t);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != g->h->device)
        return drc_fail(DRC_ERR_STATE, "step_graph_launch: current device is not the handle's device");
    // a call that changed the handle since the recording (set_params from
    // another buffer, set_fused, ...) changes what the step enqueues
    if (g->h->gen != g->gen) TRY(step_graph_record(g));
    float step_size, inv_sqrt_bc2;
    adam_factors(&g->adam, t, &step_size, &inv_sqrt_bc2);
    g->adam_args.step_size = step_size;
    g->adam_args.inv_sqrt_bc2 = inv_sqrt_bc2;
    HIPCHK(hipGraphExecKernelNodeSetParams(g->exec, g->adam_node, &g->adam_params));
    HIPCHK(hipGraphLaunch(g->exec, g->stream));
    // the step leaves the handle packed from d_params, as drc_cae_step does
    g->h->params_set = true;
    g->h->packed_from = g->params;
    return DRC_OK;
}

extern "C" drc_status drc_cae_step_graph_captures(const drc_step_graph* g, int64_t* count) {
    if (!g || !count) return drc_fail(DRC_ERR_INVALID_ARG, "step_graph_captures: NULL argument");
    *count = g->captures;
    return DRC_OK;
}

extern "C" void drc_cae_step_graph_destroy(drc_step_graph* g) {
    if (!g) return;
    step_graph_release(g);
    delete g;
}

// ------------------------------------------------------------------ FP8 calibration
extern "C" drc_status drc_cae_calibrate_fp8(drc_cae* h, const float* d_x, int n, int H, int W, void* d_ws,
                                            size_t ws_bytes, void* stream) {
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "calibrate_fp8: handle is NULL");
    if (h->prec != P_FP8) return drc_fail(DRC_ERR_STATE, "calibrate_fp8: not an FP8 handle");
    if (!h->params_set) return drc_fail(DRC_ERR_STATE, "calibrate_fp8: call drc_cae_set_params first");
    TRY(check_shape("calibrate_fp8", n, H, W));
    TRY(check_ptr("calibrate_fp8", "d_x", d_x, 16, false));
    TRY(check_ptr("calibrate_fp8", "d_ws", d_ws, 256, false));
    size_t need = 0;
    TRY(drc_cae_workspace_size(h, n, H, W, DRC_WS_CALIBRATE, &need));
    if (ws_bytes < need)
        return drc_fail(DRC_ERR_WORKSPACE, "calibrate_fp8: workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    ActSizes a = act_sizes(P_F32, n, H, W);
    char* ws = (char*)d_ws;
    void* act[5];
    size_t cur = 0;
    for (int k = 0; k < 5; ++k) {
        act[k] = ws + cur;
        cur += a.bytes[k];
    }
    float* y = (float*)(ws + cur);
    FwdBufs b{d_x, y, act[0], act[1], act[2], act[3], act[4], nullptr, nullptr};
    TRY(forward_seq<P_F32>(h, h->wcal, b, n, H, W, 0, 5, s));
    HIPCHK(hipMemsetAsync(h->amax + 6, 0, 6 * sizeof(unsigned), s));
    const long cnt[6] = {a.p0 * 7, a.p1 * 32, a.p2 * 64, a.p3 * 128, a.p2 * 64, a.p1 * 32};
    const float* src[6] = {d_x, (const float*)act[0], (const float*)act[1], (const float*)act[2],
                           (const float*)act[3], (const float*)act[4]};
    for (int k = 0; k < 6; ++k)
        hipLaunchKernelGGL(amax_f32_kernel, dim3(256), dim3(256), 0, s, src[k], cnt[k], h->amax + 6 + k);
    TRY(check_launch("calibrate_fp8/amax"));
    unsigned am[6];
    HIPCHK(hipMemcpyAsync(am, h->amax + 6, sizeof am, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float v[6];
    for (int k = 0; k < 6; ++k) memcpy(&v[k], &am[k], 4);
    auto sc = [](float m) { return m > 0.0f ? 448.0f / m : 1.0f; };
    h->host_scales[6] = sc(v[0]);                 // x
    h->host_scales[7] = sc(std::max(v[1], v[5])); // [u2|h1]
    h->host_scales[8] = sc(std::max(v[2], v[4])); // [u3|h2]
    h->host_scales[9] = sc(v[3]);                 // h3
    HIPCHK(hipMemcpyAsync(h->scales + 6, h->host_scales + 6, 4 * sizeof(float), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    h->calibrated = true;
    h->gen++;
    return DRC_OK;
}
