// Host side of libdrc_cae: argument validation, the handle and its packed
// weights, workspace layout, and the launch sequences of the forward pass,
// the backward pass and the training step. All kernels live in the headers
// included below; nothing here computes on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "drc_cae.h"
#include "common.h"
#include "conv_layer.h"
#include "aux_kernels.h"
#include "internal.h"

using namespace drc;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

drc_status drc_fail(drc_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

extern "C" const char* drc_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* drc_status_string(drc_status s) {
    switch (s) {
        case DRC_OK: return "DRC_OK";
        case DRC_ERR_INVALID_ARG: return "DRC_ERR_INVALID_ARG";
        case DRC_ERR_SHAPE: return "DRC_ERR_SHAPE";
        case DRC_ERR_UNSUPPORTED: return "DRC_ERR_UNSUPPORTED";
        case DRC_ERR_WORKSPACE: return "DRC_ERR_WORKSPACE";
        case DRC_ERR_HIP: return "DRC_ERR_HIP";
        case DRC_ERR_STATE: return "DRC_ERR_STATE";
    }
    return "DRC_ERR_UNKNOWN";
}

// ------------------------------------------------------------------ network table
const LayerDef kLayers[6] = {
    {false, 7, 32}, {false, 32, 64}, {false, 64, 128},
    {true, 128, 64}, {true, 128, 32}, {true, 64, 3},
};

long layer_w_offset(int l) {
    long off = 0;
    for (int i = 0; i < l; ++i) off += (long)kLayers[i].cout * 9 * kLayers[i].cin + kLayers[i].cout;
    return off;
}
long layer_b_offset(int l) { return layer_w_offset(l) + (long)kLayers[l].cout * 9 * kLayers[l].cin; }
static const long kNumParams = 206819;

int prec_ks(int prec) { return prec == P_F32 ? 16 : (prec == P_BF16 ? 32 : 128); }
int prec_esize(int prec) { return prec == P_F32 ? 4 : (prec == P_BF16 ? 2 : 1); }
static int rup(int v, int m) { return (v + m - 1) / m * m; }
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Forward / backward-data GEMM geometry of layer l. Transposed
// convolutions run all four output phases in one GEMM: with per-pair weight
// blocks when the output has 16 or more channels, else with the phases
// merged into one block of rows.
GemmGeom gemm_geom(int l, bool backward, int prec) {
    const LayerDef& L = kLayers[l];
    GemmGeom g;
    bool tconv;
    if (!backward) {
        tconv = L.tconv;
        g.cin_eff = (l == 0) ? 8 : L.cin;
        g.rows = L.cout;
    } else {
        tconv = !L.tconv;
        g.cin_eff = (l == 5) ? (prec == P_F32 ? 4 : 8) : L.cout;
        g.rows = L.cin;
    }
    const int ks = prec_ks(prec);
    if (!tconv) {
        g.mode = M_CONV;
        g.rows_pad = rup(g.rows, 16);
        g.nblk = 1;
        g.kstride = rup(9 * g.cin_eff, ks);
    } else if (g.rows >= 16) {
        g.mode = M_TCONV_PAIRS;
        g.rows_pad = rup(g.rows, 16);
        g.nblk = 9;
        g.kstride = rup(g.cin_eff, ks);
    } else {
        g.mode = M_TCONV_MERGED;
        g.rows_pad = rup(4 * g.rows, 16);
        g.nblk = 1;
        g.kstride = rup(4 * g.cin_eff, ks);
    }
    g.nphase = g.nblk;
    return g;
}

// ------------------------------------------------------------------ create / destroy
extern "C" drc_cae_desc drc_cae_default_desc(int compute) {
    drc_cae_desc d;
    d.in_ch = 7;
    d.out_ch = 3;
    d.widths[0] = 32;
    d.widths[1] = 64;
    d.widths[2] = 128;
    d.compute = compute;
    d.final_relu = 0;
    d.pad_w = DRC_PAD_ZERO;
    return d;
}

extern "C" drc_status drc_cae_create(const drc_cae_desc* desc, drc_cae** out) {
    if (!out) return drc_fail(DRC_ERR_INVALID_ARG, "create: out is NULL");
    *out = nullptr;
    if (!desc) return drc_fail(DRC_ERR_INVALID_ARG, "create: desc is NULL");
    if (desc->in_ch != 7 || desc->out_ch != 3 || desc->widths[0] != 32 || desc->widths[1] != 64 ||
        desc->widths[2] != 128)
        return drc_fail(DRC_ERR_UNSUPPORTED, "create: only the 7->32->64->128->64->32->3 network is built");
    if (desc->compute < DRC_F32 || desc->compute > DRC_FP8_E4M3)
        return drc_fail(DRC_ERR_INVALID_ARG, "create: unknown compute dtype %d", desc->compute);
    if (desc->final_relu != 0 && desc->final_relu != 1)
        return drc_fail(DRC_ERR_INVALID_ARG, "create: final_relu must be 0 or 1");
    if (desc->pad_w != DRC_PAD_ZERO && desc->pad_w != DRC_PAD_CIRCULAR)
        return drc_fail(DRC_ERR_INVALID_ARG, "create: pad_w must be DRC_PAD_ZERO or DRC_PAD_CIRCULAR");
    drc_cae* h = new drc_cae();
    h->desc = *desc;
    h->fused = desc->pad_w == DRC_PAD_ZERO;  // the whole-network kernels pad with zeros
    h->prec = desc->compute;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return drc_fail(DRC_ERR_HIP, "create: hipGetDevice failed");
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) {
        h->arch = prop.gcnArchName;
        h->num_cu = prop.multiProcessorCount;
    }
    auto alloc = [&](void** p, size_t bytes) -> bool {
        return hipMalloc(p, align256(bytes)) == hipSuccess;
    };
    bool ok = true;
    for (int l = 0; l < 6 && ok; ++l) {
        GemmGeom gf = gemm_geom(l, false, h->prec);
        h->wf_bytes[l] = (size_t)gf.nblk * gf.rows_pad * gf.kstride * prec_esize(h->prec);
        ok = alloc(&h->wf[l], h->wf_bytes[l]);
        if (ok && h->prec != P_FP8) {
            GemmGeom gb = gemm_geom(l, true, h->prec);
            h->wb_bytes[l] = (size_t)gb.nblk * gb.rows_pad * gb.kstride * prec_esize(h->prec);
            ok = alloc(&h->wb[l], h->wb_bytes[l]);
        }
        if (ok && h->prec == P_BF16) ok = alloc(&h->wfrag[l], h->wf_bytes[l]);
        if (ok && h->prec == P_BF16) ok = alloc(&h->wbfrag[l], h->wb_bytes[l]);
        if (ok && h->prec == P_FP8) {  // float32 packs for the calibration forward
            GemmGeom gc = gemm_geom(l, false, P_F32);
            ok = alloc(&h->wcal[l], (size_t)gc.nblk * gc.rows_pad * gc.kstride * 4);
        }
    }
    for (int k = 0; k < drc_cae::kSide && ok; ++k)
        ok = hipStreamCreateWithFlags(&h->side[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&h->ev_join[k], hipEventDisableTiming) == hipSuccess;
    for (int l = 0; l < 6 && ok; ++l) ok = hipEventCreateWithFlags(&h->ev_fork[l], hipEventDisableTiming) == hipSuccess;
    ok = ok && alloc((void**)&h->bias, 512 * sizeof(float));
    ok = ok && alloc((void**)&h->scales, 16 * sizeof(float));
    ok = ok && alloc((void**)&h->amax, 16 * sizeof(unsigned));
    if (!ok) {
        drc_cae_destroy(h);
        return drc_fail(DRC_ERR_HIP, "create: device allocation failed");
    }
    for (int i = 0; i < 16; ++i) h->host_scales[i] = 1.0f;
    const drc_status st = static_scratch_setup(h->device);
    if (st != DRC_OK) {
        drc_cae_destroy(h);
        return st;
    }
    *out = h;
    return DRC_OK;
}

extern "C" void drc_cae_destroy(drc_cae* h) {
    if (!h) return;
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    for (int k = 0; k < drc_cae::kSide; ++k) {
        if (h->side[k]) (void)hipStreamDestroy(h->side[k]);
        if (h->ev_join[k]) (void)hipEventDestroy(h->ev_join[k]);
    }
    for (int l = 0; l < 6; ++l)
        if (h->ev_fork[l]) (void)hipEventDestroy(h->ev_fork[l]);
    for (int l = 0; l < 6; ++l) {
        if (h->wf[l]) (void)hipFree(h->wf[l]);
        if (h->wb[l]) (void)hipFree(h->wb[l]);
        if (h->wcal[l]) (void)hipFree(h->wcal[l]);
        if (h->wfrag[l]) (void)hipFree(h->wfrag[l]);
        if (h->wbfrag[l]) (void)hipFree(h->wbfrag[l]);
    }
    if (h->bias) (void)hipFree(h->bias);
    if (h->scales) (void)hipFree(h->scales);
    if (h->amax) (void)hipFree(h->amax);
    delete h;
}

extern "C" size_t drc_cae_num_params(const drc_cae* h) { return h ? (size_t)kNumParams : 0; }

extern "C" drc_status drc_cae_set_recompute(drc_cae* h, int on) {
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "set_recompute: handle is NULL");
    if (on != 0 && on != 1) return drc_fail(DRC_ERR_INVALID_ARG, "set_recompute: on must be 0 or 1");
    h->recompute = on;
    return DRC_OK;
}

extern "C" drc_status drc_cae_set_fused(drc_cae* h, int on) {
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "set_fused: handle is NULL");
    if (on != 0 && on != 1) return drc_fail(DRC_ERR_INVALID_ARG, "set_fused: on must be 0 or 1");
    if (on && h->desc.pad_w != DRC_PAD_ZERO)
        return drc_fail(DRC_ERR_UNSUPPORTED, "set_fused: the whole-network kernels use zero padding only");
    h->fused = on;
    h->gen++;
    return DRC_OK;
}

extern "C" drc_status drc_cae_set_tile(drc_cae* h, int layer, int H, int npw) {
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "set_tile: handle is NULL");
    if (layer < 0 || layer > 5) return drc_fail(DRC_ERR_INVALID_ARG, "set_tile: layer %d", layer);
    if (npw != 0 && !npw_supported(h->prec, layer, false, npw))
        return drc_fail(DRC_ERR_UNSUPPORTED, "set_tile: npw %d not built for layer %d", npw, layer);
    if (npw == 0) {
        h->tile.erase({layer, H});
        h->tile_px.erase({layer, H});
    } else {
        h->tile[{layer, H}] = npw;
    }
    h->gen++;
    return DRC_OK;
}

// ------------------------------------------------------------------ validation
static bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

drc_status check_shape(const char* who, int n, int H, int W) {
    if (n < 1) return drc_fail(DRC_ERR_SHAPE, "%s: n = %d (must be >= 1)", who, n);
    if (H < 8 || W < 8 || H % 8 || W % 8)
        return drc_fail(DRC_ERR_SHAPE, "%s: H = %d, W = %d (must be multiples of 8, >= 8)", who, H, W);
    if ((long)n * H * W > (1L << 31) / 8)
        return drc_fail(DRC_ERR_SHAPE, "%s: n*H*W = %ld too large", who, (long)n * H * W);
    return DRC_OK;
}

drc_status check_ptr(const char* who, const char* name, const void* p, size_t align, bool nullable) {
    if (!p) return nullable ? DRC_OK : drc_fail(DRC_ERR_INVALID_ARG, "%s: %s is NULL", who, name);
    if (!aligned(p, align))
        return drc_fail(DRC_ERR_INVALID_ARG, "%s: %s not %zu-byte aligned", who, name, align);
    return DRC_OK;
}

#define TRY(expr)                        \
    do {                                 \
        drc_status s_ = (expr);          \
        if (s_ != DRC_OK) return s_;     \
    } while (0)

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return drc_fail(DRC_ERR_HIP, "%s:%d %s: %s", __FILE__, __LINE__, #expr,           \
                            hipGetErrorString(e_));                                           \
    } while (0)

drc_status check_launch(const char* who) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return drc_fail(DRC_ERR_HIP, "%s: launch failed: %s", who, hipGetErrorString(e));
    return DRC_OK;
}

// ------------------------------------------------------------------ activations / workspace
ActSizes act_sizes(int prec, int n, int H, int W) {
    ActSizes a;
    const long p1 = (long)n * (H / 2) * (W / 2), p2 = (long)n * (H / 4) * (W / 4),
               p3 = (long)n * (H / 8) * (W / 8);
    const int es = prec_esize(prec);
    a.p0 = (long)n * H * W;
    a.p1 = p1;
    a.p2 = p2;
    a.p3 = p3;
    a.bytes[0] = align256(p1 * 32 * es);   // h1
    a.bytes[1] = align256(p2 * 64 * es);   // h2
    a.bytes[2] = align256(p3 * 128 * es);  // h3
    a.bytes[3] = align256(p2 * 64 * es);   // u3
    a.bytes[4] = align256(p1 * 32 * es);   // u2
    return a;
}

// Saved-buffer layout under a recompute policy: offsets of h1..u2 (-1 = not saved).
static size_t saved_layout(const ActSizes& a, int recompute, int64_t off[5]) {
    size_t cur = 0;
    for (int k = 0; k < 5; ++k) {
        if (recompute && k >= 2) {
            off[k] = -1;
            continue;
        }
        off[k] = (int64_t)cur;
        cur += a.bytes[k];
    }
    return cur;
}

extern "C" drc_status drc_cae_saved_size(const drc_cae* h, int n, int H, int W, size_t* bytes,
                                         int64_t offsets[5]) {
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "saved_size: handle is NULL");
    if (!bytes) return drc_fail(DRC_ERR_INVALID_ARG, "saved_size: bytes is NULL");
    TRY(check_shape("saved_size", n, H, W));
    int64_t off[5];
    *bytes = saved_layout(act_sizes(h->prec, n, H, W), h->recompute, off);
    if (offsets)
        for (int k = 0; k < 5; ++k) offsets[k] = off[k];
    return DRC_OK;
}

// Weight-gradient work split for layer l (see wgrad_kernel): MFMA tile
// blocks, reduction pixels per workgroup and number of reduction chunks.
// Weight-gradient workgroups in one wave of the chip (one per CU).
constexpr int kWgradWave = 256;

WgradPlan wgrad_plan(int l, int n, int H, int W, int prec) {
    const LayerDef& L = kLayers[l];
    int hin, win, hout, wout;
    layer_io(l, H, W, &hin, &win, &hout, &wout);
    WgradPlan w;
    w.qc = L.tconv ? L.cout : L.cin;  // gathered operand channels
    w.pc = L.tconv ? L.cin : L.cout;  // plain operand channels
    w.Hr = L.tconv ? hin : hout;
    w.Wr = L.tconv ? win : wout;
    const int jblocks = (9 * w.qc + 15) / 16, pblocks = (w.pc + 15) / 16;
    w.JB = jblocks >= 4 ? 4 : 2;
    w.PB = (w.JB == 4 && pblocks <= 2) ? 2 : 4;
    w.VEC = (w.JB == 4 && w.PB == 4 && w.qc % 4 == 0 && w.pc % 4 == 0) ? 4 : 1;
    w.jtiles = (jblocks + w.JB - 1) / w.JB;
    w.ptiles = (pblocks + w.PB - 1) / w.PB;
    const long K = (long)n * w.Hr * w.Wr;
    // about 2048 workgroups, at most 256 chunks and 64 MB of partial tiles
    const long per_chunk_floats = 4L * 9 * w.qc * w.pc;
    long want = std::max(1L, std::min(256L, 2048L / (w.jtiles * w.ptiles)));
    want = std::max(1L, std::min(want, (16L << 20) / per_chunk_floats));
    long pb = (K + want - 1) / want;
    pb = std::max(64L, (pb + 15) / 16 * 16);
    w.per_block = pb;
    w.nchunks = (int)((K + pb - 1) / pb);
    w.partial_floats = (size_t)w.nchunks * per_chunk_floats;  // 4 wave slots per chunk

    // BF16: LDS-staged operands on bf16 MFMA when a row holds whole groups of 8 pixels
    w.bf16 = 0;
    w.tr = 0;
    if (prec == P_BF16 && w.Wr % 8 == 0) {
        w.QCP = (w.qc + 7) / 8 * 8;
        const int jb = (9 * w.qc + 15) / 16;
        w.JBW = (jb + 3) / 4;
        w.BPB = (w.pc >= 64) ? 4 : 2;
        w.bptiles = (w.pc + 16 * w.BPB - 1) / (16 * w.BPB);
        const bool inst = (w.JBW == 1 && (w.BPB == 2 || w.BPB == 4) && w.QCP == 8) ||
                          (w.JBW == 5 && w.BPB == 4 && w.QCP == 32) || (w.JBW == 9 && w.BPB == 4 && w.QCP == 64);
        // Transpose-read kernel: both operands staged as plain NHWC tiles. A
        // 16-bit gathered operand with 32 or 64 channels, or the float32 one
        // of E1 (x, 7 channels, staged as 8) and D1 (dy, 3 channels, as 4).
        w.tr = 0;
        w.QR = 0;
        const bool raw = l == 0 || l == 5;
        // D2 (32 gathered x 128 plain channels): 8 waves cover all plain
        // channels in one tile, so the gathered operand is staged once (with
        // 64 gathered channels the 8-wave tile would not fit the registers)
        int tqc = 0, tnw = 4, tjbw = 0, tpb = 0, ttg = 0, ttp = 0;
        if (!raw && (w.qc == 32 || w.qc == 64) && inst) {
            tqc = w.qc;
            if (w.qc == 32 && w.pc == 128) {
                tnw = 8; tpb = 8; tjbw = 3; ttg = kWgradTG8; ttp = kWgradTP8;
            } else {
                tjbw = w.JBW; tpb = w.BPB; ttg = kWgradTG; ttp = kWgradTP;
            }
        } else if (raw && w.qc == (l == 0 ? 7 : 3)) {
            tqc = l == 0 ? 8 : 4;
            tjbw = ((9 * tqc + 15) / 16 + 3) / 4;
            tpb = w.pc >= 64 ? 4 : 2;
            ttg = l == 0 ? kWgradTGRaw7 : kWgradTGRaw3; ttp = kWgradTP;
        }
        for (int R = w.Hr; R >= 1 && tqc; R /= 2) {
            if ((R * w.Wr) % 32) continue;
            const int GS = tqc + 8, PS = tpb * 16 + 8;
            const int lds = ((2 * R + 1) * 2 * w.Wr * GS + R * w.Wr * PS + 16) * 2;
            if (lds > (tnw == 8 ? 96 : 64) * 1024) continue;
            // staging tasks: 16-byte chunks of the gathered rows (float32: dense rows)
            const int gtasks = raw ? (2 * R + 1) * 2 * w.Wr * w.qc / 4 : (2 * R + 1) * 2 * w.Wr * (tqc / 8);
            if (gtasks > 64 * tnw * ttg) continue;  // staging tasks per thread
            if (R * w.Wr * 2 * tpb > 64 * tnw * ttp) continue;
            w.bf16 = 1;
            w.tr = 1;
            w.QR = raw ? w.qc : 0;
            w.QCP = tqc;
            w.NW = tnw;
            w.JBW = tjbw;
            w.BPB = tpb;
            w.bptiles = (w.pc + 16 * w.BPB - 1) / (16 * w.BPB);
            w.R = R;
            w.lds = lds;
            break;
        }
        for (int R = std::max(1, 128 / w.Wr); R >= 1 && inst && !w.tr; R /= 2) {
            if ((R * w.Wr) % 32) continue;
            int qcs = (2 * R + 1) * 3 * w.Wr;
            qcs = (qcs + 7) / 8 * 8;
            if ((qcs / 8) % 2 == 0) qcs += 8;
            const int lds = w.QCP * qcs * 2 + 16 * w.BPB * (R * w.Wr + 8) * 2;
            if (lds > 64 * 1024) continue;
            w.bf16 = 1;
            w.R = R;
            w.qcs = qcs;
            w.lds = lds;
            break;
        }
        if (w.bf16) {
            w.strips_per_map = (w.Hr + w.R - 1) / w.R;
            w.total_strips = n * w.strips_per_map;
            const long per_chunk = 9L * w.qc * w.pc;
            // about 4 strips per workgroup (the next strip's loads overlap the
            // current MFMAs, and fewer partial tiles are written), between 256
            // and 1024 workgroups in all
            const long lo = std::max(1L, 256L / w.bptiles), hi = std::max(1L, 1024L / w.bptiles);
            long chunks = std::min(hi, std::max(lo, (long)w.total_strips / 4));
            chunks = std::min(chunks, std::max(1L, (16L << 20) / per_chunk));
            // whole waves of 256 workgroups: the large tiles run one workgroup
            // per CU, and a partial last wave would leave CUs idle
            if (chunks * w.bptiles > kWgradWave)
                chunks = std::max(lo, chunks * w.bptiles / kWgradWave * kWgradWave / w.bptiles);
            chunks = std::min<long>(chunks, w.total_strips);
            w.strips_per_chunk = (int)((w.total_strips + chunks - 1) / chunks);
            w.bchunks = (w.total_strips + w.strips_per_chunk - 1) / w.strips_per_chunk;
            w.partial_floats = std::max(w.partial_floats, (size_t)w.bchunks * per_chunk);
        }
    }
    return w;
}

extern "C" drc_status drc_cae_wgrad_schedule(int compute, int layer, int n, int H, int W, int64_t info[4]) {
    if (!info) return drc_fail(DRC_ERR_INVALID_ARG, "wgrad_schedule: info is NULL");
    if (compute != DRC_F32 && compute != DRC_BF16)
        return drc_fail(compute == DRC_FP8_E4M3 ? DRC_ERR_UNSUPPORTED : DRC_ERR_INVALID_ARG,
                        "wgrad_schedule: compute %d (float32 and bfloat16 handles have a backward)", compute);
    if (layer < 0 || layer > 5) return drc_fail(DRC_ERR_INVALID_ARG, "wgrad_schedule: layer %d", layer);
    TRY(check_shape("wgrad_schedule", n, H, W));
    const WgradPlan w = wgrad_plan(layer, n, H, W, compute);
    if (w.bf16) {
        info[0] = w.tr ? 2 : 1;
        info[1] = w.R;
        info[2] = w.strips_per_chunk;
        info[3] = w.bchunks;
    } else {
        info[0] = 0;
        info[1] = 0;
        info[2] = w.per_block;
        info[3] = w.nchunks;
    }
    return DRC_OK;
}

void layer_io(int l, int H, int W, int* hin, int* win, int* hout, int* wout) {
    static const int din[6] = {1, 2, 4, 8, 4, 2};   // input = H / din
    static const int dout[6] = {2, 4, 8, 4, 2, 1};  // output = H / dout
    *hin = H / din[l];
    *win = W / din[l];
    *hout = H / dout[l];
    *wout = W / dout[l];
}



// Column-sum (bias gradient) grid: a multiple of 3 blocks, so that the
// element stride 256 * VW * blocks is a multiple of every channel count
// (3, 32, 64, 128) with VW = 4 (float) or 8 (bf16).
void colsum_split(long npix, int* nblocks, long* per_block) {
    (void)npix;
    *nblocks = 384;
    *per_block = 0;
}

// Backward workspace: [recompute h3 u3 u2] [gradients] [wgrad partials] [bias partials]
BwdLayout bwd_layout(int prec, int n, int H, int W, bool recompute_needed) {
    BwdLayout b;
    ActSizes a = act_sizes(prec, n, H, W);
    const int es = prec_esize(prec);
    size_t cur = 0;
    for (int k = 0; k < 3; ++k) b.recomp[k] = 0;
    if (recompute_needed) {
        b.recomp[0] = cur; cur += a.bytes[2];  // h3
        b.recomp[1] = cur; cur += a.bytes[3];  // u3
        b.recomp[2] = cur; cur += a.bytes[4];  // u2
    }
    b.dz_u2 = cur; cur += align256(a.p1 * 32 * es);
    b.dh1s = cur; cur += align256(a.p1 * 32 * es);
    b.dz_u3 = cur; cur += align256(a.p2 * 64 * es);
    b.dh2s = cur; cur += align256(a.p2 * 64 * es);
    b.dz_h3 = cur; cur += align256(a.p3 * 128 * es);
    b.dz_h2 = cur; cur += align256(a.p2 * 64 * es);
    b.dz_h1 = cur; cur += align256(a.p1 * 32 * es);
    size_t bp = 0;
    for (int l = 0; l < 6; ++l) {
        b.wpart[l] = cur;
        cur += align256(wgrad_plan(l, n, H, W, prec).partial_floats * sizeof(float));
        int hin, win, hout, wout;
        layer_io(l, H, W, &hin, &win, &hout, &wout);
        int nb;
        long per;
        colsum_split((long)n * hout * wout, &nb, &per);
        bp = std::max(bp, (size_t)nb * 128 * sizeof(float));
    }
    // the whole-network data-gradient kernel keeps 323 bias partials per workgroup
    bp = std::max(bp, (size_t)std::min(n, 2048) * 323 * sizeof(float));
    b.bpart = cur; cur += align256(bp);
    b.bpart_bytes = bp;
    b.total = cur;
    return b;
}

// Step workspace: [saved] [fwd scratch acts] [y] [dy] [loss partials] [dparams] [bwd]
StepLayout step_layout(int prec, int n, int H, int W, int recompute) {
    StepLayout s;
    ActSizes a = act_sizes(prec, n, H, W);
    int64_t off[5];
    size_t cur = 0;
    s.saved = cur;
    cur += saved_layout(a, recompute, off);
    s.fwd_scratch = cur;
    if (recompute) cur += a.bytes[2] + a.bytes[3] + a.bytes[4];
    s.y = cur; cur += align256(a.p0 * 3 * sizeof(float));
    s.dy = cur; cur += align256(a.p0 * 3 * sizeof(float));
    s.loss_part = cur;
    cur += align256(((a.p0 * 3 + kLossPerBlock - 1) / kLossPerBlock) * sizeof(double));
    s.dparams = cur; cur += align256(kNumParams * sizeof(float));
    s.bwd = cur;
    cur += bwd_layout(prec, n, H, W, recompute != 0).total;
    s.total = cur;
    return s;
}

extern "C" drc_status drc_cae_workspace_size(const drc_cae* h, int n, int H, int W, int flags,
                                             size_t* bytes) {
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "workspace_size: handle is NULL");
    if (!bytes) return drc_fail(DRC_ERR_INVALID_ARG, "workspace_size: bytes is NULL");
    if (flags & ~(DRC_WS_FORWARD | DRC_WS_BACKWARD | DRC_WS_STEP | DRC_WS_CALIBRATE | DRC_WS_AUTOTUNE) || !flags)
        return drc_fail(DRC_ERR_INVALID_ARG, "workspace_size: bad flags 0x%x", flags);
    TRY(check_shape("workspace_size", n, H, W));
    size_t need = 0;
    ActSizes a = act_sizes(h->prec, n, H, W);
    if (flags & DRC_WS_FORWARD) {
        size_t f = 0;
        for (int k = 0; k < 5; ++k) f += a.bytes[k];
        need = std::max(need, f);
    }
    if (flags & DRC_WS_BACKWARD) need = std::max(need, bwd_layout(h->prec, n, H, W, true).total);
    if (flags & DRC_WS_STEP) need = std::max(need, step_layout(h->prec, n, H, W, h->recompute).total);
    if (flags & DRC_WS_AUTOTUNE) {
        size_t f = align256((size_t)a.p0 * 3 * sizeof(float));
        for (int k = 0; k < 5; ++k) f += a.bytes[k];
        need = std::max(need, f);
    }
    if (flags & DRC_WS_CALIBRATE) {
        ActSizes c = act_sizes(P_F32, n, H, W);
        size_t f = align256((size_t)c.p0 * 3 * sizeof(float));
        for (int k = 0; k < 5; ++k) f += c.bytes[k];
        need = std::max(need, f);
    }
    *bytes = need;
    return DRC_OK;
}

// ------------------------------------------------------------------ parameter packing
static drc_status pack_all(drc_cae* h, const float* d_params, hipStream_t s) {
    if (h->prec == P_FP8) {
        HIPCHK(hipMemsetAsync(h->amax, 0, 16 * sizeof(unsigned), s));
        for (int l = 0; l < 6; ++l) {
            const long cnt = (long)kLayers[l].cout * 9 * kLayers[l].cin;
            hipLaunchKernelGGL(amax_f32_kernel, dim3(64), dim3(256), 0, s, d_params + layer_w_offset(l), cnt,
                               h->amax + l);
        }
        hipLaunchKernelGGL(fp8_scale_kernel, dim3(1), dim3(64), 0, s, (const unsigned*)h->amax, h->scales, 6);
        TRY(check_launch("set_params/fp8 scales"));
    }
    // every weight pack (and its fragment-ordered copy) and the biases in one launch
    PackAllArgs pa;
    memset(&pa, 0, sizeof pa);
    long most = 0;
    for (int l = 0; l < 6; ++l) {
        for (int dir = 0; dir < 3; ++dir) {
            void* dst = dir == 0 ? h->wf[l] : (dir == 1 ? h->wb[l] : h->wcal[l]);
            if (!dst) continue;
            const int prec = dir == 2 ? P_F32 : h->prec;
            GemmGeom g = gemm_geom(l, dir == 1, prec);
            PackArgs& a = pa.p[pa.np++];
            a.w = d_params + layer_w_offset(l);
            a.cout = kLayers[l].cout;
            a.cin = kLayers[l].cin;
            a.gemm_mode = g.mode;
            a.transpose = dir == 1;
            a.cin_eff = g.cin_eff;
            a.rows_pad = g.rows_pad;
            a.kstride = g.kstride;
            a.nblk = g.nblk;
            a.prec = prec;
            a.scale = prec == P_FP8 ? h->scales + l : nullptr;
            a.dst = dst;
            a.frag = (prec == P_BF16 && dir < 2 && g.kstride % 32 == 0) ? (dir ? h->wbfrag[l] : h->wfrag[l])
                                                                         : nullptr;
            most = std::max(most, (long)g.nblk * g.rows_pad * g.kstride);
        }
        pa.bsrc[l] = d_params + layer_b_offset(l);
        pa.bcount[l] = kLayers[l].cout;
        pa.bslot[l] = bias_slot(l);
    }
    pa.bdst = h->bias;
    const int bx = (int)std::min(256L, (most + 255) / 256);
    hipLaunchKernelGGL(pack_all_kernel, dim3(bx, pa.np + 1), dim3(256), 0, s, pa);
    TRY(check_launch("set_params/pack"));
    return DRC_OK;
}

extern "C" drc_status drc_cae_set_params(drc_cae* h, const float* d_params, void* stream) {
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "set_params: handle is NULL");
    TRY(check_ptr("set_params", "d_params", d_params, 4, false));
    hipStream_t s = (hipStream_t)stream;
    TRY(pack_all(h, d_params, s));
    if (h->prec == P_FP8) {
        HIPCHK(hipMemcpyAsync(h->host_scales, h->scales, 6 * sizeof(float), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    h->params_set = true;
    h->packed_from = d_params;
    h->gen++;
    return DRC_OK;
}

extern "C" drc_status drc_cae_get_fp8_scales(const drc_cae* h, float out[10], void* stream) {
    if (!h || !out) return drc_fail(DRC_ERR_INVALID_ARG, "get_fp8_scales: NULL argument");
    if (h->prec != P_FP8) return drc_fail(DRC_ERR_STATE, "get_fp8_scales: not an FP8 handle");
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    for (int i = 0; i < 10; ++i) out[i] = h->host_scales[i];
    return DRC_OK;
}

// ------------------------------------------------------------------ profiling hook
long prof_begin(drc_cae* h, int slot, hipStream_t s) {
    if (!h->prof || h->ev_next + 2 > h->ev_pool.size()) return -1;
    const size_t k = h->ev_next;
    h->ev_next += 2;
    if (hipEventRecord(h->ev_pool[k], s) != hipSuccess) return -1;
    h->prof_rec.push_back({slot, k});
    return (long)k;
}

void prof_end(drc_cae* h, long token, hipStream_t s) {
    if (token < 0) return;
    (void)hipEventRecord(h->ev_pool[(size_t)token + 1], s);
}

extern "C" drc_status drc_cae_profile(drc_cae* h, int enable) {
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "profile: handle is NULL");
    if (enable && h->ev_pool.empty()) {
        h->ev_pool.resize(16384);
        for (auto& e : h->ev_pool)
            if (hipEventCreate(&e) != hipSuccess) return drc_fail(DRC_ERR_HIP, "profile: hipEventCreate failed");
    }
    h->prof = enable != 0;
    return DRC_OK;
}

extern "C" drc_status drc_cae_profile_read(drc_cae* h, double ms[24], int64_t calls[24]) {
    if (!h || !ms || !calls) return drc_fail(DRC_ERR_INVALID_ARG, "profile_read: NULL argument");
    for (int i = 0; i < PROF_SLOTS; ++i) {
        ms[i] = 0.0;
        calls[i] = 0;
    }
    for (auto& r : h->prof_rec) {
        if (hipEventSynchronize(h->ev_pool[r.second + 1]) != hipSuccess)
            return drc_fail(DRC_ERR_HIP, "profile_read: event wait failed");
        float t = 0.0f;
        if (hipEventElapsedTime(&t, h->ev_pool[r.second], h->ev_pool[r.second + 1]) != hipSuccess)
            return drc_fail(DRC_ERR_HIP, "profile_read: elapsed time failed");
        ms[r.first] += t;
        calls[r.first] += 1;
    }
    h->prof_rec.clear();
    h->ev_next = 0;
    return DRC_OK;
}
