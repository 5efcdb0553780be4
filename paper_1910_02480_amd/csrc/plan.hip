// Mixed-resolution frames and tile tuning.
//
// A frame holds cache points whose hemispherical maps have different sizes
// (larger maps blur less, Sec. 6.3; the paper fixes 32x32 and names that a
// limitation, Sec. 7). The network is fully convolutional, so one set of
// weights serves every size. A plan groups the maps into resolution classes
// and runs each layer as ONE persistent launch whose work items span all
// classes; the six launches are captured once into a HIP graph and replayed
// per frame.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "drc_cae.h"
#include "common.h"
#include "conv_layer.h"
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

// ------------------------------------------------------------------ tuning cache
// One entry per line:
// {"arch": "gfx950", "prec": 1, "layer": 0, "H": 64, "W": 64, "npw": 4, "tile_px": 512, "us": 12.5}
struct TuneEntry {
    int npw = 0, tile_px = 0;
    double us = 0;
};
typedef std::map<std::string, TuneEntry> TuneTable;

static std::string arch_base(const std::string& a) { return a.substr(0, a.find(':')); }

static std::string tune_key(const std::string& arch, int prec, int layer, int H, int W) {
    char buf[128];
    snprintf(buf, sizeof buf, "%s/%d/%d/%dx%d", arch_base(arch).c_str(), prec, layer, H, W);
    return buf;
}

static void load_tune(const char* path, TuneTable& t) {
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        char arch[64] = {0};
        int prec, layer, H, W, npw, tile;
        double us = 0;
        if (sscanf(line, " {\"arch\": \"%63[^\"]\", \"prec\": %d, \"layer\": %d, \"H\": %d, \"W\": %d, \"npw\": %d, "
                         "\"tile_px\": %d, \"us\": %lf",
                   arch, &prec, &layer, &H, &W, &npw, &tile, &us) >= 7) {
            TuneEntry e;
            e.npw = npw;
            e.tile_px = tile;
            e.us = us;
            t[tune_key(arch, prec, layer, H, W)] = e;
        }
    }
    fclose(f);
}

static drc_status save_tune(const char* path, const TuneTable& t) {
    FILE* f = fopen(path, "w");
    if (!f) return drc_fail(DRC_ERR_INVALID_ARG, "autotune: cannot write %s", path);
    for (auto& kv : t) {
        char arch[64];
        int prec, layer, H, W;
        if (sscanf(kv.first.c_str(), "%63[^/]/%d/%d/%dx%d", arch, &prec, &layer, &H, &W) != 5) continue;
        fprintf(f,
                "{\"arch\": \"%s\", \"prec\": %d, \"layer\": %d, \"H\": %d, \"W\": %d, \"npw\": %d, "
                "\"tile_px\": %d, \"us\": %.3f}\n",
                arch, prec, layer, H, W, kv.second.npw, kv.second.tile_px, kv.second.us);
    }
    fclose(f);
    return DRC_OK;
}

// ------------------------------------------------------------------ plans
struct PlanClass {
    int H, W, n;
    long flops;              // forward work of the class (for picking shared tile shapes)
    std::vector<long> xoff;  // element offsets of each map's input / output
    std::vector<long> yoff;
    bool x_al16 = true;                 // every xoff is a multiple of 4 floats
    size_t dev_xoff = 0, dev_yoff = 0;  // byte offsets into the plan's device table
    size_t act[5];           // byte offsets of h1..u2 inside the workspace
    int npw[6], tile_px[6];
};

struct drc_plan {
    drc_cae* h = nullptr;
    int count = 0;
    std::vector<PlanClass> cls;
    char* d_tables = nullptr;
    size_t ws_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // ws, stream, x, y and the handle's generation of the captured graph
    const void* key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    long captures = 0;  // graphs recorded so far
};

extern "C" drc_status drc_cae_plan_create(drc_cae* h, const drc_map_desc* maps, int count,
                                          const char* tune_cache, drc_plan** out) {
    if (!out) return drc_fail(DRC_ERR_INVALID_ARG, "plan_create: out is NULL");
    *out = nullptr;
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "plan_create: handle is NULL");
    if (!maps || count < 1) return drc_fail(DRC_ERR_SHAPE, "plan_create: empty plan (count = %d)", count);
    std::map<std::pair<int, int>, int> idx;
    std::vector<PlanClass> cls;
    for (int m = 0; m < count; ++m) {
        const drc_map_desc& d = maps[m];
        if (d.h < 8 || d.w < 8 || d.h % 8 || d.w % 8)
            return drc_fail(DRC_ERR_SHAPE, "plan_create: map %d is %dx%d (multiples of 8 required)", m, d.h, d.w);
        if (d.x_off < 0 || d.y_off < 0)
            return drc_fail(DRC_ERR_INVALID_ARG, "plan_create: map %d has a bad offset", m);
        auto key = std::make_pair(d.h, d.w);
        if (!idx.count(key)) {
            if ((int)cls.size() == kMaxClasses)
                return drc_fail(DRC_ERR_UNSUPPORTED, "plan_create: more than %d map sizes", kMaxClasses);
            idx[key] = (int)cls.size();
            PlanClass c;
            c.H = d.h;
            c.W = d.w;
            c.n = 0;
            cls.push_back(c);
        }
        PlanClass& c = cls[idx[key]];
        c.n++;
        c.xoff.push_back((long)d.x_off);
        c.x_al16 = c.x_al16 && d.x_off % 4 == 0;
        c.yoff.push_back((long)d.y_off);
    }
    std::sort(cls.begin(), cls.end(), [](const PlanClass& a, const PlanClass& b) {
        return (long)a.H * a.W < (long)b.H * b.W;
    });
    TuneTable tune;
    load_tune(tune_cache, tune);
    size_t ws = 0, tab = 0;
    for (auto& c : cls) {
        c.flops = (long)c.n * c.H * c.W;
        ActSizes a = act_sizes(h->prec, c.n, c.H, c.W);
        for (int k = 0; k < 5; ++k) {
            c.act[k] = ws;
            ws += a.bytes[k];
        }
        c.dev_xoff = tab;
        tab += align256(c.xoff.size() * sizeof(long));
        c.dev_yoff = tab;
        tab += align256(c.yoff.size() * sizeof(long));
        for (int l = 0; l < 6; ++l) {
            auto it = tune.find(tune_key(h->arch, h->prec, l, c.H, c.W));
            c.npw[l] = (it != tune.end() && npw_supported(h->prec, l, false, it->second.npw)) ? it->second.npw : 0;
            c.tile_px[l] = (it != tune.end()) ? std::max(0, it->second.tile_px) : 0;
        }
    }
    drc_plan* p = new drc_plan();
    p->h = h;
    p->count = count;
    p->ws_bytes = std::max<size_t>(ws, 256);
    if (hipMalloc((void**)&p->d_tables, std::max<size_t>(tab, 256)) != hipSuccess) {
        delete p;
        return drc_fail(DRC_ERR_HIP, "plan_create: device allocation failed");
    }
    for (auto& c : cls) {
        if (hipMemcpy(p->d_tables + c.dev_xoff, c.xoff.data(), c.xoff.size() * sizeof(long),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p->d_tables + c.dev_yoff, c.yoff.data(), c.yoff.size() * sizeof(long),
                      hipMemcpyHostToDevice) != hipSuccess) {
            drc_cae_plan_destroy(p);
            return drc_fail(DRC_ERR_HIP, "plan_create: upload failed");
        }
    }
    p->cls = std::move(cls);
    *out = p;
    return DRC_OK;
}

extern "C" drc_status drc_cae_plan_workspace_size(const drc_plan* p, size_t* bytes) {
    if (!p || !bytes) return drc_fail(DRC_ERR_INVALID_ARG, "plan_workspace_size: NULL argument");
    *bytes = p->ws_bytes;
    return DRC_OK;
}

extern "C" drc_status drc_cae_plan_captures(const drc_plan* p, int64_t* count) {
    if (!p || !count) return drc_fail(DRC_ERR_INVALID_ARG, "plan_captures: NULL argument");
    *count = p->captures;
    return DRC_OK;
}

extern "C" void drc_cae_plan_destroy(drc_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_tables) (void)hipFree(p->d_tables);
    delete p;
}

// Enqueue a frame. BF16 and FP8 classes the whole-network kernel is built
// for run through it, one launch per class; BF16 128x128 classes (zero
// padding, 16-byte aligned maps) run E1-D2 in the banded kernel; the rest
// share one persistent launch per layer, and D1 of every class that is not
// whole-network is one launch.
static drc_status plan_enqueue(drc_plan* p, const float* x, float* y, char* ws, hipStream_t s) {
    drc_cae* h = p->h;
    const bool prof = h->prof;
    h->prof = false;
    const bool x16 = (uintptr_t)x % 16 == 0;
    // (its input staging reads 16-byte vectors: every map must start on a 16-byte boundary)
    auto whole_network = [&](const PlanClass& pc) {
        return h->fused && (h->prec == P_FP8 || h->prec == P_BF16) && fused_forward_size(pc.H, pc.W) &&
               pc.x_al16 && x16;
    };
    std::vector<FwdClass> fc;
    std::vector<int> from;
    for (size_t c = 0; c < p->cls.size(); ++c) {
        const PlanClass& pc = p->cls[c];
        if (whole_network(pc)) continue;
        FwdClass f;
        memset(&f, 0, sizeof f);
        f.b.x = x;
        f.b.y = y;
        f.b.h1 = ws + pc.act[0];
        f.b.h2 = ws + pc.act[1];
        f.b.h3 = ws + pc.act[2];
        f.b.u3 = ws + pc.act[3];
        f.b.u2 = ws + pc.act[4];
        f.b.x_off = (const long*)(p->d_tables + pc.dev_xoff);
        f.b.y_off = (const long*)(p->d_tables + pc.dev_yoff);
        f.n = pc.n;
        f.H = pc.H;
        f.W = pc.W;
        f.x_al16 = pc.x_al16 && x16;
        for (int l = 0; l < 6; ++l) f.tile_px[l] = pc.tile_px[l];
        fc.push_back(f);
        from.push_back((int)c);
    }
    const int nc = (int)fc.size();
    if (nc) {
        // The GEMM tile (NPW) is shared by the classes of a launch: take the
        // tuned choice of the class with the most work.
        long best = -1;
        int big = 0;
        for (size_t k = 0; k < from.size(); ++k)
            if (p->cls[from[k]].flops > best) {
                best = p->cls[from[k]].flops;
                big = from[k];
            }
        for (int l = 0; l < 6; ++l) fc[0].npw[l] = p->cls[big].npw[l];
    }
    std::vector<FwdClass> rest;
    std::vector<int> tail;
    for (int k = 0; k < nc; ++k) {
        if (h->fused && h->prec == P_BF16 && fused_tail_size(fc[k].H, fc[k].W) && h->desc.pad_w == DRC_PAD_ZERO &&
            fc[k].x_al16)
            tail.push_back(k);
        else
            rest.push_back(fc[k]);
    }
    if (!rest.empty() && !tail.empty())
        for (int l = 0; l < 6; ++l) rest[0].npw[l] = fc[0].npw[l];
    // When every class outside the banded kernel is whole-network, the
    // banded chain (one workgroup per map, so freed CUs take its maps as they
    // come) runs on a side stream, enqueued first, next to the whole-network
    // launches: each launch's last, partly filled wave of workgroups then
    // overlaps the other stream's work instead of leaving CUs idle.
    const bool fork = !tail.empty() && rest.empty();
    hipStream_t sb = fork ? h->side[0] : s;
    drc_status st = DRC_OK;
    if (fork) {
        if (hipEventRecord(h->ev_fork[0], s) != hipSuccess || hipStreamWaitEvent(sb, h->ev_fork[0], 0) != hipSuccess) {
            h->prof = prof;
            return drc_fail(DRC_ERR_HIP, "plan: side stream fork failed");
        }
    }
    auto banded_chain = [&]() -> drc_status {
        for (size_t k = 0; k < tail.size(); ++k) {
            const FwdClass& f = fc[tail[k]];
            TRY(fused_tail(h, f.n, f.H, f.W, f.b.x, f.b.x_off, f.b.h1, f.b.h2, f.b.u2, sb));
        }
        // beside the whole-network launches D1 starts on the CUs they free:
        // eight workgroups per CU (band lists a quarter as long) for 0.905 vs
        // 0.921 ms per frame
        return forward_classes<P_BF16>(h, h->wf, fc.data(), nc, 5, 5, sb, fork ? 8 : 2);
    };
    if (fork) st = banded_chain();
    for (size_t c = 0; c < p->cls.size() && st == DRC_OK; ++c) {
        const PlanClass& pc = p->cls[c];
        if (!whole_network(pc)) continue;
        const long* xo = (const long*)(p->d_tables + pc.dev_xoff);
        const long* yo = (const long*)(p->d_tables + pc.dev_yoff);
        if (h->prec == P_FP8)
            st = fused_fp8_forward(h, x, y, pc.n, pc.H, pc.W, xo, yo, s);
        else  // the class's h1 region (n maps) holds the per-workgroup slots
            st = fused_forward(h, x, y, pc.n, pc.H, pc.W, xo, yo, ws + pc.act[0],
                               (size_t)pc.n * 16 * pc.H * pc.W, s);
    }
    if (st == DRC_OK && nc && !fork) {
        if (tail.empty()) {
            if (h->prec == P_F32) st = forward_classes<P_F32>(h, h->wf, fc.data(), nc, 0, 5, s);
            if (h->prec == P_BF16) st = forward_classes<P_BF16>(h, h->wf, fc.data(), nc, 0, 5, s);
            if (h->prec == P_FP8) st = forward_classes<P_FP8>(h, h->wf, fc.data(), nc, 0, 5, s);
        } else {
            st = forward_classes<P_BF16>(h, h->wf, rest.data(), (int)rest.size(), 0, 4, s);
            if (st == DRC_OK) st = banded_chain();
        }
    }
    // join the side stream whatever happened (a capture needs every fork joined)
    if (fork && (hipEventRecord(h->ev_join[0], sb) != hipSuccess || hipStreamWaitEvent(s, h->ev_join[0], 0) != hipSuccess) &&
        st == DRC_OK)
        st = drc_fail(DRC_ERR_HIP, "plan: side stream join failed");
    h->prof = prof;
    return st;
}

extern "C" drc_status drc_cae_plan_launch(drc_plan* p, const float* d_x, float* d_y, void* d_ws, size_t ws_bytes,
                                          void* stream) {
    if (!p) return drc_fail(DRC_ERR_INVALID_ARG, "plan_launch: plan is NULL");
    drc_cae* h = p->h;
    if (!h->params_set) return drc_fail(DRC_ERR_STATE, "plan_launch: call drc_cae_set_params first");
    if (h->prec == P_FP8 && !h->calibrated)
        return drc_fail(DRC_ERR_STATE, "plan_launch: FP8 handle needs drc_cae_calibrate_fp8 first");
    TRY(check_ptr("plan_launch", "d_x", d_x, 16, false));
    TRY(check_ptr("plan_launch", "d_y", d_y, 16, false));
    TRY(check_ptr("plan_launch", "d_ws", d_ws, 256, false));
    if (ws_bytes < p->ws_bytes)
        return drc_fail(DRC_ERR_WORKSPACE, "plan_launch: workspace %zu < %zu bytes", ws_bytes, p->ws_bytes);
    hipStream_t s = (hipStream_t)stream;
    if (!s) return plan_enqueue(p, d_x, d_y, (char*)d_ws, s);  // the null stream cannot be captured
    const void* key[5] = {d_ws, (const void*)s, d_x, d_y, (const void*)(uintptr_t)h->gen};
    if (!p->exec || memcmp(key, p->key, sizeof key) != 0) {
        if (p->exec) {
            (void)hipGraphExecDestroy(p->exec);
            p->exec = nullptr;
        }
        if (p->graph) {
            (void)hipGraphDestroy(p->graph);
            p->graph = nullptr;
        }
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        drc_status st = plan_enqueue(p, d_x, d_y, (char*)d_ws, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st != DRC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return drc_fail(DRC_ERR_HIP, "plan_launch: capture failed: %s", hipGetErrorString(e));
        p->graph = g;
        HIPCHK(hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0));
        memcpy(p->key, key, sizeof key);
        p->captures++;
    }
    HIPCHK(hipGraphLaunch(p->exec, s));
    return DRC_OK;
}

namespace drc {
bool e1_band_fits(int Hin, int Win);
bool d1_band_fits(int Hin, int Win);
}  // namespace drc

// ------------------------------------------------------------------ autotuner
extern "C" drc_status drc_cae_autotune(drc_cae* h, int n, int H, int W, const float* d_x, void* d_ws,
                                       size_t ws_bytes, const char* tune_cache, void* stream) {
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "autotune: handle is NULL");
    if (!tune_cache) return drc_fail(DRC_ERR_INVALID_ARG, "autotune: cache path is NULL");
    if (!h->params_set) return drc_fail(DRC_ERR_STATE, "autotune: call drc_cae_set_params first");
    if (h->prec == P_FP8 && !h->calibrated)
        return drc_fail(DRC_ERR_STATE, "autotune: FP8 handle needs drc_cae_calibrate_fp8 first");
    TRY(check_shape("autotune", n, H, W));
    TRY(check_ptr("autotune", "d_x", d_x, 16, false));
    TRY(check_ptr("autotune", "d_ws", d_ws, 256, false));
    size_t need = 0;
    TRY(drc_cae_workspace_size(h, n, H, W, DRC_WS_FORWARD, &need));
    need += align256((size_t)n * H * W * 3 * sizeof(float));
    if (ws_bytes < need) return drc_fail(DRC_ERR_WORKSPACE, "autotune: workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    ActSizes a = act_sizes(h->prec, n, H, W);
    char* ws = (char*)d_ws;
    FwdClass fc;
    memset(&fc, 0, sizeof fc);
    size_t cur = 0;
    void* act[5];
    for (int k = 0; k < 5; ++k) {
        act[k] = ws + cur;
        cur += a.bytes[k];
    }
    fc.b = FwdBufs{d_x, (float*)(ws + cur), act[0], act[1], act[2], act[3], act[4], nullptr, nullptr};
    fc.n = n;
    fc.H = H;
    fc.W = W;
    fc.x_al16 = 1;  // d_x is 16-byte aligned and packed
    auto run = [&](int l0, int l1) -> drc_status {
        if (h->prec == P_F32) return forward_classes<P_F32>(h, h->wf, &fc, 1, l0, l1, s);
        if (h->prec == P_BF16) return forward_classes<P_BF16>(h, h->wf, &fc, 1, l0, l1, s);
        return forward_classes<P_FP8>(h, h->wf, &fc, 1, l0, l1, s);
    };
    const bool prof = h->prof;
    h->prof = false;
    TRY(run(0, 5));  // valid activations for every layer's input
    TuneTable tune;
    load_tune(tune_cache, tune);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    drc_status st = DRC_OK;
    for (int l = 0; l < 6 && st == DRC_OK; ++l) {
        TuneEntry best;
        best.us = 1e30;
        // E1 / D1 (BF16, FP8) in band-staged kernels: the GEMM tile is not a choice (one timing)
        const bool banded = h->prec != P_F32 && ((l == 0 && e1_band_fits(H, W)) || (l == 5 && d1_band_fits(H / 2, W / 2)));
        bool timed = false;
        for (int npw : {1, 2, 4, 8}) {
            if (!npw_supported(h->prec, l, false, npw)) continue;
            for (int mult : {1, 2, 4, 8}) {
                if (banded && timed) continue;
                timed = true;
                fc.npw[l] = npw;
                fc.tile_px[l] = 64 * npw * mult;
                for (int r = 0; r < 2 && st == DRC_OK; ++r) st = run(l, l);  // warm-up
                if (hipEventRecord(e0, s) != hipSuccess) st = DRC_ERR_HIP;
                const int reps = 5;
                for (int r = 0; r < reps && st == DRC_OK; ++r) st = run(l, l);
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) st = DRC_ERR_HIP;
                float ms = 0;
                if (st == DRC_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = DRC_ERR_HIP;
                if (st != DRC_OK) break;
                const double us = ms * 1000.0 / reps;
                if (us < best.us) {
                    best.us = us;
                    best.npw = npw;
                    best.tile_px = fc.tile_px[l];
                }
            }
            if (st != DRC_OK) break;
        }
        if (st == DRC_OK) {
            tune[tune_key(h->arch, h->prec, l, H, W)] = best;
            h->gen++;
            h->tile[{l, H}] = best.npw;
            h->tile_px[{l, H}] = best.tile_px;
            fc.npw[l] = best.npw;
            fc.tile_px[l] = best.tile_px;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->prof = prof;
    if (st != DRC_OK) return st == DRC_ERR_HIP ? drc_fail(st, "autotune: HIP event failure") : st;
    return save_tune(tune_cache, tune);
}
