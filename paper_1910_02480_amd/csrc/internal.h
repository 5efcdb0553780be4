// Library-internal declarations shared by the host translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "drc_cae.h"

struct LayerDef {
    bool tconv;
    int cin, cout;
};
extern const LayerDef kLayers[6];

// Geometry of one layer GEMM (forward or backward-data).
struct GemmGeom {
    int mode;      // drc::M_CONV / M_TCONV_PAIRS / M_TCONV_MERGED
    int cin_eff;   // K elements per tap or neighbour
    int rows;      // output channels of the GEMM
    int rows_pad;  // packed rows per block (merged: 4 * rows), padded to 16
    int nblk;      // weight blocks: 1, or 9 (phase, neighbour) pairs
    int nphase;    // same as nblk (kept for the pack launch)
    int kstride;   // K elements per packed row (padded to the MFMA K step)
};

struct drc_cae {
    drc_cae_desc desc;
    int prec = 0;
    int device = 0;
    std::string arch;
    int num_cu = 256;
    void* wf[6] = {};      // forward packs
    void* wb[6] = {};      // backward-data (transposed) packs
    void* wcal[6] = {};    // float32 forward packs of FP8 handles (calibration)
    void* wfrag[6] = {};   // BF16 handles: forward packs in MFMA fragment order (fused forward)
    void* wbfrag[6] = {};  // BF16 handles: backward-data packs in fragment order (fused data gradients)
    size_t wf_bytes[6] = {}, wb_bytes[6] = {};
    float* bias = nullptr; // float32 biases, layer l at bias_slot(l)
    float* scales = nullptr;   // [0..5] weight scales, [6..9] activation scales (FP8)
    unsigned* amax = nullptr;  // scratch for amax reductions
    float host_scales[16];
    int recompute = 0;
    int fused = 1;         // BF16 inference forward of 32x32 / 64x64 maps in one kernel
    bool params_set = false;
    bool calibrated = false;
    const float* packed_from = nullptr;
    // Bumped by every call that changes what a forward computes or how it is
    // scheduled (set_params, calibrate_fp8, set_fused, set_tile, autotune):
    // a plan's captured graph bakes in kernel arguments (FP8 scales, the
    // fused/layer route, tile shapes) and is re-recorded when this changes.
    unsigned long gen = 1;
    std::map<std::pair<int, int>, int> tile;     // (layer, H) -> pixel blocks per wave
    std::map<std::pair<int, int>, int> tile_px;  // (layer, H) -> GEMM pixels per work item
    // optional timing of kernel groups with events on the caller's stream
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_next = 0;
    std::vector<std::pair<int, size_t>> prof_rec;  // (slot, index of the start event)
    // side streams of the backward: the six weight gradients run beside the
    // data-gradient chain (fork and join by events; recorded into graphs as
    // parallel branches)
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {};
    hipEvent_t ev_fork[6] = {};
    hipEvent_t ev_join[kSide] = {};
};

// Timing slots (drc_cae_profile_read): 0..5 forward GEMM of E1..D1,
// 6..11 backward-data GEMM of E1..D1, 12..17 weight gradient of E1..D1,
// 18 bias gradients, 19 L1 loss, 20 Adam and repack, 21 fused forward, 22 fused
// data-gradient chain.
enum { PROF_FWD = 0, PROF_BWD = 6, PROF_WGRAD = 12, PROF_BIAS = 18, PROF_LOSS = 19, PROF_ADAM = 20,
       PROF_FUSED = 21, PROF_FUSED_BWD = 22, PROF_SLOTS = 24 };
// Records the start event of a slot; returns a token for prof_end (or -1).
long prof_begin(drc_cae* h, int slot, hipStream_t s);
void prof_end(drc_cae* h, long token, hipStream_t s);

struct ActSizes {
    long p0, p1, p2, p3;  // pixels at H, H/2, H/4, H/8 (whole batch)
    size_t bytes[5];      // h1 h2 h3 u3 u2
};

struct BwdLayout {
    size_t recomp[3];
    size_t dz_u2, dh1s, dz_u3, dh2s, dz_h3, dz_h2, dz_h1;
    size_t wpart[6];  // weight-gradient partial tiles of each layer (the six run concurrently)
    size_t bpart, bpart_bytes, total;
};

struct StepLayout {
    size_t saved, fwd_scratch, y, dy, loss_part, dparams, bwd, total;
};

drc_status drc_fail(drc_status s, const char* fmt, ...);
drc_status check_shape(const char* who, int n, int H, int W);
drc_status check_ptr(const char* who, const char* name, const void* p, size_t align, bool nullable);
drc_status check_launch(const char* who);

long layer_w_offset(int l);
long layer_b_offset(int l);
inline int bias_slot(int l) {
    static const int off[6] = {0, 32, 96, 224, 288, 320};
    return off[l];
}
int prec_ks(int prec);
int prec_esize(int prec);
size_t align256(size_t v);
GemmGeom gemm_geom(int l, bool backward, int prec);
ActSizes act_sizes(int prec, int n, int H, int W);
void layer_io(int l, int H, int W, int* hin, int* win, int* hout, int* wout);
// Staging tasks (16-byte chunks) per thread of the transpose-read weight
// gradient, gathered and plain operand: the plan keeps a strip within them.
constexpr long kLossPerBlock = 4096;  // L1 loss elements per workgroup (16 per thread)
constexpr int kWgradTG = 9, kWgradTP = 4;   // 4-wave workgroups
constexpr int kWgradTG8 = 5, kWgradTP8 = 4;  // 8-wave workgroups
constexpr int kWgradTGRaw7 = 8, kWgradTGRaw3 = 2;  // float32 gathered operand of E1 / D1 (4 waves): 16-byte chunks
struct WgradPlan {
    int qc, pc, Hr, Wr, JB, PB, VEC, jtiles, ptiles, nchunks;
    long per_block;
    size_t partial_floats;
    // BF16 path with LDS-staged operands (bf16 = 1 when it applies)
    int bf16, QCP, JBW, BPB, R, strips_per_map, total_strips, strips_per_chunk, bchunks, bptiles, qcs, lds;
    int tr;  // bf16 == 1 and the transpose-read kernel applies (QCP staged channels, QR float32 ones)
    int QR, NW;
};
WgradPlan wgrad_plan(int l, int n, int H, int W, int prec);
// Device address of the file-scope scratch array of drc_cae_forward_static
// on the current device (static_ws.hip); called once per device at create.
drc_status static_scratch_setup(int device);
void colsum_split(long npix, int* nblocks, long* per_block);
BwdLayout bwd_layout(int prec, int n, int H, int W, bool recompute_needed);
StepLayout step_layout(int prec, int n, int H, int W, int recompute);

// Buffers of one forward pass over a batch of equal-size maps. x_off/y_off
// (device, per map, may be NULL) place each map's input/output inside packed
// buffers of a mixed-resolution frame.
struct FwdBufs {
    const float* x;
    float* y;
    void *h1, *h2, *h3, *u3, *u2;
    const long* x_off;
    const long* y_off;
};

// One resolution class of a forward launch: its maps, buffers and the tile
// shape per layer (0 = default).
struct FwdClass {
    FwdBufs b;
    int n, H, W;
    int tile_px[6];
    int npw[6];
    int x_al16;  // every map of x starts on a 16-byte boundary
};

drc_status forward_dispatch(drc_cae* h, const FwdBufs& b, int n, int H, int W, int l0, int l1,
                            hipStream_t s);
// d1_per_cu: persistent workgroups per CU of the band-staged D1 launch
template <int P>
drc_status forward_classes(drc_cae* h, void* const* packs, const FwdClass* fc, int nclass, int l0, int l1,
                           hipStream_t s, int d1_per_cu = 2);
int pick_npw(const drc_cae* h, int l, int H, int prec, bool bwd);

// Tile shapes: pixel blocks of 16 per wave built for each layer GEMM.
bool npw_supported(int prec, int layer, bool backward, int npw);
int default_npw(int prec, int layer, bool backward);

// Whole-network BF16 forward with activations in LDS (fused_fwd.hip).
bool fused_forward_size(int H, int W);
int fused_forward_grid(const drc_cae* h, int n, int H, int W);
size_t fused_forward_scratch(const drc_cae* h, int n, int H, int W);
// save: null, or h1 h2 h3 u3 u2 destinations (plain NHWC, null entries skipped).
// FP8 handles, 32x32 / 64x64 maps: the whole network in one kernel (inference).
drc_status fused_fp8_forward(drc_cae* h, const float* x, float* y, int n, int H, int W, const long* x_off,
                             const long* y_off, hipStream_t s);
drc_status fused_forward(drc_cae* h, const float* x, float* y, int n, int H, int W, const long* x_off,
                         const long* y_off, void* scratch, size_t scratch_bytes, hipStream_t s,
                         char* const* save = nullptr, const int32_t* roll = nullptr,
                         const int32_t* flip = nullptr);
// BF16 128x128 maps (zero padding): E1, E2, E3, D3 and D2 in one kernel, x
// in (16-byte aligned maps, x_off as in LayerArgs or null for packed maps),
// h1, h2 and u2 out (plain NHWC, as the layer path writes them, for D1);
// h3 and u3 stay on chip.
bool fused_tail_size(int H, int W);
drc_status fused_tail(drc_cae* h, int n, int H, int W, const float* x, const long* x_off, void* h1, void* h2,
                      void* u2, hipStream_t s);
// h2 -> h3, u3, u2 (the layers a recomputing backward rebuilds), all plain NHWC.
drc_status fused_recompute(drc_cae* h, int n, int H, int W, const void* h2, void* h3, void* u3, void* u2,
                           hipStream_t s);
// The fixed-order gradient sums of a backward pass, collected while its
// kernels are enqueued and run as one launch at its end (grad_final_launch):
// the weight gradient of each layer from its partial tiles (the sum of
// wgrad_final_kernel), the bias gradients from the per-workgroup column sums
// of the whole-network data-gradient chain (the sum of bias_final_kernel)
// and a training step's mean L1 loss from its partial sums (the sum of
// l1_final_kernel). Results are bitwise those of the separate kernels.
struct GradFinal {
    struct Wjob {
        const float* partial;  // [nchunks][9 * qc][pc]
        int nchunks, qc, pc, q_is_cout;
        float scale;
        float* dw;             // the layer's weights in dparams
    } w[6];
    int nw = 0;
    const float* bpart = nullptr;  // [bnrows][bslots] (null: no bias job)
    int bnrows = 0, bslots = 0;
    float bscale = 0.0f;
    float* bdparams = nullptr;
    long boff[6] = {};             // offsets of the six bias vectors in dparams
    int bs0[7] = {};               // first slot of each bias vector, and the slot count
    const double* lpart = nullptr; // L1 loss: per-workgroup partial sums (the sum of l1_final_kernel)
    int lnparts = 0;
    long lcount = 0;
    float* loss = nullptr;
};
drc_status grad_final_launch(const GradFinal& g, hipStream_t s);

// dy -> dz_u2, dh1s, dz_u3, dz_h3, dz_h2, dz_h1 (the data gradients of D1..E2)
// in one kernel, from the saved activations u2 u3 h3 h2 h1 (plain NHWC BF16);
// it also forms every bias gradient (column sums of dy and of the stored
// output gradients), written scaled by gscale into dparams, or, with defer
// set, recorded in *defer for grad_final_launch.
drc_status fused_dgrad(drc_cae* h, int n, int H, int W, const float* dy, const void* u2, const void* u3,
                       const void* h3, const void* h2, const void* h1, void* dz_u2, void* dh1s, void* dz_u3,
                       void* dz_h3, void* dz_h2, void* dz_h1, float* bias_part, size_t bias_part_bytes,
                       float* dparams, float gscale, hipStream_t s, GradFinal* defer = nullptr);
