// Mixed-resolution frames and tile tuning (placeholder until implemented).
#include <hip/hip_runtime.h>

#include "drc_cae.h"
#include "internal.h"

extern "C" drc_status drc_cae_plan_create(drc_cae* h, const drc_map_desc* maps, int count,
                                          const char* tune_cache, drc_plan** out) {
    (void)h; (void)maps; (void)count; (void)tune_cache;
    if (out) *out = nullptr;
    return drc_fail(DRC_ERR_UNSUPPORTED, "plan_create: not built yet");
}
extern "C" drc_status drc_cae_plan_workspace_size(const drc_plan* p, size_t* bytes) {
    (void)p; (void)bytes;
    return drc_fail(DRC_ERR_UNSUPPORTED, "plan_workspace_size: not built yet");
}
extern "C" drc_status drc_cae_plan_launch(drc_plan* p, const float* x, float* y, void* ws, size_t wsb,
                                          void* stream) {
    (void)p; (void)x; (void)y; (void)ws; (void)wsb; (void)stream;
    return drc_fail(DRC_ERR_UNSUPPORTED, "plan_launch: not built yet");
}
extern "C" void drc_cae_plan_destroy(drc_plan* p) { (void)p; }
extern "C" drc_status drc_cae_autotune(drc_cae* h, int n, int H, int W, const float* x, void* ws,
                                       size_t wsb, const char* cache, void* stream) {
    (void)h; (void)n; (void)H; (void)W; (void)x; (void)ws; (void)wsb; (void)cache; (void)stream;
    return drc_fail(DRC_ERR_UNSUPPORTED, "autotune: not built yet");
}
