// hx_tune.cpp -- the autotuner (placeholder until the schedule search lands).
#include "hx_pipeline.h"

using namespace hx;

extern "C" {

hx_status hx_autotune(hx_pipeline* p, int64_t height, int64_t width, const char* cache_path) {
    (void)p; (void)height; (void)width; (void)cache_path;
    return fail(HX_E_UNSUPPORTED, "autotuner not built yet");
}

hx_status hx_autotune_load(hx_pipeline* p, const char* cache_path) {
    (void)p; (void)cache_path;
    return fail(HX_E_UNSUPPORTED, "autotuner not built yet");
}

}
