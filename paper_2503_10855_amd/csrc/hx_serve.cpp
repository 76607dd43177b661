// hx_serve.cpp -- the serving loop (placeholder until it lands).
#include "hx_pipeline.h"

using namespace hx;

extern "C" {

hx_status hx_serve_create(hx_pipeline* p, const hx_serve_params* sp, void* d_arena,
                          size_t arena_bytes, hx_server** out) {
    (void)p; (void)sp; (void)d_arena; (void)arena_bytes; (void)out;
    return fail(HX_E_UNSUPPORTED, "server not built yet");
}
hx_status hx_serve_submit(hx_server* s, const float* h_src, int64_t h, int64_t w, int64_t pitch,
                          double arrival_s, uint64_t* ticket) {
    (void)s; (void)h_src; (void)h; (void)w; (void)pitch; (void)arrival_s; (void)ticket;
    return fail(HX_E_UNSUPPORTED, "server not built yet");
}
hx_status hx_serve_poll(hx_server* s, uint64_t ticket, uint8_t* h_mask, int64_t mask_pitch,
                        double* latency_s) {
    (void)s; (void)ticket; (void)h_mask; (void)mask_pitch; (void)latency_s;
    return fail(HX_E_UNSUPPORTED, "server not built yet");
}
double hx_serve_now(const hx_server* s) { (void)s; return 0.0; }
hx_status hx_serve_stats(const hx_server* s, uint64_t* a, uint64_t* b, uint64_t* c, uint64_t* d) {
    (void)s; (void)a; (void)b; (void)c; (void)d;
    return fail(HX_E_UNSUPPORTED, "server not built yet");
}
hx_status hx_serve_destroy(hx_server* s) { (void)s; return HX_OK; }

}
