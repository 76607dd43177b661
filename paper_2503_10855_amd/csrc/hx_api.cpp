// hx_api.cpp -- the C ABI of libhx.so: pipeline lifetime, validation,
// schedule choice, and the host side of the per-image, stage-hook and
// batched forms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <string>

#include "../../include/hx.h"
#include "hx_kernels.h"
#include "hx_pipeline.h"
#include "srad_kernels.h"

namespace hx {

namespace {
thread_local std::string t_err;
}

void set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
}

hx_status fail(hx_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    logf(1, "error %s: %s", hx_status_str(st), buf);
    return st;
}

hx_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? HX_E_NOMEM : HX_E_HIP, "%s: %s", what,
                hipGetErrorString(e));
}

hipError_t DevBuf::alloc(size_t n, MemStats& m) {
    release();
    if (n == 0) return hipSuccess;
    const size_t want = n < 256 ? 256 : n;
    ++m.allocations;
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        ptr = nullptr;
        return e;
    }
    bytes = want;
    m.device_bytes += want;
    return hipSuccess;
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

hipError_t HostBuf::alloc(size_t n, MemStats& m) {
    release();
    if (n == 0) return hipSuccess;
    ++m.allocations;
    hipError_t e = hipHostMalloc(&ptr, n, hipHostMallocDefault);
    if (e != hipSuccess) {
        ptr = nullptr;
        return e;
    }
    bytes = n;
    m.pinned_bytes += n;
    return hipSuccess;
}

void HostBuf::release() {
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

// Elements of one per-image plane (rows of round_up(W, 4) elements).
static int64_t plane_capacity(int64_t max_pixels) { return max_pixels + 3 * 65536; }

static int64_t round4(int64_t v) { return (v + 3) & ~int64_t(3); }

static int64_t plane_need(int64_t H, int64_t W) { return H * round4(W); }

// Capacities of one batch context.  Pass-1 items: about twice the tiles
// of max_pixels in full tiles plus 16 per image; a batch of images so thin
// or small that it needs more runs as several launches (run_batched).
static BatchCaps batch_caps(const hx_params& prm, bool store_plane) {
    BatchCaps c;
    const SweepGeom g{prm.ksize, batch_sweep_c(), kBatchTyMin};
    const int64_t P = prm.max_pixels, n = prm.max_images;
    c.items1 = 2 * ((P + (int64_t)g.ow() * g.ty - 1) / ((int64_t)g.ow() * g.ty)) + 16 * n + 4096;
    c.items2 = std::max<int64_t>(c.items1, P / 1024 + 2 * n + 1024);
    c.items0 = 5 * c.items1;
    c.list_entries = P / 16 + 16;
    c.table_bytes = batch_table_bytes((int)n, c.items1, c.items2, c.items0);
    c.code_elems = store_plane ? plane_capacity(P) : 0;
    return c;
}

ShapeClass shape_class(int64_t H, int64_t W) {
    auto lg = [](int64_t v) {
        int b = 0;
        while ((v >> (b + 1)) > 0) ++b;
        return b;
    };
    return ShapeClass{lg(H), lg(W)};
}

static bool fused_ks(int ks) { return ks == 3 || ks == 5 || ks == 7; }

hx_status validate_schedule(const hx_pipeline* p, const hx_schedule& s) {
    if (s.fusion_depth < 1 || s.fusion_depth > 4)
        return fail(HX_E_INVALID, "fusion_depth %d not in 1..4", s.fusion_depth);
    if (s.reduce_mode < HX_REDUCE_TREE || s.reduce_mode > HX_REDUCE_SEQUENTIAL)
        return fail(HX_E_INVALID, "reduce_mode %d unknown", s.reduce_mode);
    if (s.reduce_mode != HX_REDUCE_TREE && s.fusion_depth != 1)
        return fail(HX_E_INVALID, "reduce_mode %d needs fusion_depth 1", s.reduce_mode);
    if (s.fusion_depth == 1) {
        if (!(s.tile_w == 16 || s.tile_w == 32 || s.tile_w == 64) ||
            !(s.tile_h == 16 || s.tile_h == 32))
            return fail(HX_E_INVALID, "depth-1 tile %dx%d not in {16,32,64}x{16,32}",
                        s.tile_w, s.tile_h);
        return HX_OK;
    }
    if (!fused_ks(p->prm.ksize))
        return fail(HX_E_UNSUPPORTED, "fused depths need ksize 3, 5 or 7 (have %d)",
                    p->prm.ksize);
    if (!(s.tile_w == 64 || s.tile_w == 128 || s.tile_w == 256) ||
        !sweep_supported(p->prm.ksize, s.tile_w / 64, s.tile_h))
        return fail(HX_E_INVALID,
                    "sweep tile %dx%d: width not 64, 128 or 256, or height not a multiple "
                    "of 8 in 8..256",
                    s.tile_w, s.tile_h);
    if (s.fusion_depth == 4 && s.pass_mode != HX_PASS_STORE &&
        s.pass_mode != HX_PASS_RECOMPUTE && s.pass_mode != HX_PASS_SPECULATE)
        return fail(HX_E_INVALID, "pass_mode %d unknown", s.pass_mode);
    if (s.fusion_depth == 4 && s.pass_mode == HX_PASS_SPECULATE &&
        (s.tile_w != 64 * batch_sweep_c() || s.tile_h < kBatchTyMin || s.tile_h > kBatchTyMax))
        return fail(HX_E_INVALID, "SPECULATE runs %d-column sweep tiles of %d..%d rows",
                    64 * batch_sweep_c(), kBatchTyMin, kBatchTyMax);
    return HX_OK;
}

hx_schedule choose_schedule(const hx_pipeline* p, int64_t H, int64_t W) {
    if (p->forced) return p->forced_sched;
    hx_schedule s;
    auto it = p->tuned.find(shape_class(H, W));
    if (it != p->tuned.end()) {
        s = it->second;
    } else if (fused_ks(p->prm.ksize)) {
        // Untuned: 256-column tiles, one wave each, and the tallest tile of
        // 64, 32, 16 or 8 rows that still gives every SIMD a wave (taller
        // tiles re-read fewer halo rows; a 1080p image in 64-row tiles
        // would leave seven SIMDs in eight idle, and its 8-row tiles
        // finish a call 5 % sooner than 16-row ones).
        const int64_t simds = 4 * (int64_t)(p->cu_count > 0 ? p->cu_count : 256);
        const int64_t strips = (W + 239) / 240;
        int th = 64;
        while (th > 8 && strips * ((H + th - 1) / th) < simds) th /= 2;
        s = hx_schedule{256, th, 4, HX_PASS_STORE, HX_REDUCE_TREE};
    } else {
        s = hx_schedule{64, 16, 1, HX_PASS_STORE, HX_REDUCE_TREE};
    }
    // Knobs fixed at creation override the automatic choice.
    if (p->prm.fusion_depth) s.fusion_depth = p->prm.fusion_depth;
    if (p->prm.tile_w) s.tile_w = p->prm.tile_w;
    if (p->prm.tile_h) s.tile_h = p->prm.tile_h;
    if (p->prm.pass_mode) s.pass_mode = p->prm.pass_mode;
    // SPECULATE runs the batch sweep's tile; a tuned tile of another shape
    // gives way to it unless the tile was fixed at creation.
    if (s.fusion_depth == 4 && s.pass_mode == HX_PASS_SPECULATE && !p->prm.tile_w &&
        !p->prm.tile_h &&
        (s.tile_w != 64 * batch_sweep_c() || s.tile_h < kBatchTyMin || s.tile_h > kBatchTyMax)) {
        s.tile_w = 64 * batch_sweep_c();
        s.tile_h = batch_sweep_ty();
    }
    return s;
}

hx_status validate_image(const hx_pipeline* p, const hx_image* img) {
    if (!img) return fail(HX_E_INVALID, "image descriptor is NULL");
    if (!img->src || !img->mask) return fail(HX_E_INVALID, "src or mask is NULL");
    if (img->height < 1 || img->width < 1)
        return fail(HX_E_INVALID, "image %lldx%lld has no pixels",
                    (long long)img->height, (long long)img->width);
    if (img->height >= (int64_t(1) << 31) || img->width >= (int64_t(1) << 31) - 64)
        return fail(HX_E_INVALID, "image side too large");
    if (img->src_pitch < img->width || img->mask_pitch < img->width)
        return fail(HX_E_INVALID, "pitch (src %lld, mask %lld) below width %lld",
                    (long long)img->src_pitch, (long long)img->mask_pitch,
                    (long long)img->width);
    if (img->height * img->width > p->prm.max_pixels)
        return fail(HX_E_INVALID, "image of %lld pixels exceeds max_pixels %lld",
                    (long long)(img->height * img->width), (long long)p->prm.max_pixels);
    return HX_OK;
}

static ImgArgs base_args(const hx_image* img, uint32_t* slot, float* d_max) {
    ImgArgs a{};
    a.src = img->src;
    a.sp = img->src_pitch;
    a.mask = img->mask;
    a.mp = img->mask_pitch;
    a.slot = slot;
    a.dmax = d_max;
    a.H = (int32_t)img->height;
    a.W = (int32_t)img->width;
    a.op = round4(img->width);
    return a;
}

#define HX_TRY(call)                                      \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// Does the pipeline hold scratch for `form`?
static bool has_form(const hx_pipeline* p, int form) { return (p->prm.forms & form) != 0; }

hx_status run_image(hx_pipeline* p, const hx_image* img, float* d_max,
                    const hx_schedule& s, hipStream_t stream) {
    // SPECULATE runs the batch kernels on a batch of one.
    if (s.fusion_depth == 4 && s.pass_mode == HX_PASS_SPECULATE)
        return run_batched(p, img, 1, d_max, HX_PASS_SPECULATE, s.tile_h, stream);
    const int need_form = s.fusion_depth == 4 ? HX_FORM_IMAGE : HX_FORM_STAGES;
    if (!has_form(p, need_form))
        return fail(HX_E_UNSUPPORTED, "the pipeline was created without the %s scratch",
                    need_form == HX_FORM_IMAGE ? "HX_FORM_IMAGE" : "HX_FORM_STAGES");
    if (plane_need(img->height, img->width) > p->plane_elems)
        return fail(HX_E_UNSUPPORTED,
                    "a %lldx%lld image needs stage planes of %lld elements; the pipeline's "
                    "hold %lld (raise max_pixels)",
                    (long long)img->height, (long long)img->width,
                    (long long)plane_need(img->height, img->width), (long long)p->plane_elems);
    // The max slot: this call's of the pair, the other left at zero for the
    // next call.  The fused STORE form's threshold kernel zeroes the other
    // slot, so when the previous call left this one at zero the form needs
    // no clearing launch; every other form clears both slots first.
    uint32_t* const slots = (uint32_t*)p->slot1.ptr;
    uint32_t* const slot = slots + p->img_parity;
    uint32_t* const next = slots + (p->img_parity ^ 1);
    p->img_parity ^= 1;
    p->img_last_slot = slot;
    const bool store_fused = s.fusion_depth == 4 && s.pass_mode == HX_PASS_STORE;
    const bool slot_zero = p->img_next_zero;
    p->img_next_zero = false;  // until this call's launches are all enqueued
    ImgArgs a = base_args(img, slot, d_max);
    const float theta = p->prm.thresh_frac;
    const int ks = p->prm.ksize;
    if (!(store_fused && slot_zero)) HX_TRY(launch_fill_u32(slots, 0u, 2, stream));
    if (s.fusion_depth == 4) {
        const int c = s.tile_w / 64;
        if (s.pass_mode == HX_PASS_STORE) {
            a.fout = (float*)p->planeA.ptr;
            HX_TRY(launch_sweep(SM_STORE, ks, c, s.tile_h, a, p->taps, theta, stream));
            HX_TRY(launch_threshold_code(a, theta, stream, next));
        } else {
            HX_TRY(launch_sweep(SM_MAXONLY, ks, c, s.tile_h, a, p->taps, theta, stream));
            HX_TRY(launch_sweep(SM_MASK, ks, c, s.tile_h, a, p->taps, theta, stream));
            if (d_max) HX_TRY(launch_write_max(a, stream));
        }
        p->img_next_zero = true;
        return HX_OK;
    }
    StageBufs b{};
    b.op = a.op;
    b.B = (float*)p->planeA.ptr;
    b.L = (float*)p->planeL.ptr;
    b.G2 = (float*)p->planeG2.ptr;
    b.Z = (uint8_t*)p->planeZ.ptr;
    b.partial = (float*)p->bufPart.ptr;
    const int tw1 = 64, th1 = 16;  // per-pixel second kernels of depths 2, 3
    if (s.fusion_depth == 2 || s.fusion_depth == 3) {
        const int c = s.tile_w / 64;
        a.fout = s.fusion_depth == 2 ? b.B : b.L;
        a.g2 = b.G2;
        if (s.fusion_depth == 2) {
            HX_TRY(launch_sweep(SM_BG, ks, c, s.tile_h, a, p->taps, theta, stream));
            HX_TRY(launch_lap_zero_cross(a, b, tw1, th1, stream));
        } else {
            HX_TRY(launch_sweep(SM_BGL, ks, c, s.tile_h, a, p->taps, theta, stream));
            HX_TRY(launch_zero_cross(a, b, b.L, tw1, th1, stream));
        }
        HX_TRY(launch_threshold_zg(a, b, theta, tw1, th1, stream));
        p->img_next_zero = true;
        return HX_OK;
    }
    // Depth 1: one kernel per stage.
    HX_TRY(launch_blur(a, b, p->taps, ks, s.tile_w, s.tile_h, stream));
    HX_TRY(launch_laplacian(a, b, s.tile_w, s.tile_h, stream));
    HX_TRY(launch_zero_cross(a, b, b.L, s.tile_w, s.tile_h, stream));
    HX_TRY(launch_sobel_max(a, b, s.tile_w, s.tile_h, s.reduce_mode, stream));
    HX_TRY(launch_threshold_zg(a, b, theta, s.tile_w, s.tile_h, stream));
    p->img_next_zero = true;
    return HX_OK;
}

// Per-image calls share the pipeline's per-image scratch: one on a stream
// other than the previous one's waits (on the device) for the previous
// one's work first.
static hx_status img_order_begin(hx_pipeline* p, hipStream_t stream) {
    if (p->img_used && p->img_stream != stream)
        HX_TRY(hipStreamWaitEvent(stream, p->img_ev, 0));
    return HX_OK;
}
static hx_status img_order_end(hx_pipeline* p, hipStream_t stream) {
    HX_TRY(hipEventRecord(p->img_ev, stream));
    p->img_used = true;
    p->img_stream = stream;
    return HX_OK;
}

hx_status run_image_ordered(hx_pipeline* p, const hx_image* img, float* d_max,
                            const hx_schedule& s, hipStream_t stream) {
    if (s.fusion_depth == 4 && s.pass_mode == HX_PASS_SPECULATE)
        return run_image(p, img, d_max, s, stream);
    hx_status st = img_order_begin(p, stream);
    if (st != HX_OK) return st;
    st = run_image(p, img, d_max, s, stream);
    hx_status st2 = img_order_end(p, stream);
    return st != HX_OK ? st : st2;
}

// ------------------------------------------------------------- batched --
// Allocate one batch context: everything a batched call on it can need,
// sized by the pipeline's capacities.
static hx_status ctx_init(hx_pipeline* p, BatchContext& c) {
    if (c.ready) return HX_OK;
    MemStats& m = p->mem;
    const BatchCaps& k = p->caps;
    const int64_t n = p->prm.max_images;
    HX_TRY(c.slots.alloc(sizeof(uint32_t) * n, m));
    // Bounds (8 B each) and the epoch, cleared once here.
    const int64_t words = 2 * n + 2;
    HX_TRY(c.spec_state.alloc(sizeof(uint32_t) * words, m));
    HX_TRY(hipMemset(c.spec_state.ptr, 0, sizeof(uint32_t) * words));
    HX_TRY(c.table.alloc(k.table_bytes, m));
    HX_TRY(c.h_table.alloc(k.table_bytes, m));
    HX_TRY(c.cand_code.alloc((size_t)k.list_entries * batch_sweep_c() * sizeof(float), m));
    HX_TRY(c.cand_row.alloc((size_t)k.list_entries * sizeof(int32_t), m));
    HX_TRY(c.cand_n.alloc((size_t)k.items1 * sizeof(uint32_t), m));
    if (k.code_elems) HX_TRY(c.code.alloc((size_t)k.code_elems * sizeof(float), m));
    HX_TRY(hipEventCreateWithFlags(&c.ev_done, hipEventDisableTiming));
    for (auto& e : c.ev_t) HX_TRY(hipEventCreate(&e));
    c.ready = true;
    return HX_OK;
}

static void ctx_release(BatchContext& c) {
    for (int i = 0; i < 4; ++i) {
        if (c.exec[i]) (void)hipGraphExecDestroy(c.exec[i]);
        if (c.graph[i]) (void)hipGraphDestroy(c.graph[i]);
    }
    c.table.release();
    c.h_table.release();
    c.slots.release();
    c.spec_state.release();
    c.code.release();
    c.cand_code.release();
    c.cand_row.release();
    c.cand_n.release();
    if (c.ev_done) (void)hipEventDestroy(c.ev_done);
    for (auto& e : c.ev_t)
        if (e) (void)hipEventDestroy(e);
    c = BatchContext{};
}

hx_status ctx_wait(BatchContext& c) {
    if (!c.in_flight) return HX_OK;
    HX_TRY(hipEventSynchronize(c.ev_done));
    c.in_flight = false;
    return HX_OK;
}

// Enqueue [reset, pass 1, pass 2] (SPECULATE: [pass 0, pass 1, pass 2])
// for this context on stream s;
// with `timed`, bracket each launch with the context's timing events
// (ev_t: 0 reset 1 pass-0 4 pass-1 2 pass-2 3).  Each pass runs one wave
// per item (batch_wg_waves() waves per workgroup): a grid sized to the
// batch measured faster than persistent workgroups striding over the
// items.
static int phase_grid(const BatchContext& c, int ph) {
    const int w = batch_wg_waves();
    return (int)std::max<int64_t>(1, (c.n_items[ph] + w - 1) / w);
}

static hipError_t enqueue_phases(hx_pipeline* p, BatchContext& c, int pass, hipStream_t s,
                                 bool timed = false) {
    const int ks = p->prm.ksize;
    hipError_t e = timed ? hipEventRecord(c.ev_t[0], s) : hipSuccess;
    if (e == hipSuccess && pass != HX_PASS_SPECULATE)
        e = launch_batch_reset(c.table.ptr, (uint32_t*)c.slots.ptr, (int)p->prm.max_images, s);
    if (e == hipSuccess && timed) e = hipEventRecord(c.ev_t[1], s);
    if (e == hipSuccess && pass == HX_PASS_SPECULATE)
        e = launch_batch_phase(ks, pass, 0, c.table.ptr, p->taps, phase_grid(c, 0), s);
    if (e == hipSuccess && timed) e = hipEventRecord(c.ev_t[4], s);
    if (e == hipSuccess)
        e = launch_batch_phase(ks, pass, 1, c.table.ptr, p->taps, phase_grid(c, 1), s);
    if (e == hipSuccess && timed) e = hipEventRecord(c.ev_t[2], s);
    if (e == hipSuccess)
        e = launch_batch_phase(ks, pass, 2, c.table.ptr, p->taps, phase_grid(c, 2), s);
    if (e == hipSuccess && timed) e = hipEventRecord(c.ev_t[3], s);
    return e;
}

// Capture the launches once per (context, pass mode, item counts).
static hx_status ctx_graph(hx_pipeline* p, BatchContext& c, int pass) {
    if (c.exec[pass] && std::memcmp(c.graph_items[pass], c.n_items, sizeof c.n_items) == 0)
        return HX_OK;
    if (c.exec[pass]) {
        (void)hipGraphExecDestroy(c.exec[pass]);
        (void)hipGraphDestroy(c.graph[pass]);
        c.exec[pass] = nullptr;
        c.graph[pass] = nullptr;
    }
    hipStream_t cs = p->capture_stream;
    HX_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = enqueue_phases(p, c, pass, cs);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e1 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e1, "capturing the batched launch");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e3, "hipGraphInstantiate");
    }
    c.graph[pass] = g;
    c.exec[pass] = ex;
    std::memcpy(c.graph_items[pass], c.n_items, sizeof c.n_items);
    return HX_OK;
}

// Work items of one image in each pass, and its STORE code elements.
struct ImgWork {
    int64_t tiles = 0, p2 = 0, p0 = 0, code = 0;
};
static ImgWork img_work(const hx_image& im, int pass, const SweepGeom& geo) {
    ImgWork w;
    w.tiles = geo.tiles(im.height, im.width);
    const int64_t rb = batch_p2_rows(im.width);
    w.p2 = pass == HX_PASS_STORE ? (im.height + rb - 1) / rb : w.tiles;
    w.p0 = pass == HX_PASS_SPECULATE ? batch_sample_items(geo.ks, im.height, im.width) : 0;
    w.code = pass == HX_PASS_STORE ? plane_need(im.height, im.width) : 0;
    return w;
}
static bool fits(const BatchCaps& k, const ImgWork& t, int pass) {
    return t.tiles <= k.items1 && t.p2 <= k.items2 && t.p0 <= k.items0 &&
           (pass != HX_PASS_STORE || t.code <= k.code_elems);
}

// Build the descriptor table of a batch in the context's pinned staging
// buffer and copy it to the device on `stream`.  The caller has checked
// that the batch fits the context's capacities.
static hx_status build_table(hx_pipeline* p, BatchContext& c, const hx_image* imgs,
                             int32_t n, float* d_max, int pass, const SweepGeom& geo,
                             hipStream_t stream) {
    c.last_pass = -1;  // the device table is stale until the copy is queued
    const bool spec = pass == HX_PASS_SPECULATE;
    std::vector<ImgWork> w(n);
    ImgWork tot;
    for (int i = 0; i < n; ++i) {
        w[i] = img_work(imgs[i], pass, geo);
        tot.tiles += w[i].tiles;
        tot.p2 += w[i].p2;
        tot.p0 += w[i].p0;
        tot.code += w[i].code;
    }
    if (!fits(p->caps, tot, pass))
        return fail(HX_E_INVALID, "batch exceeds the context's capacities");
    const size_t bytes = batch_table_bytes(n, tot.tiles, tot.p2, tot.p0);

    // Fill the pinned table: header, images, pass-1, pass-2, pass-0 items.
    uint8_t* h = (uint8_t*)c.h_table.ptr;
    BatchHeader hdr{};
    hdr.n_images = n;
    hdr.n_items1 = (int32_t)tot.tiles;
    hdr.n_items2 = (int32_t)tot.p2;
    hdr.pass_mode = pass;
    hdr.theta = p->prm.thresh_frac;
    hdr.n_items0 = (int32_t)tot.p0;
    if (spec) {
        hdr.cand_code = (float*)c.cand_code.ptr;
        hdr.cand_row = (int32_t*)c.cand_row.ptr;
        hdr.cand_n = (uint32_t*)c.cand_n.ptr;
        hdr.bound = (unsigned long long*)c.spec_state.ptr;
        hdr.epoch = (uint32_t*)(hdr.bound + p->prm.max_images);
    }
    std::memcpy(h, &hdr, sizeof hdr);
    ImgArgs* ia = (ImgArgs*)(h + sizeof(BatchHeader));
    int64_t code_off = 0, list_off = 0;
    for (int i = 0; i < n; ++i) {
        ia[i] = base_args(&imgs[i], (uint32_t*)c.slots.ptr + i, d_max ? d_max + i : nullptr);
        ia[i].ty = geo.ty;
        if (pass == HX_PASS_STORE) ia[i].fout = (float*)c.code.ptr + code_off;
        code_off += w[i].code;
        if (spec) {
            const uint32_t cap = spec_tile_cap(imgs[i].height, imgs[i].width, w[i].tiles);
            ia[i].list_base = (uint32_t)list_off;
            ia[i].list_cap = cap;
            list_off += (int64_t)cap * w[i].tiles;
        }
    }
    if (list_off > p->caps.list_entries)
        return fail(HX_E_INVALID, "listing capacity exceeded");  // cannot happen: sum <= P/16
    BatchItem* it = (BatchItem*)(ia + n);
    for (int i = 0; i < n; ++i)
        for (int64_t t = 0; t < w[i].tiles; ++t) *it++ = BatchItem{i, (int32_t)t};
    for (int i = 0; i < n; ++i)
        for (int64_t t = 0; t < w[i].p2; ++t) *it++ = BatchItem{i, (int32_t)t};
    for (int i = 0; i < n; ++i)
        for (int64_t t = 0; t < w[i].p0; ++t) *it++ = BatchItem{i, (int32_t)t};

    HX_TRY(hipMemcpyAsync(c.table.ptr, h, bytes, hipMemcpyHostToDevice, stream));
    c.n_items[0] = tot.p0;
    c.n_items[1] = tot.tiles;
    c.n_items[2] = tot.p2;
    c.last_imgs.assign(imgs, imgs + n);
    c.last_dmax = d_max;
    c.last_pass = pass;
    c.last_ty = geo.ty;
    return HX_OK;
}

// One image whose tiles alone exceed a context's table: the per-image
// RECOMPUTE form (two sweeps and no tables), with the image's max in the
// context's first slot.  Same bits as the batched passes.
static hx_status run_oversized(hx_pipeline* p, BatchContext& c, const hx_image& im,
                               float* d_max, hipStream_t stream) {
    ImgArgs a = base_args(&im, (uint32_t*)c.slots.ptr, d_max);
    const int ks = p->prm.ksize, cw = batch_sweep_c(), ty = batch_sweep_ty();
    HX_TRY(launch_fill_u32(a.slot, 0u, 1, stream));
    HX_TRY(launch_sweep(SM_MAXONLY, ks, cw, ty, a, p->taps, p->prm.thresh_frac, stream));
    HX_TRY(launch_sweep(SM_MASK, ks, cw, ty, a, p->taps, p->prm.thresh_frac, stream));
    if (d_max) HX_TRY(launch_write_max(a, stream));
    return HX_OK;
}

// Launch a batch that fits one context on context c.
static hx_status launch_on(hx_pipeline* p, BatchContext& c, const hx_image* imgs, int32_t n,
                           float* d_max, int pass, const SweepGeom& geo, bool allow_graph,
                           hipStream_t stream) {
    const bool same = c.ready && c.last_pass == pass && c.last_ty == geo.ty &&
                      c.last_dmax == d_max && c.last_imgs.size() == (size_t)n &&
                      std::memcmp(c.last_imgs.data(), imgs, sizeof(hx_image) * n) == 0;
    if (!same) {
        TraceRange tr("hx.batch.table");
        hx_status st = build_table(p, c, imgs, n, d_max, pass, geo, stream);
        if (st != HX_OK) return st;
    }
    TraceRange tr("hx.batch.enqueue");
    // A batch seen again on this context replays a captured graph; a new
    // composition launches its kernels directly (capturing every new batch
    // would cost more than it saves, e.g. when serving).
    static const bool no_graph = std::getenv("HX_NO_GRAPH") != nullptr;
    const char* how;
    if (p->timing) {
        HX_TRY(enqueue_phases(p, c, pass, stream, true));
        p->last_timed_ctx = (int)(&c - p->ctx);
        how = "timed launches";
    } else if (no_graph || !same || !allow_graph) {
        HX_TRY(enqueue_phases(p, c, pass, stream));
        how = "direct launches";
    } else {
        const bool captured = c.exec[pass] != nullptr &&
                              std::memcmp(c.graph_items[pass], c.n_items, sizeof c.n_items) == 0;
        hx_status st = ctx_graph(p, c, pass);
        if (st != HX_OK) return st;
        HX_TRY(hipGraphLaunch(c.exec[pass], stream));
        how = captured ? "graph replay" : "graph capture + launch";
    }
    logf(2, "batch context %d: %d images, items %lld / %lld / %lld (pass 1 / 2 / 0), %s",
         (int)(&c - p->ctx), n, (long long)c.n_items[1], (long long)c.n_items[2],
         (long long)c.n_items[0], how);
    return HX_OK;
}

BatchKey batch_key(const hx_image* imgs, int32_t n) {
    int64_t px = 0;
    for (int i = 0; i < n; ++i) px += imgs[i].height * imgs[i].width;
    auto lg = [](int64_t v) {
        int b = 0;
        while ((v >> (b + 1)) > 0) ++b;
        return b;
    };
    return BatchKey{lg(px), lg(n)};
}

hx_status run_batched(hx_pipeline* p, const hx_image* imgs, int32_t n,
                      float* d_max, int pass, int ty, hipStream_t stream, int ctx) {
    const int ks = p->prm.ksize;
    TraceRange trace("hx.batch");
    const char* ty_from = ty ? "fixed" : "default";
    {
        auto it = p->batch_tuned.find(batch_key(imgs, n));
        if (it != p->batch_tuned.end()) {
            if (!ty) {
                ty = it->second.ty;
                ty_from = "tuned";
            }
            // A tuned STORE needs the STORE plane; without it the default
            // pass structure runs.
            if (!pass && (it->second.pass != HX_PASS_STORE || has_form(p, HX_FORM_BATCH_STORE)))
                pass = it->second.pass;
        }
    }
    if (!ty) ty = batch_sweep_ty();
    if (!pass) pass = kBatchPass;
    if (ty < kBatchTyMin || ty > kBatchTyMax || ty % 8 != 0)
        return fail(HX_E_INVALID, "batch tile height %d not a multiple of 8 in %d..%d", ty,
                    kBatchTyMin, kBatchTyMax);
    const SweepGeom geo{ks, batch_sweep_c(), ty};
    if (pass < HX_PASS_STORE || pass > HX_PASS_SPECULATE)
        return fail(HX_E_INVALID, "pass_mode %d unknown", pass);
    if (!has_form(p, HX_FORM_BATCH))
        return fail(HX_E_UNSUPPORTED, "the pipeline was created without HX_FORM_BATCH scratch");
    if (pass == HX_PASS_STORE && !has_form(p, HX_FORM_BATCH_STORE))
        return fail(HX_E_UNSUPPORTED,
                    "batched STORE needs a pipeline created with HX_FORM_BATCH_STORE");
    std::lock_guard<std::mutex> lk(p->batch_mu);
    // Which context: one that already holds this batch (its table and
    // graph are reused as they are) and is idle; else the oldest of those
    // holding it; else the oldest context.  Consecutive calls that
    // alternate between a few output sets thus settle on contexts of their
    // own, whatever the order of the first calls was.
    auto holds = [&](const BatchContext& c) {
        return c.ready && c.last_pass == pass && c.last_ty == ty && c.last_dmax == d_max &&
               c.last_imgs.size() == (size_t)n &&
               std::memcmp(c.last_imgs.data(), imgs, sizeof(hx_image) * n) == 0;
    };
    int pick = -1, oldest_match = -1, oldest = -1;
    for (int i = 0; i < p->n_ctx; ++i) {
        BatchContext& c = p->ctx[i];
        if (holds(c)) {
            if (!c.in_flight || hipEventQuery(c.ev_done) == hipSuccess) {
                pick = i;
                break;
            }
            if (oldest_match < 0 || c.last_use < p->ctx[oldest_match].last_use) oldest_match = i;
        }
        if (oldest < 0 || c.last_use < p->ctx[oldest].last_use) oldest = i;
    }
    if (pick < 0) pick = oldest_match >= 0 ? oldest_match : oldest;
    if (ctx >= 0) pick = ctx % p->n_ctx;
    BatchContext& c = p->ctx[pick];
    c.last_use = ++p->use_clock;
    hx_status st = ctx_wait(c);
    if (st != HX_OK) return st;

    // The common case: the whole batch fits the context.
    ImgWork tot;
    for (int i = 0; i < n; ++i) {
        const ImgWork w = img_work(imgs[i], pass, geo);
        tot.tiles += w.tiles;
        tot.p2 += w.p2;
        tot.p0 += w.p0;
        tot.code += w.code;
    }
    static const char* const kPassName[] = {"auto", "STORE", "RECOMPUTE", "SPECULATE"};
    if (log_level() >= 1) {
        int64_t px = 0;
        for (int i = 0; i < n; ++i) px += imgs[i].height * imgs[i].width;
        logf(1, "batched call: %d images, %lld px, %s, %d-row tiles (%s), context %d%s", n,
             (long long)px, kPassName[pass], ty, ty_from, pick,
             fits(p->caps, tot, pass) ? "" : ", split into groups");
    }
    if (fits(p->caps, tot, pass)) {
        st = launch_on(p, c, imgs, n, d_max, pass, geo, true, stream);
        if (st != HX_OK) return st;
    } else {
        // Consecutive groups that fit, one after another on this context
        // (each waits for the previous one's table copy before the staging
        // buffer is rewritten); an image that alone does not fit runs in
        // the per-image RECOMPUTE form.
        int i = 0;
        while (i < n) {
            ImgWork acc;
            int j = i;
            while (j < n) {
                const ImgWork w = img_work(imgs[j], pass, geo);
                ImgWork t = acc;
                t.tiles += w.tiles;
                t.p2 += w.p2;
                t.p0 += w.p0;
                t.code += w.code;
                if (!fits(p->caps, t, pass)) break;
                acc = t;
                ++j;
            }
            if (j == i) {
                logf(2, "image %d (%lldx%lld) exceeds a batch table: per-image RECOMPUTE", i,
                     (long long)imgs[i].height, (long long)imgs[i].width);
                st = run_oversized(p, c, imgs[i], d_max ? d_max + i : nullptr, stream);
                c.last_pass = -1;  // the table no longer matches any batch
                ++i;
            } else {
                st = launch_on(p, c, imgs + i, j - i, d_max ? d_max + i : nullptr, pass, geo,
                               false, stream);
                c.last_pass = -1;
                i = j;
            }
            if (st != HX_OK) return st;
            HX_TRY(hipEventRecord(c.ev_done, stream));
            c.in_flight = true;
            if (i < n) {
                st = ctx_wait(c);
                if (st != HX_OK) return st;
            }
        }
    }
    HX_TRY(hipEventRecord(c.ev_done, stream));
    c.in_flight = true;
    return HX_OK;
}

static void compute_taps(int ks, double sigma, Taps& t) {
    const int r = ks / 2;
    double g[kMaxK], sum = 0.0;
    for (int i = 0; i < ks; ++i) {
        const double d = i - r;
        g[i] = std::exp(-(d * d) / (2.0 * sigma * sigma));
        sum += g[i];
    }
    for (int i = 0; i < kMaxK; ++i) t.g[i] = i < ks ? (float)(g[i] / sum) : 0.0f;
}

// Scratch of hx_edge_detect_static: the max slot (first 256 bytes) and the
// pass-1 code plane, in a fixed array that each device holds once.  Host
// code never uses the array's name as an address (on the host it is only a
// stand-in): static_scratch_ptr holds each device's address, looked up with
// hipGetSymbolAddress while that device is current.
static __device__ __align__(256) uint8_t scratch[HX_STATIC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_static_mu;
static void* g_static_ptr[kMaxDevices];

// Look up (once per device) the static scratch's address on `dev`, which
// must be the current device.
static hx_status static_scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(HX_E_INVALID, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_ptr[dev]) return HX_OK;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_static_ptr[dev] = ptr;
    return HX_OK;
}

static uint8_t* static_scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_static_mu);
    return static_cast<uint8_t*>(g_static_ptr[dev]);
}

// SRAD's partial sums: 4 doubles per workgroup of one launch, for any
// image of at most max_pixels pixels (each side at least 1).
static int64_t srad_part_capacity(int64_t P) {
    return (P / 8192 + P / 256 + P / 32 + 4) / 4 + 2;
}

// Everything the pipeline will use, for the forms it was created with.
static hx_status alloc_scratch(hx_pipeline* p) {
    MemStats& m = p->mem;
    const int f = p->prm.forms;
    p->plane_elems = plane_capacity(p->prm.max_pixels);
    const size_t pe = (size_t)p->plane_elems;
    HX_TRY(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking));
    HX_TRY(hipEventCreateWithFlags(&p->img_ev, hipEventDisableTiming));
    HX_TRY(p->slot1.alloc(256, m));
    if (f & (HX_FORM_IMAGE | HX_FORM_STAGES | HX_FORM_SRAD))
        HX_TRY(p->planeA.alloc(pe * sizeof(float), m));
    if (f & (HX_FORM_STAGES | HX_FORM_SRAD)) HX_TRY(p->planeL.alloc(pe * sizeof(float), m));
    if (f & HX_FORM_STAGES) {
        HX_TRY(p->planeG2.alloc(pe * sizeof(float), m));
        HX_TRY(p->planeZ.alloc(pe, m));
        HX_TRY(p->bufPart.alloc((size_t)kTreeThreads * sizeof(float), m));
    }
    if (f & HX_FORM_SRAD)
        HX_TRY(p->srad_part.alloc(
            (size_t)srad_part_capacity(p->prm.max_pixels) * 4 * sizeof(double), m));
    if (f & HX_FORM_BATCH) {
        p->caps = batch_caps(p->prm, (f & HX_FORM_BATCH_STORE) != 0);
        p->n_ctx = p->prm.batch_contexts;
        for (int i = 0; i < p->n_ctx; ++i) {
            hx_status st = ctx_init(p, p->ctx[i]);
            if (st != HX_OK) return st;
        }
    }
    return HX_OK;
}

}  // namespace hx

using namespace hx;

extern "C" {

const char* hx_status_str(hx_status s) {
    switch (s) {
        case HX_OK: return "HX_OK";
        case HX_E_INVALID: return "HX_E_INVALID";
        case HX_E_NOMEM: return "HX_E_NOMEM";
        case HX_E_HIP: return "HX_E_HIP";
        case HX_E_UNSUPPORTED: return "HX_E_UNSUPPORTED";
        case HX_E_BUSY: return "HX_E_BUSY";
        case HX_E_PENDING: return "HX_E_PENDING";
        case HX_E_NOT_FOUND: return "HX_E_NOT_FOUND";
    }
    return "HX_E_UNKNOWN";
}

const char* hx_last_error(void) { return t_err.c_str(); }

hx_status hx_pipeline_create(const hx_params* params, int device, hx_pipeline** out) {
    if (!out) return fail(HX_E_INVALID, "out is NULL");
    hx_params prm{};
    if (params) prm = *params;
    if (prm.ksize == 0) prm.ksize = 5;
    if (prm.sigma == 0.0f) prm.sigma = 1.0f;
    if (prm.thresh_frac == 0.0f) prm.thresh_frac = 0.1f;
    if (prm.max_pixels == 0) prm.max_pixels = int64_t(1) << 25;
    if (prm.max_images == 0) prm.max_images = 1024;
    if (prm.forms == 0) prm.forms = HX_FORM_ALL;
    if (prm.batch_contexts == 0) prm.batch_contexts = 4;
    if ((prm.forms & ~HX_FORM_ALL) != 0)
        return fail(HX_E_INVALID, "forms 0x%x has unknown bits", prm.forms);
    if (prm.batch_contexts < 1 || prm.batch_contexts > hx_pipeline::kMaxContexts)
        return fail(HX_E_INVALID, "batch_contexts %d not in 1..%d", prm.batch_contexts,
                    hx_pipeline::kMaxContexts);
    if (prm.ksize < 1 || prm.ksize > kMaxK || prm.ksize % 2 == 0)
        return fail(HX_E_INVALID, "ksize %d must be odd in 1..%d", prm.ksize, kMaxK);
    if (!(prm.sigma > 0.0f) || !std::isfinite(prm.sigma))
        return fail(HX_E_INVALID, "sigma must be positive and finite");
    if (!(prm.thresh_frac >= 0.0f && prm.thresh_frac <= 1.0f))
        return fail(HX_E_INVALID, "thresh_frac must be in [0, 1]");
    if (prm.max_pixels < 1 || prm.max_images < 1 || prm.max_images > (1 << 20))
        return fail(HX_E_INVALID, "max_pixels and max_images must be positive");
    if (prm.max_pixels > (int64_t(1) << 31))
        return fail(HX_E_INVALID, "max_pixels %lld above 2^31", (long long)prm.max_pixels);
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) return fail(HX_E_HIP, "no HIP device available");
    if (device < 0 || device >= ndev)
        return fail(HX_E_INVALID, "device %d out of range (have %d)", device, ndev);

    hx_pipeline* p = new (std::nothrow) hx_pipeline();
    if (!p) return fail(HX_E_NOMEM, "host allocation failed");
    p->device = device;
    p->prm = prm;
    compute_taps(prm.ksize, prm.sigma, p->taps);
    if (prm.fusion_depth || prm.tile_w || prm.tile_h || prm.pass_mode) {
        hx_schedule s = choose_schedule(p, 1, 1);
        s.reduce_mode = HX_REDUCE_TREE;
        hx_status st = validate_schedule(p, s);
        if (st != HX_OK) {
            delete p;
            return st;
        }
    }
    DeviceGuard g(device);
    (void)hipDeviceGetAttribute(&p->cu_count, hipDeviceAttributeMultiprocessorCount, device);
    hx_status st = alloc_scratch(p);
    if (st == HX_OK) st = static_scratch_init(device);
    if (st != HX_OK) {
        hx_pipeline_destroy(p);
        return st;
    }
    logf(1, "pipeline on device %d: ksize %d, forms 0x%x, %d batch contexts, max_pixels %lld, "
         "max_images %lld; %zu device bytes, %zu pinned bytes in %llu allocations",
         device, p->prm.ksize, (unsigned)p->prm.forms, p->n_ctx, (long long)p->prm.max_pixels,
         (long long)p->prm.max_images, p->mem.device_bytes, p->mem.pinned_bytes,
         (unsigned long long)p->mem.allocations);
    *out = p;
    return HX_OK;
}

void hx_pipeline_destroy(hx_pipeline* p) {
    if (!p) return;
    DeviceGuard g(p->device);
    (void)hipDeviceSynchronize();
    for (auto& c : p->ctx) ctx_release(c);
    p->slot1.release();
    p->planeA.release();
    p->planeL.release();
    p->planeG2.release();
    p->planeZ.release();
    p->bufPart.release();
    p->srad_part.release();
    if (p->img_ev) (void)hipEventDestroy(p->img_ev);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    delete p;
}

hx_status hx_pipeline_memory(const hx_pipeline* p, size_t* device_bytes, size_t* pinned_bytes,
                             uint64_t* allocations) {
    if (!p) return fail(HX_E_INVALID, "pipeline is NULL");
    if (device_bytes) *device_bytes = p->mem.device_bytes;
    if (pinned_bytes) *pinned_bytes = p->mem.pinned_bytes;
    if (allocations) *allocations = p->mem.allocations;
    return HX_OK;
}

hx_status hx_pipeline_sync(hx_pipeline* p) {
    if (!p) return fail(HX_E_INVALID, "pipeline is NULL");
    DeviceGuard g(p->device);
    std::lock_guard<std::mutex> lk(p->batch_mu);
    hx_status first = HX_OK;
    for (auto& c : p->ctx) {
        hx_status st = ctx_wait(c);
        if (first == HX_OK) first = st;
    }
    hipError_t e = hipDeviceSynchronize();
    if (first == HX_OK && e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    return first;
}

hx_status hx_pipeline_set_timing(hx_pipeline* p, int enable) {
    if (!p) return fail(HX_E_INVALID, "pipeline is NULL");
    std::lock_guard<std::mutex> lk(p->batch_mu);
    p->timing = enable != 0;
    if (!p->timing) p->last_timed_ctx = -1;
    return HX_OK;
}

hx_status hx_pipeline_last_timing(hx_pipeline* p, float* ms) {
    if (!p || !ms) return fail(HX_E_INVALID, "NULL argument");
    DeviceGuard g(p->device);
    std::lock_guard<std::mutex> lk(p->batch_mu);
    if (p->last_timed_ctx < 0) return fail(HX_E_INVALID, "no batched call ran in timing mode");
    BatchContext& c = p->ctx[p->last_timed_ctx];
    HX_TRY(hipEventSynchronize(c.ev_t[3]));
    HX_TRY(hipEventElapsedTime(&ms[0], c.ev_t[0], c.ev_t[1]));  // reset
    HX_TRY(hipEventElapsedTime(&ms[1], c.ev_t[4], c.ev_t[2]));  // pass 1
    HX_TRY(hipEventElapsedTime(&ms[2], c.ev_t[2], c.ev_t[3]));  // pass 2
    HX_TRY(hipEventElapsedTime(&ms[3], c.ev_t[1], c.ev_t[4]));  // pass 0
    return HX_OK;
}

hx_status hx_pipeline_set_schedule(hx_pipeline* p, const hx_schedule* s) {
    if (!p) return fail(HX_E_INVALID, "pipeline is NULL");
    if (!s) {
        p->forced = false;
        return HX_OK;
    }
    hx_status st = validate_schedule(p, *s);
    if (st != HX_OK) return st;
    p->forced = true;
    p->forced_sched = *s;
    return HX_OK;
}

hx_status hx_pipeline_get_schedule(const hx_pipeline* p, int64_t height, int64_t width,
                                   hx_schedule* out) {
    if (!p || !out) return fail(HX_E_INVALID, "NULL argument");
    *out = choose_schedule(p, height, width);
    return HX_OK;
}

hx_status hx_edge_detect(hx_pipeline* p, const hx_image* img, float* d_max,
                         hipStream_t stream) {
    if (!p) return fail(HX_E_INVALID, "pipeline is NULL");
    hx_status st = validate_image(p, img);
    if (st != HX_OK) return st;
    const hx_schedule s = choose_schedule(p, img->height, img->width);
    st = validate_schedule(p, s);
    if (st != HX_OK) return st;
    TraceRange trace("hx.edge_detect");
    logf(2, "per-image call %lldx%lld: %s", (long long)img->height, (long long)img->width,
         schedule_text(s).c_str());
    DeviceGuard g(p->device);
    return run_image_ordered(p, img, d_max, s, stream);
}

hx_status hx_edge_detect_static(hx_pipeline* p, const hx_image* img, float* d_max,
                                hipStream_t stream) {
    if (!p) return fail(HX_E_INVALID, "pipeline is NULL");
    hx_status st = validate_image(p, img);
    if (st != HX_OK) return st;
    if (!fused_ks(p->prm.ksize))
        return fail(HX_E_UNSUPPORTED, "the static form needs ksize 3, 5 or 7 (have %d)",
                    p->prm.ksize);
    const int64_t need = plane_need(img->height, img->width);
    if (need > (int64_t)HX_STATIC_MAX_ELEMS)
        return fail(HX_E_INVALID, "a %lldx%lld image needs %lld code elements; the static "
                    "scratch holds %lld", (long long)img->height, (long long)img->width,
                    (long long)need, (long long)HX_STATIC_MAX_ELEMS);
    uint8_t* base = static_scratch_ptr(p->device);
    if (!base) return fail(HX_E_HIP, "static scratch of device %d not set up", p->device);
    // The untuned fused tile: 256 columns, the tallest of 64/32/16 rows that
    // gives every SIMD a tile.
    const int64_t simds = 4 * (int64_t)(p->cu_count > 0 ? p->cu_count : 256);
    const int64_t strips = (img->width + 239) / 240;
    int th = 64;
    while (th > 16 && strips * ((img->height + th - 1) / th) < simds) th /= 2;
    DeviceGuard g(p->device);
    uint32_t* slot = reinterpret_cast<uint32_t*>(base);
    ImgArgs a = base_args(img, slot, d_max);
    a.fout = reinterpret_cast<float*>(base + 256);
    const float theta = p->prm.thresh_frac;
    HX_TRY(launch_fill_u32(slot, 0u, 1, stream));
    HX_TRY(launch_sweep(SM_STORE, p->prm.ksize, 4, th, a, p->taps, theta, stream));
    HX_TRY(launch_threshold_code(a, theta, stream));
    return HX_OK;
}

hx_status hx_edge_detect_batched(hx_pipeline* p, const hx_image* imgs, int32_t n,
                                 float* d_max, hipStream_t stream) {
    if (!p) return fail(HX_E_INVALID, "pipeline is NULL");
    if (!imgs) return fail(HX_E_INVALID, "imgs is NULL");
    if (n < 1 || n > p->prm.max_images)
        return fail(HX_E_INVALID, "n = %d not in 1..max_images (%lld)", n,
                    (long long)p->prm.max_images);
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        hx_status st = validate_image(p, &imgs[i]);
        if (st != HX_OK) {
            std::string m = t_err;
            return fail(st, "image %d: %s", i, m.c_str());
        }
        total += imgs[i].height * imgs[i].width;
    }
    if (total > p->prm.max_pixels)
        return fail(HX_E_INVALID, "batch of %lld pixels exceeds max_pixels %lld",
                    (long long)total, (long long)p->prm.max_pixels);
    DeviceGuard g(p->device);
    if (!fused_ks(p->prm.ksize)) {
        // Only the stage kernels exist for this blur size: run per image.
        for (int i = 0; i < n; ++i) {
            const hx_schedule s = choose_schedule(p, imgs[i].height, imgs[i].width);
            hx_status st =
                run_image_ordered(p, &imgs[i], d_max ? d_max + i : nullptr, s, stream);
            if (st != HX_OK) return st;
        }
        return HX_OK;
    }
    // The pass structure and tile height: fixed at creation or forced, else
    // the batch autotuner's for this batch's class, else the default.
    int pass = 0, ty = 0;
    if (p->prm.pass_mode) pass = p->prm.pass_mode;
    if (p->forced && p->forced_sched.fusion_depth == 4) {
        pass = p->forced_sched.pass_mode;
        if (p->forced_sched.tile_w == 64 * batch_sweep_c() &&
            p->forced_sched.tile_h >= kBatchTyMin && p->forced_sched.tile_h <= kBatchTyMax &&
            p->forced_sched.tile_h % 8 == 0)
            ty = p->forced_sched.tile_h;
    }
    return run_batched(p, imgs, n, d_max, pass, ty, stream);
}

hx_status hx_edge_detect_stages(hx_pipeline* p, const hx_image* img, float* d_B,
                                float* d_L, uint8_t* d_Z, float* d_G, float* d_max,
                                hipStream_t stream) {
    if (!p) return fail(HX_E_INVALID, "pipeline is NULL");
    hx_status st = validate_image(p, img);
    if (st != HX_OK) return st;
    DeviceGuard g(p->device);
    // Depth 1 unless a depth-1, -2 or -3 schedule is forced; depths 2 and 3
    // keep one stage on chip (L, respectively B), which cannot be exported.
    hx_schedule s{64, 16, 1, HX_PASS_STORE, HX_REDUCE_TREE};
    if (p->forced && p->forced_sched.fusion_depth <= 3) s = p->forced_sched;
    if (s.fusion_depth == 2 && d_L)
        return fail(HX_E_UNSUPPORTED, "fusion depth 2 keeps L on chip: pass d_L = NULL");
    if (s.fusion_depth == 3 && d_B)
        return fail(HX_E_UNSUPPORTED, "fusion depth 3 keeps B on chip: pass d_B = NULL");
    st = img_order_begin(p, stream);
    if (st != HX_OK) return st;
    st = run_image(p, img, d_max, s, stream);
    if (st == HX_OK) {
        ImgArgs a = base_args(img, p->img_last_slot, d_max);
        StageBufs b{};
        b.op = a.op;
        b.B = (float*)p->planeA.ptr;
        b.L = (float*)p->planeL.ptr;
        b.G2 = (float*)p->planeG2.ptr;
        b.Z = (uint8_t*)p->planeZ.ptr;
        hipError_t e = launch_export_stages(a, b, d_B, d_L, d_Z, d_G, stream);
        if (e != hipSuccess) st = hip_fail(e, "launch_export_stages");
    }
    hx_status st2 = img_order_end(p, stream);
    return st != HX_OK ? st : st2;
}

hx_status hx_srad(hx_pipeline* p, float* d_J, int64_t height, int64_t width, int64_t pitch,
                  int32_t niter, float lambda, int32_t fused, double* d_q0sqr,
                  hipStream_t stream) {
    TraceRange trace("hx.srad");
    if (!p) return fail(HX_E_INVALID, "pipeline is NULL");
    if (!d_J) return fail(HX_E_INVALID, "d_J is NULL");
    if (height < 1 || width < 1 || pitch < width)
        return fail(HX_E_INVALID, "bad image shape %lldx%lld or pitch %lld",
                    (long long)height, (long long)width, (long long)pitch);
    if (height * width > p->prm.max_pixels)
        return fail(HX_E_INVALID, "image of %lld pixels exceeds max_pixels %lld",
                    (long long)(height * width), (long long)p->prm.max_pixels);
    if (niter < 0) return fail(HX_E_INVALID, "niter %d is negative", niter);
    if (!(lambda == lambda) || lambda < 0.0f || lambda > 4.0f)
        return fail(HX_E_INVALID, "lambda %g not in [0, 4]", (double)lambda);
    if (!has_form(p, HX_FORM_SRAD))
        return fail(HX_E_UNSUPPORTED, "the pipeline was created without HX_FORM_SRAD scratch");
    if (plane_need(height, width) > p->plane_elems)
        return fail(HX_E_UNSUPPORTED, "a %lldx%lld image needs planes of %lld elements; the "
                    "pipeline's hold %lld (raise max_pixels)", (long long)height,
                    (long long)width, (long long)plane_need(height, width),
                    (long long)p->plane_elems);
    if (srad_blocks(height, width) > srad_part_capacity(p->prm.max_pixels))
        return fail(HX_E_UNSUPPORTED, "SRAD partial sums exceed the pipeline's capacity");
    DeviceGuard g(p->device);
    const int64_t pb = (width + 3) & ~int64_t(3);
    hx_status st = img_order_begin(p, stream);
    if (st != HX_OK) return st;
    float* jb = (float*)p->planeA.ptr;
    hipError_t e = launch_srad(d_J, jb, pitch, pb, fused ? nullptr : (float*)p->planeL.ptr, pb,
                               (double*)p->srad_part.ptr, d_q0sqr, (int)height, (int)width,
                               niter, lambda, fused != 0, stream);
    if (e == hipSuccess && niter % 2 == 1)
        e = hipMemcpy2DAsync(d_J, (size_t)pitch * sizeof(float), jb,
                             (size_t)pb * sizeof(float), (size_t)width * sizeof(float),
                             (size_t)height, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) st = hip_fail(e, "SRAD launch");
    hx_status st2 = img_order_end(p, stream);
    return st != HX_OK ? st : st2;
}

}  // extern "C"
