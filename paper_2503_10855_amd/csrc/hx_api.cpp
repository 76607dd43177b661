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
    return st;
}

hx_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? HX_E_NOMEM : HX_E_HIP, "%s: %s", what,
                hipGetErrorString(e));
}

hipError_t DevBuf::ensure(size_t need) {
    if (need <= bytes && ptr) return hipSuccess;
    release();
    const size_t n = need < 256 ? 256 : need;
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
        ptr = nullptr;
        return e;
    }
    bytes = n;
    return hipSuccess;
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

ShapeClass shape_class(int64_t H, int64_t W) {
    auto lg = [](int64_t v) {
        int b = 0;
        while ((v >> (b + 1)) > 0) ++b;
        return b;
    };
    return ShapeClass{lg(H), lg(W)};
}

static int64_t round4(int64_t v) { return (v + 3) & ~int64_t(3); }

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
        return fail(HX_E_INVALID, "sweep tile %dx%d not in {64,128,256}x{16,32,64,128}",
                    s.tile_w, s.tile_h);
    if (s.fusion_depth == 4 && s.pass_mode != HX_PASS_STORE &&
        s.pass_mode != HX_PASS_RECOMPUTE && s.pass_mode != HX_PASS_SPECULATE)
        return fail(HX_E_INVALID, "pass_mode %d unknown", s.pass_mode);
    if (s.fusion_depth == 4 && s.pass_mode == HX_PASS_SPECULATE &&
        (s.tile_w != 64 * batch_sweep_c() || s.tile_h != batch_sweep_ty()))
        return fail(HX_E_INVALID, "SPECULATE runs the %dx%d sweep tile only",
                    64 * batch_sweep_c(), batch_sweep_ty());
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
        // 64, 32 or 16 rows that still gives every SIMD a wave (taller
        // tiles re-read fewer halo rows; a 1080p image in 64-row tiles
        // would leave seven SIMDs in eight idle).
        const int64_t simds = 4 * (int64_t)(p->cu_count > 0 ? p->cu_count : 256);
        const int64_t strips = (W + 239) / 240;
        int th = 64;
        while (th > 16 && strips * ((H + th - 1) / th) < simds) th /= 2;
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
        !p->prm.tile_h) {
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

hx_status run_image(hx_pipeline* p, const hx_image* img, float* d_max,
                    const hx_schedule& s, hipStream_t stream) {
    // SPECULATE runs the batch kernels on a batch of one.
    if (s.fusion_depth == 4 && s.pass_mode == HX_PASS_SPECULATE)
        return run_batched(p, img, 1, d_max, HX_PASS_SPECULATE, stream);
    ImgArgs a = base_args(img, p->slot1, d_max);
    const size_t plane = (size_t)a.H * (size_t)a.op;
    const float theta = p->prm.thresh_frac;
    const int ks = p->prm.ksize;
    HX_TRY(launch_fill_u32(p->slot1, 0u, 1, stream));
    if (s.fusion_depth == 4) {
        const int c = s.tile_w / 64;
        if (s.pass_mode == HX_PASS_STORE) {
            HX_TRY(p->code1.ensure(plane * sizeof(float)));
            a.fout = (float*)p->code1.ptr;
            HX_TRY(launch_sweep(SM_STORE, ks, c, s.tile_h, a, p->taps, theta, stream));
            HX_TRY(launch_threshold_code(a, theta, stream));
        } else {
            HX_TRY(launch_sweep(SM_MAXONLY, ks, c, s.tile_h, a, p->taps, theta, stream));
            HX_TRY(launch_sweep(SM_MASK, ks, c, s.tile_h, a, p->taps, theta, stream));
            if (d_max) HX_TRY(launch_write_max(a, stream));
        }
        return HX_OK;
    }
    StageBufs b{};
    b.op = a.op;
    HX_TRY(p->bufG2.ensure(plane * sizeof(float)));
    HX_TRY(p->bufZ.ensure(plane));
    b.G2 = (float*)p->bufG2.ptr;
    b.Z = (uint8_t*)p->bufZ.ptr;
    const int tw1 = 64, th1 = 16;  // per-pixel second kernels of depths 2, 3
    if (s.fusion_depth == 2 || s.fusion_depth == 3) {
        const int c = s.tile_w / 64;
        DevBuf& first = s.fusion_depth == 2 ? p->bufB : p->bufL;
        HX_TRY(first.ensure(plane * sizeof(float)));
        a.fout = (float*)first.ptr;
        a.g2 = b.G2;
        if (s.fusion_depth == 2) {
            b.B = a.fout;
            HX_TRY(launch_sweep(SM_BG, ks, c, s.tile_h, a, p->taps, theta, stream));
            HX_TRY(launch_lap_zero_cross(a, b, tw1, th1, stream));
        } else {
            b.L = a.fout;
            HX_TRY(launch_sweep(SM_BGL, ks, c, s.tile_h, a, p->taps, theta, stream));
            HX_TRY(launch_zero_cross(a, b, b.L, tw1, th1, stream));
        }
        HX_TRY(launch_threshold_zg(a, b, theta, tw1, th1, stream));
        return HX_OK;
    }
    // Depth 1: one kernel per stage.
    HX_TRY(p->bufB.ensure(plane * sizeof(float)));
    HX_TRY(p->bufL.ensure(plane * sizeof(float)));
    b.B = (float*)p->bufB.ptr;
    b.L = (float*)p->bufL.ptr;
    if (s.reduce_mode == HX_REDUCE_TWO_LEVEL) {
        HX_TRY(p->bufPart.ensure((size_t)kTreeThreads * sizeof(float)));
        b.partial = (float*)p->bufPart.ptr;
    }
    HX_TRY(launch_blur(a, b, p->taps, ks, s.tile_w, s.tile_h, stream));
    HX_TRY(launch_laplacian(a, b, s.tile_w, s.tile_h, stream));
    HX_TRY(launch_zero_cross(a, b, b.L, s.tile_w, s.tile_h, stream));
    HX_TRY(launch_sobel_max(a, b, s.tile_w, s.tile_h, s.reduce_mode, stream));
    HX_TRY(launch_threshold_zg(a, b, theta, s.tile_w, s.tile_h, stream));
    return HX_OK;
}

// ------------------------------------------------------------- batched --
static hx_status ctx_init(hx_pipeline* p, BatchContext& c) {
    if (c.ready) return HX_OK;
    HX_TRY(hipMalloc(&c.slots, sizeof(uint32_t) * p->prm.max_images));
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
    c.code.release();
    c.cand_code.release();
    c.cand_row.release();
    c.cand_n.release();
    if (c.h_table) (void)hipHostFree(c.h_table);
    if (c.slots) (void)hipFree(c.slots);
    if (c.spec_state) (void)hipFree(c.spec_state);
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
// per item (workgroups of four waves): a grid sized to the batch measured
// faster than persistent workgroups striding over the items.
static int phase_grid(const BatchContext& c, int ph) {
    return (int)std::max<int64_t>(1, (c.n_items[ph] + 3) / 4);
}

static hipError_t enqueue_phases(hx_pipeline* p, BatchContext& c, int pass, hipStream_t s,
                                 bool timed = false) {
    const int ks = p->prm.ksize;
    hipError_t e = timed ? hipEventRecord(c.ev_t[0], s) : hipSuccess;
    if (e == hipSuccess && pass != HX_PASS_SPECULATE)
        e = launch_batch_reset(c.table.ptr, c.slots, (int)p->prm.max_images, s);
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

// Capture the launches once per (context, pass mode, table address, item
// counts).
static hx_status ctx_graph(hx_pipeline* p, BatchContext& c, int pass) {
    if (c.exec[pass] && c.graph_table[pass] == c.table.ptr &&
        std::memcmp(c.graph_items[pass], c.n_items, sizeof c.n_items) == 0)
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
    c.graph_table[pass] = c.table.ptr;
    std::memcpy(c.graph_items[pass], c.n_items, sizeof c.n_items);
    return HX_OK;
}

static hx_status build_table(hx_pipeline* p, BatchContext& c, const hx_image* imgs,
                             int32_t n, float* d_max, int pass, const SweepGeom& geo,
                             hipStream_t stream);

hx_status run_batched(hx_pipeline* p, const hx_image* imgs, int32_t n,
                      float* d_max, int pass, hipStream_t stream) {
    const int ks = p->prm.ksize;
    const SweepGeom geo{ks, batch_sweep_c(), batch_sweep_ty()};
    std::lock_guard<std::mutex> lk(p->batch_mu);
    if (pass < HX_PASS_STORE || pass > HX_PASS_SPECULATE)
        return fail(HX_E_INVALID, "pass_mode %d unknown", pass);
    BatchContext& c = p->ctx[p->next_ctx];
    p->next_ctx = (p->next_ctx + 1) % hx_pipeline::kContexts;
    hx_status st = ctx_init(p, c);
    if (st != HX_OK) return st;
    st = ctx_wait(c);
    if (st != HX_OK) return st;

    const bool same = c.last_pass == pass && c.last_dmax == d_max &&
                      c.last_imgs.size() == (size_t)n &&
                      std::memcmp(c.last_imgs.data(), imgs, sizeof(hx_image) * n) == 0;
    if (!same) {
        st = build_table(p, c, imgs, n, d_max, pass, geo, stream);
        if (st != HX_OK) return st;
    }
    // A batch seen again on this context replays a captured graph; a new
    // composition launches its kernels directly (capturing every new batch
    // would cost more than it saves, e.g. when serving).
    static const bool no_graph = std::getenv("HX_NO_GRAPH") != nullptr;
    if (p->timing) {
        HX_TRY(enqueue_phases(p, c, pass, stream, true));
        p->last_timed_ctx = (int)(&c - p->ctx);
    } else if (no_graph || !same) {
        HX_TRY(enqueue_phases(p, c, pass, stream));
    } else {
        st = ctx_graph(p, c, pass);
        if (st != HX_OK) return st;
        HX_TRY(hipGraphLaunch(c.exec[pass], stream));
    }
    HX_TRY(hipEventRecord(c.ev_done, stream));
    c.in_flight = true;
    return HX_OK;
}

// Build the descriptor table of a batch in the context's pinned staging
// buffer and copy it to the device on `stream`.
static hx_status build_table(hx_pipeline* p, BatchContext& c, const hx_image* imgs,
                             int32_t n, float* d_max, int pass, const SweepGeom& geo,
                             hipStream_t stream) {
    c.last_pass = -1;  // the device table is stale until the copy is queued
    // Item counts and pass-1 store offsets.
    const bool spec = pass == HX_PASS_SPECULATE;
    std::vector<int64_t> tiles(n), p2n(n), p0n(n), off(n);
    int64_t n1 = 0, n2 = 0, n0 = 0, code_elems = 0;
    for (int i = 0; i < n; ++i) {
        tiles[i] = geo.tiles(imgs[i].height, imgs[i].width);
        const int64_t rb = batch_p2_rows(imgs[i].width);
        p2n[i] = pass == HX_PASS_STORE ? (imgs[i].height + rb - 1) / rb : tiles[i];
        p0n[i] = spec ? batch_sample_items(geo.ks, imgs[i].height, imgs[i].width) : 0;
        n1 += tiles[i];
        n2 += p2n[i];
        n0 += p0n[i];
        off[i] = code_elems;
        if (pass == HX_PASS_STORE) code_elems += imgs[i].height * round4(imgs[i].width);
    }
    if (n1 >= (int64_t(1) << 31) || n2 >= (int64_t(1) << 31) || n0 >= (int64_t(1) << 31))
        return fail(HX_E_INVALID, "batch has too many work items");
    if (pass == HX_PASS_STORE) HX_TRY(c.code.ensure((size_t)code_elems * sizeof(float)));
    if (spec && !c.spec_state) {
        // Bounds (8 B each) and the epoch, cleared once by a fill kernel.
        const int64_t words = 2 * p->prm.max_images + 2;
        HX_TRY(hipMalloc(&c.spec_state, sizeof(uint32_t) * words));
        HX_TRY(launch_fill_u32((uint32_t*)c.spec_state, 0u, words, stream));
    }
    if (spec) {
        const size_t entries = (size_t)n1 * batch_spec_entries();
        HX_TRY(c.cand_code.ensure(entries * geo.c * sizeof(float)));
        HX_TRY(c.cand_row.ensure(entries * sizeof(int32_t)));
        HX_TRY(c.cand_n.ensure((size_t)n1 * sizeof(uint32_t)));
    }
    const size_t bytes = batch_table_bytes(n, n1, n2, n0);
    HX_TRY(c.table.ensure(bytes));
    if (c.h_table_bytes < bytes) {
        if (c.h_table) (void)hipHostFree(c.h_table);
        c.h_table = nullptr;
        c.h_table_bytes = 0;
        HX_TRY(hipHostMalloc(&c.h_table, bytes, hipHostMallocDefault));
        c.h_table_bytes = bytes;
    }

    // Fill the pinned table: header, images, pass-1 items, pass-2 items.
    uint8_t* h = (uint8_t*)c.h_table;
    BatchHeader hdr{};
    hdr.n_images = n;
    hdr.n_items1 = (int32_t)n1;
    hdr.n_items2 = (int32_t)n2;
    hdr.pass_mode = pass;
    hdr.theta = p->prm.thresh_frac;
    hdr.n_items0 = (int32_t)n0;
    if (spec) {
        hdr.cand_code = (float*)c.cand_code.ptr;
        hdr.cand_row = (int32_t*)c.cand_row.ptr;
        hdr.cand_n = (uint32_t*)c.cand_n.ptr;
        hdr.bound = (unsigned long long*)c.spec_state;
        hdr.epoch = (uint32_t*)(hdr.bound + p->prm.max_images);
    }
    std::memcpy(h, &hdr, sizeof hdr);
    ImgArgs* ia = (ImgArgs*)(h + sizeof(BatchHeader));
    for (int i = 0; i < n; ++i) {
        ia[i] = base_args(&imgs[i], c.slots + i, d_max ? d_max + i : nullptr);
        if (pass == HX_PASS_STORE) ia[i].fout = (float*)c.code.ptr + off[i];
    }
    BatchItem* it = (BatchItem*)(ia + n);
    for (int i = 0; i < n; ++i)
        for (int64_t t = 0; t < tiles[i]; ++t) *it++ = BatchItem{i, (int32_t)t};
    for (int i = 0; i < n; ++i)
        for (int64_t t = 0; t < p2n[i]; ++t) *it++ = BatchItem{i, (int32_t)t};
    for (int i = 0; i < n; ++i)
        for (int64_t t = 0; t < p0n[i]; ++t) *it++ = BatchItem{i, (int32_t)t};

    HX_TRY(hipMemcpyAsync(c.table.ptr, h, bytes, hipMemcpyHostToDevice, stream));
    c.n_items[0] = n0;
    c.n_items[1] = n1;
    c.n_items[2] = n2;
    c.last_imgs.assign(imgs, imgs + n);
    c.last_dmax = d_max;
    c.last_pass = pass;
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
    if (prm.ksize < 1 || prm.ksize > kMaxK || prm.ksize % 2 == 0)
        return fail(HX_E_INVALID, "ksize %d must be odd in 1..%d", prm.ksize, kMaxK);
    if (!(prm.sigma > 0.0f) || !std::isfinite(prm.sigma))
        return fail(HX_E_INVALID, "sigma must be positive and finite");
    if (!(prm.thresh_frac >= 0.0f && prm.thresh_frac <= 1.0f))
        return fail(HX_E_INVALID, "thresh_frac must be in [0, 1]");
    if (prm.max_pixels < 1 || prm.max_images < 1 || prm.max_images > (1 << 20))
        return fail(HX_E_INVALID, "max_pixels and max_images must be positive");
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
    e = hipMalloc(&p->slot1, 64);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        hx_status st = hip_fail(e, "pipeline allocation");
        hx_pipeline_destroy(p);
        return st;
    }
    hx_status st = ctx_init(p, p->ctx[0]);
    if (st != HX_OK) {
        hx_pipeline_destroy(p);
        return st;
    }
    *out = p;
    return HX_OK;
}

void hx_pipeline_destroy(hx_pipeline* p) {
    if (!p) return;
    DeviceGuard g(p->device);
    (void)hipDeviceSynchronize();
    for (auto& c : p->ctx) ctx_release(c);
    p->code1.release();
    p->bufB.release();
    p->bufL.release();
    p->bufG2.release();
    p->bufZ.release();
    p->bufPart.release();
    p->srad_j.release();
    p->srad_c.release();
    p->srad_part.release();
    if (p->slot1) (void)hipFree(p->slot1);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    delete p;
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
    DeviceGuard g(p->device);
    return run_image(p, img, d_max, s, stream);
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
            hx_status st = run_image(p, &imgs[i], d_max ? d_max + i : nullptr, s, stream);
            if (st != HX_OK) return st;
        }
        return HX_OK;
    }
    int pass = kBatchPass;
    if (p->prm.pass_mode) pass = p->prm.pass_mode;
    if (p->forced && p->forced_sched.fusion_depth == 4) pass = p->forced_sched.pass_mode;
    return run_batched(p, imgs, n, d_max, pass, stream);
}

hx_status hx_edge_detect_stages(hx_pipeline* p, const hx_image* img, float* d_B,
                                float* d_L, uint8_t* d_Z, float* d_G, float* d_max,
                                hipStream_t stream) {
    if (!p) return fail(HX_E_INVALID, "pipeline is NULL");
    hx_status st = validate_image(p, img);
    if (st != HX_OK) return st;
    DeviceGuard g(p->device);
    hx_schedule s{64, 16, 1, HX_PASS_STORE, HX_REDUCE_TREE};
    if (p->forced && p->forced_sched.fusion_depth == 1) s = p->forced_sched;
    st = run_image(p, img, d_max, s, stream);
    if (st != HX_OK) return st;
    ImgArgs a = base_args(img, p->slot1, d_max);
    StageBufs b{};
    b.op = a.op;
    b.B = (float*)p->bufB.ptr;
    b.L = (float*)p->bufL.ptr;
    b.G2 = (float*)p->bufG2.ptr;
    b.Z = (uint8_t*)p->bufZ.ptr;
    HX_TRY(launch_export_stages(a, b, d_B, d_L, d_Z, d_G, stream));
    return HX_OK;
}

hx_status hx_srad(hx_pipeline* p, float* d_J, int64_t height, int64_t width, int64_t pitch,
                  int32_t niter, float lambda, int32_t fused, double* d_q0sqr,
                  hipStream_t stream) {
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
    DeviceGuard g(p->device);
    const int64_t pb = (width + 3) & ~int64_t(3);
    const size_t plane = (size_t)height * (size_t)pb * sizeof(float);
    HX_TRY(p->srad_j.ensure(plane));
    if (!fused) HX_TRY(p->srad_c.ensure(plane));
    HX_TRY(p->srad_part.ensure((size_t)srad_blocks(height, width) * 4 * sizeof(double)));
    float* jb = (float*)p->srad_j.ptr;
    HX_TRY(launch_srad(d_J, jb, pitch, pb, fused ? nullptr : (float*)p->srad_c.ptr, pb,
                       (double*)p->srad_part.ptr, d_q0sqr,
                       (int)height, (int)width, niter, lambda, fused != 0, stream));
    if (niter % 2 == 1)
        HX_TRY(hipMemcpy2DAsync(d_J, (size_t)pitch * sizeof(float), jb, (size_t)pb * sizeof(float),
                                (size_t)width * sizeof(float), (size_t)height,
                                hipMemcpyDeviceToDevice, stream));
    return HX_OK;
}

}  // extern "C"
