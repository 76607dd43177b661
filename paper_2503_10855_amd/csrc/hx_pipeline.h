// hx_pipeline.h -- host-side state behind the hx_pipeline handle.
// Internal to libhx.so.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hx.h"
#include "hx_kernels.h"

namespace hx {

// Thread-local error text behind hx_last_error().
void set_error(const char* fmt, ...);
hx_status fail(hx_status st, const char* fmt, ...);
// The scheduling language (hx_sched.cpp): text -> schedule, and back.
hx_status compile_schedule(const char* text, hx_schedule* out);
std::string schedule_text(const hx_schedule& s);
hx_status hip_fail(hipError_t e, const char* what);

// Diagnostics (hx_log.cpp): HX_LOG=<level> prints lines of at most that
// level to stderr; HX_TRACE=1 turns TraceRange into a roctx range.
int log_level();
void logf(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
struct TraceRange {
    bool on;
    explicit TraceRange(const char* name);
    ~TraceRange();
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

// Make `dev` current for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1, dev;
    explicit DeviceGuard(int d) : dev(d) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
    }
};

// A device or pinned host buffer of the pipeline.  Every one is allocated
// by hx_pipeline_create (alloc) and released by hx_pipeline_destroy; no
// call path allocates.  Allocations are counted on the owning pipeline's
// MemStats.
struct MemStats {
    size_t device_bytes = 0, pinned_bytes = 0;
    uint64_t allocations = 0;
};
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipError_t alloc(size_t n, MemStats& m);
    void release();
};
struct HostBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipError_t alloc(size_t n, MemStats& m);
    void release();
};

// Capacities of one batch context, fixed at creation.
struct BatchCaps {
    int64_t items1 = 0, items2 = 0, items0 = 0;  // work items per pass
    int64_t list_entries = 0;                    // SPECULATE listing
    size_t table_bytes = 0;
    int64_t code_elems = 0;                      // STORE code plane (0: none)
};

// Resources of one in-flight batched launch.  Batched calls pick one of a
// few of these so launches on different streams never share scratch.
struct BatchContext {
    bool ready = false;
    DevBuf table;               // device descriptor table
    HostBuf h_table;            // pinned staging copy of the table
    DevBuf slots;               // max_images max slots
    DevBuf spec_state;          // SPECULATE: max_images bounds, the epoch
    DevBuf code;                // pass-1 store buffer (STORE batches)
    DevBuf cand_code, cand_row, cand_n;  // SPECULATE: listed pixels
    hipEvent_t ev_done = nullptr;
    hipEvent_t ev_t[5] = {};    // timing mode
    bool in_flight = false;
    uint64_t last_use = 0;      // the pipeline's call counter at the last use
    // Captured [reset, (pass 0,) pass 1, pass 2] per pass mode, with the
    // table address and grid sizes baked into the kernel nodes.
    hipGraphExec_t exec[4] = {};
    hipGraph_t graph[4] = {};
    int64_t graph_items[4][3] = {};  // item counts baked into each graph
    int64_t n_items[3] = {0, 0, 0};  // the table's items of pass 0, 1, 2
    // The call whose table the device copy holds: a repeat of the same
    // batch (same descriptors, outputs and pass mode) reuses it as is.
    std::vector<hx_image> last_imgs;
    float* last_dmax = nullptr;
    int last_pass = -1;
    int last_ty = 0;
};

// A batch's class for the batch autotuner: floor(log2) of its total
// pixels and of its image count.
struct BatchKey {
    int px, n;
    bool operator<(const BatchKey& o) const { return px != o.px ? px < o.px : n < o.n; }
};
BatchKey batch_key(const hx_image* imgs, int32_t n);
// The batched launch's schedule: rows per sweep tile and pass structure.
struct BatchChoice {
    int ty = 0;
    int pass = 0;
};
// Tile heights the batched form accepts (multiples of 8 in [kBatchTyMin,
// kBatchTyMax]) and the ones the batch autotuner tries.
constexpr int kBatchTyMin = 16, kBatchTyMax = 256;

struct ShapeClass {
    int hb, wb;  // floor(log2(H)), floor(log2(W))
    bool operator<(const ShapeClass& o) const {
        return hb != o.hb ? hb < o.hb : wb < o.wb;
    }
};
ShapeClass shape_class(int64_t H, int64_t W);

}  // namespace hx

struct hx_pipeline {
    int device = 0;
    hx_params prm{};
    hx::Taps taps{};
    int cu_count = 0;
    hx::MemStats mem;

    bool forced = false;
    hx_schedule forced_sched{};
    std::map<hx::ShapeClass, hx_schedule> tuned;
    std::map<hx::BatchKey, hx::BatchChoice> batch_tuned;  // the batch autotuner's

    // Per-image scratch (forms IMAGE, STAGES, SRAD), one set shared by
    // every per-image call; plane_elems is each plane's capacity.
    int64_t plane_elems = 0;
    hx::DevBuf slot1;
    hx::DevBuf planeA;   // STORE code / B / SRAD's second J plane
    hx::DevBuf planeL;   // L / SRAD's c plane
    hx::DevBuf planeG2, planeZ, bufPart;
    hx::DevBuf srad_part;
    // Ordering of per-image calls: each records img_ev on its stream; a
    // call on another stream waits for it first.
    hipEvent_t img_ev = nullptr;
    hipStream_t img_stream = nullptr;
    bool img_used = false;
    // The per-image max slots: slot1 holds two; each call uses one and
    // leaves the other at zero for the next call (img_next_zero says the
    // previous call did).  img_last_slot: the slot of the last call.
    int img_parity = 0;
    bool img_next_zero = false;
    uint32_t* img_last_slot = nullptr;

    // Batched launches.
    static constexpr int kMaxContexts = 8;
    int n_ctx = 0;
    hx::BatchCaps caps;
    hx::BatchContext ctx[kMaxContexts];
    uint64_t use_clock = 0;
    std::mutex batch_mu;  // guards context choice (the server calls from
                          // its own thread)
    hipStream_t capture_stream = nullptr;
    bool timing = false;
    int last_timed_ctx = -1;
};

namespace hx {

// The schedule a call on an H x W image uses (forced > tuned > default),
// with the pipeline's fixed knobs applied.
hx_schedule choose_schedule(const hx_pipeline* p, int64_t H, int64_t W);
hx_status validate_schedule(const hx_pipeline* p, const hx_schedule& s);
hx_status validate_image(const hx_pipeline* p, const hx_image* img);

// The per-image form with an explicit schedule (used by hx_edge_detect
// and the autotuner).
hx_status run_image(hx_pipeline* p, const hx_image* img, float* d_max,
                    const hx_schedule& s, hipStream_t stream);
// run_image ordered after the previous per-image call (see img_ev).
hx_status run_image_ordered(hx_pipeline* p, const hx_image* img, float* d_max,
                            const hx_schedule& s, hipStream_t stream);
// Pass structure of batched calls unless one is fixed: SPECULATE reads
// the input about 1.1 times (once, plus the sampled bands) and measured
// fastest on the 64 x 1920x1080 batch (0.30 ms per step against 0.36 ms
// for RECOMPUTE and 0.46 ms for STORE).
constexpr int kBatchPass = HX_PASS_SPECULATE;

// The batched form.  pass_mode / ty 0: the batch autotuner's choice for
// the batch's class, else SPECULATE / the default tile height.  ctx >= 0
// runs on that batch context (waiting for its previous batch) instead of
// the one the context policy picks; the batch autotuner uses it to keep
// one batch in flight per context.
hx_status run_batched(hx_pipeline* p, const hx_image* imgs, int32_t n,
                      float* d_max, int pass_mode, int ty, hipStream_t stream,
                      int ctx = -1);
// Wait for a context's last launch.
hx_status ctx_wait(BatchContext& c);

}  // namespace hx
