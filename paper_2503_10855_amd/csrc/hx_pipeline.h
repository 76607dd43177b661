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

// A device buffer that grows on demand (growth frees and reallocates,
// which waits for the device; it happens only the first time a larger
// size is needed).
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need);
    void release();
};

// Resources of one in-flight batched launch.  Batched calls rotate over a
// few of these so launches on different streams never share scratch.
struct BatchContext {
    bool ready = false;
    DevBuf table;               // device descriptor table (grows on demand)
    void* h_table = nullptr;    // pinned staging copy of the table
    size_t h_table_bytes = 0;
    uint32_t* slots = nullptr;  // max_images max slots
    void* spec_state = nullptr; // SPECULATE: max_images bounds, the epoch
    DevBuf code;                // pass-1 store buffer
    DevBuf cand_code, cand_row, cand_n;  // SPECULATE: listed pixels
    hipEvent_t ev_done = nullptr;
    hipEvent_t ev_t[5] = {};    // timing mode
    bool in_flight = false;
    // Captured [reset, (pass 0,) pass 1, pass 2] per pass mode, with the
    // table address and grid sizes baked into the kernel nodes.
    hipGraphExec_t exec[4] = {};
    hipGraph_t graph[4] = {};
    const void* graph_table[4] = {};
    int64_t graph_items[4][3] = {};  // item counts baked into each graph
    int64_t n_items[3] = {0, 0, 0};  // the table's items of pass 0, 1, 2
    // The call whose table the device copy holds: a repeat of the same
    // batch (same descriptors, outputs and pass mode) reuses it as is.
    std::vector<hx_image> last_imgs;
    float* last_dmax = nullptr;
    int last_pass = -1;
};

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

    bool forced = false;
    hx_schedule forced_sched{};
    std::map<hx::ShapeClass, hx_schedule> tuned;

    // Per-image scratch.
    uint32_t* slot1 = nullptr;
    hx::DevBuf code1, bufB, bufL, bufG2, bufZ, bufPart;
    // SRAD scratch: the second J plane, the c plane (unfused form), the
    // per-wave partial sums, q0^2.
    hx::DevBuf srad_j, srad_c, srad_part;

    // Batched launches.
    static constexpr int kContexts = 6;
    hx::BatchContext ctx[kContexts];
    int next_ctx = 0;
    std::mutex batch_mu;  // guards context rotation (the server calls from
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
// Pass structure of batched calls unless one is fixed: SPECULATE reads
// the input about 1.1 times (once, plus the sampled bands) and measured
// fastest on the 64 x 1920x1080 batch (0.30 ms per step against 0.36 ms
// for RECOMPUTE and 0.46 ms for STORE).
constexpr int kBatchPass = HX_PASS_SPECULATE;

// The batched form with an explicit pass mode.
hx_status run_batched(hx_pipeline* p, const hx_image* imgs, int32_t n,
                      float* d_max, int pass_mode, hipStream_t stream);
// Wait for a context's last launch.
hx_status ctx_wait(BatchContext& c);

}  // namespace hx
