// hx_tune.cpp -- the autotuner: the role the paper gives its schedules
// (fork tiling / chunking / reshaping, fusion, fission; Juno Scheduling
// Language and Use and Impact of Schedules) played by a search over the
// knobs this implementation exposes: tile shape x fusion depth x pass
// structure.  Every candidate computes bit-identical results (the per-pixel
// operation order is fixed), so the choice is purely a matter of speed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hx_kernels.h"
#include "hx_pipeline.h"

namespace hx {

namespace {

// A seeded test image: hashed noise in [0, 0.2) plus a grid of bright
// rectangles, written on the device (timing does not depend on content:
// the kernels have no data-dependent control flow).
__global__ void k_tune_image(float* img, int64_t pitch, int H, int W) {
    const int64_t n = (int64_t)H * W;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
        uint32_t h = (uint32_t)i * 2654435761u ^ 0x9e3779b9u;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        float v = (float)(h & 0xffffu) * (0.2f / 65536.0f);
        if (((x / 97) + (y / 61)) % 5 == 0) v = 0.5f + 0.1f * (float)((x / 97) % 5);
        img[(int64_t)y * pitch + x] = v;
    }
}

// The candidates are schedule programs (see hx_schedule_compile): every
// tile of the unfused stages, and every fusion grouping x sweep tile x
// pass structure, each reducing the max with wave primitives.
std::vector<hx_schedule> candidates(int ks) {
    std::vector<std::string> texts;
    char b[160];
    for (int tw : {16, 32, 64})
        for (int th : {16, 32}) {
            std::snprintf(b, sizeof b,
                          "fork-tile[%d, %d](blur, laplacian, zero_cross, sobel); ", th, tw);
            texts.push_back(std::string(b) + "warp-reduce(max_gradient);");
        }
    if (ks == 3 || ks == 5 || ks == 7) {
        const char* fuse[3] = {"fork-fuse(blur, sobel); fork-fuse(laplacian, zero_cross); ",
                               "fork-fuse(blur, sobel, laplacian); ",
                               "fork-fuse(blur, sobel, laplacian, zero_cross); "};
        for (int depth = 2; depth <= 4; ++depth)
            for (int tw : {64, 128, 256})
                for (int th : {8, 16, 32, 64, 128}) {
                    std::snprintf(b, sizeof b, "fork-tile[%d, %d](blur); ", th, tw);
                    const std::string t =
                        std::string(fuse[depth - 2]) + b + "warp-reduce(max_gradient);";
                    if (depth < 4) {
                        texts.push_back(t);
                    } else {
                        texts.push_back(t + " pass[store](threshold);");
                        texts.push_back(t + " pass[recompute](threshold);");
                    }
                }
        // SPECULATE runs one tile shape.
        texts.push_back(std::string(fuse[2]) +
                        "fork-tile[64, 256](blur); warp-reduce(max_gradient); "
                        "pass[speculate](threshold);");
    }
    std::vector<hx_schedule> c;
    for (const std::string& t : texts) {
        hx_schedule s{};
        if (compile_schedule(t.c_str(), &s) == HX_OK) c.push_back(s);
    }
    return c;
}

// Batch candidates: tile heights x pass structures (STORE only where the
// pipeline holds its code planes).
std::vector<BatchChoice> batch_candidates(const hx_pipeline* p) {
    std::vector<BatchChoice> c;
    std::vector<int> passes = {HX_PASS_SPECULATE, HX_PASS_RECOMPUTE};
    if (p->prm.forms & HX_FORM_BATCH_STORE) passes.push_back(HX_PASS_STORE);
    for (int pass : passes)
        for (int ty : {16, 24, 32, 48, 64, 72, 80, 96, 112, 128, 160})
            c.push_back(BatchChoice{ty, pass});
    return c;
}

bool parse_batch_entry(const char* line, int* ks, BatchKey* k, BatchChoice* c) {
    return std::sscanf(line, " {\"batch\": {\"ksize\": %d, \"px_log2\": %d, \"n_log2\": %d, "
                             "\"tile_h\": %d, \"pass\": %d",
                       ks, &k->px, &k->n, &c->ty, &c->pass) == 5;
}

// Minimal reader for the cache lines this file writes.
bool parse_entry(const char* line, int* ks, int* hb, int* wb, hx_schedule* s) {
    return std::sscanf(line,
                       " {\"ksize\": %d, \"hb\": %d, \"wb\": %d, \"schedule\": [%d, %d, %d, %d, %d]",
                       ks, hb, wb, &s->tile_w, &s->tile_h, &s->fusion_depth, &s->pass_mode,
                       &s->reduce_mode) == 8;
}

}  // namespace

}  // namespace hx

using namespace hx;

extern "C" {

hx_status hx_autotune(hx_pipeline* p, int64_t height, int64_t width, const char* cache_path) {
    if (!p) return fail(HX_E_INVALID, "pipeline is NULL");
    if (height < 1 || width < 1 || height * width > p->prm.max_pixels)
        return fail(HX_E_INVALID, "tuning shape %lldx%lld invalid or above max_pixels",
                    (long long)height, (long long)width);
    DeviceGuard g(p->device);
    const int64_t pitch = (width + 63) & ~int64_t(63);
    float* img = nullptr;
    uint8_t* mask = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&img, sizeof(float) * pitch * height);
    if (e == hipSuccess) e = hipMalloc(&mask, (size_t)pitch * height);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto cleanup = [&]() {
        if (img) (void)hipFree(img);
        if (mask) (void)hipFree(mask);
        if (s) (void)hipStreamDestroy(s);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "autotune allocation");
    }
    hipLaunchKernelGGL(k_tune_image, dim3(1024), dim3(256), 0, s, img, pitch, (int)height,
                       (int)width);
    hx_image im{img, height, width, pitch, mask, pitch};
    hx_schedule best{};
    float best_ms = 1e30f;
    hx_status st = HX_OK;
    const bool was_forced = p->forced;
    p->forced = false;
    struct Trial {
        hx_schedule s;
        float ms;
    };
    std::vector<Trial> trials;
    for (const hx_schedule& c : candidates(p->prm.ksize)) {
        if (validate_schedule(p, c) != HX_OK) continue;
        // One warm-up call (allocates scratch), then the fastest of three.
        st = run_image_ordered(p, &im, nullptr, c, s);
        if (st != HX_OK) break;
        float ms_min = 1e30f;
        for (int r = 0; r < 3 && st == HX_OK; ++r) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) st = run_image_ordered(p, &im, nullptr, c, s);
            if (e == hipSuccess && st == HX_OK) e = hipEventRecord(e1, s);
            if (e == hipSuccess && st == HX_OK) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess && st == HX_OK) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) st = hip_fail(e, "autotune timing");
            if (ms < ms_min) ms_min = ms;
        }
        if (st != HX_OK) break;
        if (std::getenv("HX_TUNE_LOG"))
            std::fprintf(stderr, "tune %lldx%lld k%d: %dx%d depth %d pass %d: %.4f ms\n",
                         (long long)height, (long long)width, p->prm.ksize, c.tile_w, c.tile_h,
                         c.fusion_depth, c.pass_mode, ms_min);
        trials.push_back({c, ms_min});
        if (ms_min < best_ms) {
            best_ms = ms_min;
            best = c;
        }
    }
    p->forced = was_forced;
    e = hipStreamSynchronize(s);
    cleanup();
    if (st != HX_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "autotune");
    if (best_ms >= 1e30f) return fail(HX_E_UNSUPPORTED, "no schedule could run");
    const ShapeClass sc = shape_class(height, width);
    p->tuned[sc] = best;
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f) return fail(HX_E_INVALID, "cannot open autotune cache %s", cache_path);
        // Every measured candidate first (lines the loader skips), then the
        // chosen schedule.
        for (const Trial& t : trials)
            std::fprintf(f,
                         "{\"trial\": {\"ksize\": %d, \"height\": %lld, \"width\": %lld, "
                         "\"schedule\": [%d, %d, %d, %d, %d], \"ms\": %.5f, "
                         "\"text\": \"%s\"}}\n",
                         p->prm.ksize, (long long)height, (long long)width, t.s.tile_w,
                         t.s.tile_h, t.s.fusion_depth, t.s.pass_mode, t.s.reduce_mode, t.ms,
                         schedule_text(t.s).c_str());
        std::fprintf(f,
                     "{\"ksize\": %d, \"hb\": %d, \"wb\": %d, \"schedule\": [%d, %d, %d, %d, %d], "
                     "\"ms\": %.5f, \"height\": %lld, \"width\": %lld}\n",
                     p->prm.ksize, sc.hb, sc.wb, best.tile_w, best.tile_h, best.fusion_depth,
                     best.pass_mode, best.reduce_mode, best_ms, (long long)height,
                     (long long)width);
        std::fclose(f);
    }
    return HX_OK;
}

hx_status hx_autotune_batch(hx_pipeline* p, const hx_image* imgs, int32_t n,
                           const char* cache_path, int32_t* tile_h, int32_t* pass_mode) {
    if (!p || !imgs) return fail(HX_E_INVALID, "NULL argument");
    if (n < 1 || n > p->prm.max_images)
        return fail(HX_E_INVALID, "n = %d not in 1..max_images", n);
    if (!(p->prm.forms & HX_FORM_BATCH))
        return fail(HX_E_UNSUPPORTED, "the pipeline was created without HX_FORM_BATCH scratch");
    if (p->prm.ksize != 3 && p->prm.ksize != 5 && p->prm.ksize != 7)
        return fail(HX_E_UNSUPPORTED, "the batched sweep needs ksize 3, 5 or 7");
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        hx_status st = validate_image(p, &imgs[i]);
        if (st != HX_OK) return st;
        total += imgs[i].height * imgs[i].width;
    }
    if (total > p->prm.max_pixels) return fail(HX_E_INVALID, "batch exceeds max_pixels");
    TraceRange trace("hx.autotune_batch");
    DeviceGuard g(p->device);
    // One stream per batch context, call k on stream and context k mod S:
    // the throughput trials keep that many calls in flight, as a caller
    // feeding batches on as many streams does.  All calls write the same masks with the same bits;
    // after the last one the masks hold the result of any of them.
    const int S = std::max(1, std::min(p->n_ctx, hx_pipeline::kMaxContexts));
    hipStream_t st_[hx_pipeline::kMaxContexts] = {};
    hipEvent_t done_[hx_pipeline::kMaxContexts] = {};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int i = 0; i < S && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&st_[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&done_[i], hipEventDisableTiming);
    }
    auto cleanup = [&]() {
        for (int i = 0; i < S; ++i) {
            if (st_[i]) (void)hipStreamDestroy(st_[i]);
            if (done_[i]) (void)hipEventDestroy(done_[i]);
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "batch autotune setup");
    }
    hipStream_t s = st_[0];
    const BatchKey key = batch_key(imgs, n);
    struct Trial {
        BatchChoice c;
        float ms;       // one call alone: median of five
        float tput_ms;  // per call with S calls in flight: median of three runs
    };
    std::vector<Trial> trials;
    BatchChoice best{};
    float best_ms = 1e30f;
    hx_status st = HX_OK;
    // Elapsed ms between e0 and e1 once e1 has completed.
    auto elapsed = [&](float* t) {
        e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(t, e0, e1);
        if (e != hipSuccess) st = hip_fail(e, "batch autotune timing");
    };
    const std::vector<BatchChoice> cands = batch_candidates(p);
    // Bring the clocks up before the first trial: about 30 ms of calls
    // under the first candidate (a cold start would favour later ones).
    {
        const auto t_end = std::chrono::steady_clock::now() + std::chrono::milliseconds(30);
        int k = 0;
        while (st == HX_OK && (k < 3 * S || std::chrono::steady_clock::now() < t_end)) {
            st = run_batched(p, imgs, n, nullptr, cands[0].pass, cands[0].ty, st_[k % S], k % S);
            if (++k % S == 0 && st == HX_OK)
                for (int i = 0; i < S && st == HX_OK; ++i)
                    if ((e = hipStreamSynchronize(st_[i])) != hipSuccess)
                        st = hip_fail(e, "batch autotune warm-up");
        }
    }
    for (const BatchChoice& c : cands) {
        // Untimed: three calls per stream (each context builds its table,
        // captures its graph and replays it).
        for (int r = 0; r < 3 * S && st == HX_OK; ++r)
            st = run_batched(p, imgs, n, nullptr, c.pass, c.ty, st_[r % S], r % S);
        for (int i = 0; i < S && st == HX_OK; ++i)
            if ((e = hipStreamSynchronize(st_[i])) != hipSuccess)
                st = hip_fail(e, "batch autotune warm-up");
        std::vector<float> ms;
        for (int r = 0; r < 5 && st == HX_OK; ++r) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) st = run_batched(p, imgs, n, nullptr, c.pass, c.ty, s, 0);
            if (e == hipSuccess && st == HX_OK) e = hipEventRecord(e1, s);
            float t = 0.0f;
            if (e != hipSuccess) st = hip_fail(e, "batch autotune timing");
            if (st == HX_OK) elapsed(&t);
            ms.push_back(t);
        }
        // Throughput: 12 S calls round-robin over the S streams, bracketed
        // by e0 (every stream waits for it) and e1 (after every stream);
        // the median of three such runs.  (Runs of 4 S calls let the
        // un-overlapped first and last calls of a run sway the ranking.)
        std::vector<float> tp;
        const int K = 12 * S;
        for (int r = 0; r < 3 && st == HX_OK; ++r) {
            e = hipEventRecord(e0, s);
            for (int i = 1; i < S && e == hipSuccess; ++i) e = hipStreamWaitEvent(st_[i], e0, 0);
            for (int k = 0; k < K && e == hipSuccess && st == HX_OK; ++k)
                st = run_batched(p, imgs, n, nullptr, c.pass, c.ty, st_[k % S], k % S);
            for (int i = 1; i < S && e == hipSuccess && st == HX_OK; ++i) {
                e = hipEventRecord(done_[i], st_[i]);
                if (e == hipSuccess) e = hipStreamWaitEvent(s, done_[i], 0);
            }
            if (e == hipSuccess && st == HX_OK) e = hipEventRecord(e1, s);
            float t = 0.0f;
            if (e != hipSuccess && st == HX_OK) st = hip_fail(e, "batch autotune timing");
            if (st == HX_OK) elapsed(&t);
            tp.push_back(t / K);
        }
        if (st != HX_OK) break;
        std::sort(ms.begin(), ms.end());
        std::sort(tp.begin(), tp.end());
        const Trial t{c, ms[ms.size() / 2], tp[tp.size() / 2]};
        logf(1, "batch tuner: %d-row tiles, pass %d: %.4f ms per call with %d in flight, "
             "%.4f ms alone", c.ty, c.pass, t.tput_ms, S, t.ms);
        trials.push_back(t);
        if (t.tput_ms < best_ms) {
            best_ms = t.tput_ms;
            best = c;
        }
    }
    for (int i = 0; i < S; ++i) {
        const hipError_t ei = hipStreamSynchronize(st_[i]);
        if (e == hipSuccess) e = ei;
    }
    cleanup();
    if (st != HX_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "batch autotune");
    if (best_ms >= 1e30f) return fail(HX_E_UNSUPPORTED, "no batch schedule could run");
    p->batch_tuned[key] = best;
    logf(1, "batch tuner: class (2^%d px, 2^%d images) -> %d-row tiles, pass %d", key.px,
         key.n, best.ty, best.pass);
    if (tile_h) *tile_h = best.ty;
    if (pass_mode) *pass_mode = best.pass;
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f) return fail(HX_E_INVALID, "cannot open autotune cache %s", cache_path);
        for (const Trial& t : trials)
            std::fprintf(f,
                         "{\"batch_trial\": {\"ksize\": %d, \"px_log2\": %d, \"n_log2\": %d, "
                         "\"tile_h\": %d, \"pass\": %d, \"ms\": %.5f, \"tput_ms\": %.5f, "
                         "\"in_flight\": %d, \"pixels\": %lld, \"images\": %d}}\n",
                         p->prm.ksize, key.px, key.n, t.c.ty, t.c.pass, t.ms, t.tput_ms, S,
                         (long long)total, n);
        std::fprintf(f,
                     "{\"batch\": {\"ksize\": %d, \"px_log2\": %d, \"n_log2\": %d, "
                     "\"tile_h\": %d, \"pass\": %d, \"tput_ms\": %.5f}}\n",
                     p->prm.ksize, key.px, key.n, best.ty, best.pass, best_ms);
        std::fclose(f);
    }
    return HX_OK;
}

hx_status hx_autotune_load(hx_pipeline* p, const char* cache_path) {
    if (!p || !cache_path) return fail(HX_E_INVALID, "NULL argument");
    FILE* f = std::fopen(cache_path, "r");
    if (!f) return fail(HX_E_NOT_FOUND, "cannot open autotune cache %s", cache_path);
    char line[512];
    int loaded = 0;
    while (std::fgets(line, sizeof line, f)) {
        int ks, hb, wb;
        BatchKey bk{};
        BatchChoice bc{};
        if (parse_batch_entry(line, &ks, &bk, &bc)) {
            if (ks == p->prm.ksize && bc.ty >= kBatchTyMin && bc.ty <= kBatchTyMax &&
                bc.ty % 8 == 0 && bc.pass >= HX_PASS_STORE && bc.pass <= HX_PASS_SPECULATE) {
                p->batch_tuned[bk] = bc;
                ++loaded;
            }
            continue;
        }
        hx_schedule s{};
        if (!parse_entry(line, &ks, &hb, &wb, &s) || ks != p->prm.ksize) continue;
        if (validate_schedule(p, s) != HX_OK) continue;
        p->tuned[ShapeClass{hb, wb}] = s;  // later lines win
        ++loaded;
    }
    std::fclose(f);
    if (!loaded) return fail(HX_E_NOT_FOUND, "no usable entries in %s", cache_path);
    return HX_OK;
}

}  // extern "C"
