// hx_serve.cpp -- a request loop with continuous batching.
//
// The paper's host backend runs independent calls as concurrent tasks
// (the AsyncCall attribute) and allocates all memory up front from dynamic
// constants (Global Code Motion; The Host Rust Interface).  Here that
// becomes a serving loop:
//   submit   copies the request image into a pinned host pool and queues it
//            (or: reserve hands the caller a slot of that pool to write
//            the image into, commit queues it);
//   admit    a scheduler thread moves queued requests, oldest first, into
//            the device arena while their buffers fit the HBM budget;
//   launch   every admitted request not yet launched joins the next batch
//            (one batched graph launch of the pipeline) on the least busy of
//            S compute streams, bracketed by its host-to-device and
//            device-to-host copies, so batches overlap on the device;
//   retire   a host callback at the end of the batch stamps completion;
//            the scheduler releases the device buffers;
//   poll     hands the mask and the latency (completion minus the
//            request's scheduled arrival) to the caller (or: view lends
//            the mask where it lies in the pool until release).
// Requests that arrive while others are on the device are admitted as
// memory frees up and launched in the next batch.  Batches run the
// pipeline's batched form (SPECULATE); its scratch -- batch contexts with
// their tables and listing stores -- was allocated when the pipeline was
// created, and the HBM budget covers it too: the arena may hold request
// buffers only up to the budget less the pipeline's device bytes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hx_pipeline.h"

namespace hx {
namespace {

// Host copies of request images into and out of the pinned pool, split by
// rows over a pool of threads the server starts once: one thread moves
// host memory at a fraction of what the memory system sustains, a typical
// request (about 1 Mpx, 4 MB in) would otherwise hold its caller for
// hundreds of microseconds, and starting threads per copy costs tens of
// microseconds each.
class CopyPool {
   public:
    explicit CopyPool(int workers) {
        for (int i = 0; i < workers; ++i) {
            try {
                threads_.emplace_back([this] { run(); });
            } catch (...) {
                break;  // fewer helpers: the callers copy more themselves
            }
        }
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : threads_) t.join();
    }
    int helpers() const { return (int)threads_.size(); }

    // Copy rows [0, rows) of row_bytes each; returns when all are copied.
    void copy(void* dst, size_t dst_pitch, const void* src, size_t src_pitch,
              size_t row_bytes, int64_t rows) {
        const size_t total = row_bytes * (size_t)rows;
        const int64_t parts =
            std::min<int64_t>({(int64_t)helpers() + 1, rows,
                               std::max<int64_t>(1, (int64_t)(total / kMinPart))});
        if (parts <= 1) {
            copy_part(dst, dst_pitch, src, src_pitch, row_bytes, 0, rows);
            return;
        }
        const int64_t per = (rows + parts - 1) / parts;
        Latch latch;
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (int64_t k = 1; k < parts; ++k) {
                const int64_t r0 = k * per, r1 = std::min(rows, r0 + per);
                if (r0 >= r1) continue;
                ++latch.left;
                tasks_.push_back(Task{dst, dst_pitch, src, src_pitch, row_bytes, r0, r1, &latch});
            }
        }
        cv_.notify_all();
        copy_part(dst, dst_pitch, src, src_pitch, row_bytes, 0, std::min(rows, per));
        // Help with this copy's parts that no helper has taken yet, then wait.
        for (;;) {
            Task t;
            {
                std::unique_lock<std::mutex> lk(mu_);
                auto it = std::find_if(tasks_.begin(), tasks_.end(),
                                       [&](const Task& x) { return x.latch == &latch; });
                if (it == tasks_.end()) {
                    done_cv_.wait(lk, [&] { return latch.left == 0; });
                    return;
                }
                t = *it;
                tasks_.erase(it);
            }
            finish(t);
        }
    }

   private:
    static constexpr size_t kMinPart = size_t(256) << 10;  // bytes per part, at least
    struct Latch {
        int64_t left = 0;
    };
    struct Task {
        void* dst;
        size_t dst_pitch;
        const void* src;
        size_t src_pitch, row_bytes;
        int64_t r0, r1;
        Latch* latch;
    };
    static void copy_part(void* dst, size_t dst_pitch, const void* src, size_t src_pitch,
                          size_t row_bytes, int64_t r0, int64_t r1) {
        if (dst_pitch == row_bytes && src_pitch == row_bytes) {
            std::memcpy(static_cast<char*>(dst) + (size_t)r0 * dst_pitch,
                        static_cast<const char*>(src) + (size_t)r0 * src_pitch,
                        (size_t)(r1 - r0) * row_bytes);
            return;
        }
        for (int64_t y = r0; y < r1; ++y)
            std::memcpy(static_cast<char*>(dst) + (size_t)y * dst_pitch,
                        static_cast<const char*>(src) + (size_t)y * src_pitch, row_bytes);
    }
    void finish(const Task& t) {
        copy_part(t.dst, t.dst_pitch, t.src, t.src_pitch, t.row_bytes, t.r0, t.r1);
        {
            std::lock_guard<std::mutex> lk(mu_);
            --t.latch->left;
        }
        done_cv_.notify_all();
    }
    void run() {
        for (;;) {
            Task t;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || !tasks_.empty(); });
                if (tasks_.empty()) return;  // stopping
                t = tasks_.front();
                tasks_.pop_front();
            }
            finish(t);
        }
    }
    std::vector<std::thread> threads_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<Task> tasks_;
    bool stop_ = false;
};

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size) with coalescing frees.
class RangeAlloc {
   public:
    explicit RangeAlloc(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t n, size_t* off) {
        n = align_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += n;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = align_up(n);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

   private:
    size_t size_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

// RESERVED: a slot handed to the caller (hx_serve_reserve) not yet
// committed; the scheduler never sees it.
enum ReqState { RESERVED, QUEUED, ADMITTED, LAUNCHED, DONE };

struct Request {
    uint64_t id;
    int64_t h, w;
    double arrival;
    double launch_t = 0.0;  // the scheduler enqueued its batch's copy-in
    double done_t = 0.0;    // its batch's mask copy-out completed
    ReqState state = QUEUED;
    size_t host_off = 0, host_bytes = 0;  // pinned: input then mask
    size_t dev_off = 0, dev_bytes = 0;    // arena: input then mask
    size_t in_bytes() const { return (size_t)h * w * sizeof(float); }
    size_t mask_bytes() const { return (size_t)h * w; }
};

struct Batch;

}  // namespace
}  // namespace hx

struct hx_server {
    hx_pipeline* p = nullptr;
    std::unique_ptr<hx::CopyPool> copies;  // host copies of request images
    hx_serve_params sp{};
    uint8_t* arena = nullptr;
    uint8_t* host = nullptr;  // pinned pool
    std::unique_ptr<hx::RangeAlloc> dev_alloc, host_alloc;
    std::vector<hipStream_t> streams;
    std::vector<int> in_flight;  // batches per stream

    std::mutex mu;
    std::condition_variable cv;        // wakes the scheduler
    std::unordered_map<uint64_t, std::unique_ptr<hx::Request>> reqs;
    std::deque<hx::Request*> queued, admitted;
    std::deque<std::pair<int, std::vector<hx::Request*>>> finished;  // (stream, reqs)
    uint64_t next_id = 1;
    bool stop = false;
    hx_status sticky = HX_OK;
    std::string sticky_msg;
    std::thread sched;
    std::chrono::steady_clock::time_point t0;

    uint64_t completed = 0, batches = 0, pixels = 0;
    int launched_batches_live = 0;
};

namespace hx {
namespace {

double now_s(const hx_server* s) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

struct CallbackData {
    hx_server* s;
    int stream;
    std::vector<Request*> reqs;
};

void on_batch_done(void* arg) {
    // Runs on a runtime thread once the batch's copies and kernels are
    // done: stamp completion and hand the batch to the scheduler.
    std::unique_ptr<CallbackData> d(static_cast<CallbackData*>(arg));
    hx_server* s = d->s;
    const double t = now_s(s);
    std::lock_guard<std::mutex> lk(s->mu);
    for (Request* r : d->reqs) r->done_t = t;
    s->finished.emplace_back(d->stream, std::move(d->reqs));
    s->cv.notify_all();
}

void set_sticky(hx_server* s, hx_status st) {
    if (s->sticky == HX_OK) {
        s->sticky = st;
        s->sticky_msg = hx_last_error();
    }
}

// Launch one batch on stream k.  Called with s->mu held; drops it around
// the HIP calls (the scheduler thread is the only launcher).
void launch_batch(hx_server* s, std::unique_lock<std::mutex>& lk, int k,
                  std::vector<Request*> batch) {
    hipStream_t st = s->streams[k];
    TraceRange trace("hx.serve.batch");
    std::vector<hx_image> imgs;
    imgs.reserve(batch.size());
    const double t_launch = now_s(s);
    for (Request* r : batch) {
        r->state = LAUNCHED;
        r->launch_t = t_launch;
        float* d_in = reinterpret_cast<float*>(s->arena + r->dev_off);
        uint8_t* d_mask = s->arena + r->dev_off + align_up(r->in_bytes());
        imgs.push_back(hx_image{d_in, r->h, r->w, r->w, d_mask, r->w});
    }
    s->in_flight[k]++;
    s->batches++;
    logf(2, "serve: batch of %zu requests on stream %d", batch.size(), k);
    lk.unlock();
    hx_status rc = HX_OK;
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < batch.size() && e == hipSuccess; ++i)
        e = hipMemcpyAsync(const_cast<float*>(imgs[i].src), s->host + batch[i]->host_off,
                           batch[i]->in_bytes(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        rc = run_batched(s->p, imgs.data(), (int32_t)imgs.size(), nullptr, 0, 0, st);
    for (size_t i = 0; i < batch.size() && e == hipSuccess && rc == HX_OK; ++i)
        e = hipMemcpyAsync(s->host + batch[i]->host_off + align_up(batch[i]->in_bytes()),
                           imgs[i].mask, batch[i]->mask_bytes(), hipMemcpyDeviceToHost, st);
    CallbackData* cd = new CallbackData{s, k, batch};
    if (e == hipSuccess && rc == HX_OK) e = hipLaunchHostFunc(st, on_batch_done, cd);
    lk.lock();
    if (e != hipSuccess || rc != HX_OK) {
        delete cd;
        if (rc == HX_OK) rc = hip_fail(e, "serving batch launch");
        set_sticky(s, rc);
        // The batch will never complete: retire it as failed.
        s->finished.emplace_back(k, batch);
    }
}

void scheduler(hx_server* s) {
    DeviceGuard g(s->p->device);
    std::unique_lock<std::mutex> lk(s->mu);
    const int max_batch =
        (int)std::min<int64_t>(std::max(1, s->sp.max_batch), s->p->prm.max_images);
    for (;;) {
        // Retire finished batches: free their device buffers and inputs.
        while (!s->finished.empty()) {
            auto fin = std::move(s->finished.front());
            s->finished.pop_front();
            s->in_flight[fin.first]--;
            for (Request* r : fin.second) {
                s->dev_alloc->release(r->dev_off, r->dev_bytes);
                r->state = DONE;
                s->completed++;
                s->pixels += (uint64_t)(r->h * r->w);
            }
        }
        // Admit queued requests, oldest first, while they fit the budget.
        while (!s->queued.empty()) {
            Request* r = s->queued.front();
            r->dev_bytes = align_up(r->in_bytes()) + align_up(r->mask_bytes());
            if (!s->dev_alloc->alloc(r->dev_bytes, &r->dev_off)) break;
            r->state = ADMITTED;
            s->admitted.push_back(r);
            s->queued.pop_front();
        }
        // Launch: every admitted request joins the next batch, on the least
        // busy stream, while fewer than two batches wait on each stream.
        if (!s->admitted.empty() && s->sticky == HX_OK) {
            int k = (int)(std::min_element(s->in_flight.begin(), s->in_flight.end()) -
                          s->in_flight.begin());
            if (s->in_flight[k] < 2) {
                std::vector<Request*> batch;
                int64_t px = 0;
                while (!s->admitted.empty() && (int)batch.size() < max_batch) {
                    Request* r = s->admitted.front();
                    if (!batch.empty() && px + r->h * r->w > s->p->prm.max_pixels) break;
                    px += r->h * r->w;
                    batch.push_back(r);
                    s->admitted.pop_front();
                }
                launch_batch(s, lk, k, std::move(batch));
                continue;
            }
        }
        if (s->sticky != HX_OK) {
            // After a device error nothing more is launched: retire the
            // waiting requests (polling them reports the error).
            for (Request* r : s->admitted) {
                s->dev_alloc->release(r->dev_off, r->dev_bytes);
                r->state = DONE;
            }
            for (Request* r : s->queued) r->state = DONE;
            s->admitted.clear();
            s->queued.clear();
        }
        if (s->stop && s->queued.empty() && s->admitted.empty() && s->finished.empty() &&
            std::all_of(s->in_flight.begin(), s->in_flight.end(), [](int v) { return v == 0; }))
            break;
        s->cv.wait(lk);
    }
}

}  // namespace
}  // namespace hx

namespace hx {
namespace {

// A new request of h x w with room in the pinned pool, in state RESERVED
// (invisible to the scheduler).  Called with s->mu held.
hx_status new_request(hx_server* s, int64_t h, int64_t w, Request** out) {
    if (h < 1 || w < 1) return fail(HX_E_INVALID, "bad image shape");
    if (h * w > s->p->prm.max_pixels)
        return fail(HX_E_INVALID, "request of %lld pixels exceeds max_pixels",
                    (long long)(h * w));
    auto r = std::make_unique<Request>();
    r->h = h;
    r->w = w;
    r->state = RESERVED;
    r->host_bytes = align_up(r->in_bytes()) + align_up(r->mask_bytes());
    const size_t dev_need = r->host_bytes;
    if (s->sticky != HX_OK) return fail(s->sticky, "server failed: %s", s->sticky_msg.c_str());
    if (dev_need > s->dev_alloc->size() || r->host_bytes > s->host_alloc->size())
        return fail(HX_E_BUSY, "request of %zu bytes can never fit the budget", dev_need);
    if (s->stop) return fail(HX_E_INVALID, "server is shutting down");
    // Never wait here for pool room: it is freed only by collecting
    // finished requests, which a single-threaded caller could then never do.
    if (!s->host_alloc->alloc(r->host_bytes, &r->host_off))
        return fail(HX_E_PENDING, "pinned pool full: poll finished requests, then retry");
    r->id = s->next_id++;
    *out = r.get();
    s->reqs.emplace(r->id, std::move(r));
    return HX_OK;
}

// Queue a filled request.  Called with s->mu held.
void queue_request(hx_server* s, Request* r, double arrival_s) {
    r->arrival = arrival_s;
    r->state = QUEUED;
    s->queued.push_back(r);
    s->cv.notify_all();
}

// The request of `ticket` in state `want`, or an error.  Called with
// s->mu held.
hx_status find_request(hx_server* s, uint64_t ticket, ReqState want, Request** out) {
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return fail(HX_E_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second.get();
    if (r->state != want) {
        if (want == DONE) {
            if (s->sticky != HX_OK)
                return fail(s->sticky, "server failed: %s", s->sticky_msg.c_str());
            if (r->state != RESERVED) return HX_E_PENDING;
        }
        return fail(HX_E_INVALID, "ticket %llu is not %s", (unsigned long long)ticket,
                    want == DONE ? "a committed request" : "a reserved slot");
    }
    if (want == DONE && s->sticky != HX_OK)
        return fail(s->sticky, "server failed: %s", s->sticky_msg.c_str());
    *out = r;
    return HX_OK;
}

// Give a request's pool room back and forget it.  Called with s->mu held.
void drop_request(hx_server* s, Request* r) {
    s->host_alloc->release(r->host_off, r->host_bytes);
    s->reqs.erase(r->id);
}

}  // namespace
}  // namespace hx

using namespace hx;

extern "C" {

hx_status hx_serve_create(hx_pipeline* p, const hx_serve_params* sp, void* d_arena,
                          size_t arena_bytes, hx_server** out) {
    if (!p || !sp || !d_arena || !out) return fail(HX_E_INVALID, "NULL argument");
    if (sp->streams < 1 || sp->streams > 8)
        return fail(HX_E_INVALID, "streams %d not in 1..8", sp->streams);
    if (sp->max_batch < 1) return fail(HX_E_INVALID, "max_batch must be positive");
    if (p->prm.ksize != 3 && p->prm.ksize != 5 && p->prm.ksize != 7)
        return fail(HX_E_UNSUPPORTED, "serving needs ksize 3, 5 or 7");
    if (!(p->prm.forms & HX_FORM_BATCH))
        return fail(HX_E_UNSUPPORTED, "serving needs a pipeline with HX_FORM_BATCH scratch");
    // The pipeline's own device memory counts against the budget.
    const size_t own = p->mem.device_bytes;
    if (sp->hbm_budget <= own + 4 * kAlign)
        return fail(HX_E_INVALID, "HBM budget %zu bytes does not exceed the pipeline's own "
                    "%zu bytes of scratch", sp->hbm_budget, own);
    const size_t budget = std::min(sp->hbm_budget - own, arena_bytes);
    if (budget < 4 * kAlign) return fail(HX_E_INVALID, "HBM budget too small");
    std::unique_ptr<hx_server> s(new (std::nothrow) hx_server());
    if (!s) return fail(HX_E_NOMEM, "host allocation failed");
    s->p = p;
    s->sp = *sp;
    s->arena = static_cast<uint8_t*>(d_arena);
    s->dev_alloc.reset(new RangeAlloc(budget & ~(kAlign - 1)));
    const size_t host_pool = std::max<size_t>(std::min<size_t>(budget, size_t(1) << 30),
                                              size_t(64) << 20);
    DeviceGuard g(p->device);
    hipError_t e = hipHostMalloc((void**)&s->host, host_pool, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "pinned host pool");
    s->host_alloc.reset(new RangeAlloc(host_pool));
    for (int i = 0; i < sp->streams; ++i) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            (void)hipHostFree(s->host);
            return hip_fail(e, "serving streams");
        }
        s->streams.push_back(st);
        s->in_flight.push_back(0);
    }
    s->t0 = std::chrono::steady_clock::now();
    {
        const unsigned hc = std::thread::hardware_concurrency();
        s->copies.reset(new (std::nothrow) CopyPool((int)std::min(7u, hc > 1 ? hc - 1 : 0u)));
        if (!s->copies) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            (void)hipHostFree(s->host);
            return fail(HX_E_NOMEM, "host allocation failed");
        }
    }
    hx_server* raw = s.get();
    try {
        raw->sched = std::thread(scheduler, raw);
    } catch (...) {
        for (auto x : s->streams) (void)hipStreamDestroy(x);
        (void)hipHostFree(s->host);
        return fail(HX_E_NOMEM, "could not start the scheduler thread");
    }
    logf(1, "server: budget %zu bytes (pipeline %zu, arena %zu), %d streams, max batch %d, "
         "pinned pool %zu bytes, %d copy helpers", sp->hbm_budget, own, budget, sp->streams,
         sp->max_batch, host_pool, s->copies->helpers());
    *out = s.release();
    return HX_OK;
}

double hx_serve_now(const hx_server* s) { return s ? now_s(s) : 0.0; }


hx_status hx_serve_submit(hx_server* s, const float* h_src, int64_t h, int64_t w,
                          int64_t pitch, double arrival_s, uint64_t* ticket) {
    if (!s || !h_src || !ticket) return fail(HX_E_INVALID, "NULL argument");
    if (pitch < w) return fail(HX_E_INVALID, "bad image shape or pitch");
    std::unique_lock<std::mutex> lk(s->mu);
    Request* rp = nullptr;
    hx_status st = new_request(s, h, w, &rp);
    if (st != HX_OK) return st;
    lk.unlock();
    // Copy the rows into the pinned pool (the caller may reuse h_src).
    // The request is RESERVED meanwhile: nothing else touches its room.
    s->copies->copy(s->host + rp->host_off, sizeof(float) * (size_t)w, h_src,
                    sizeof(float) * (size_t)pitch, sizeof(float) * (size_t)w, h);
    lk.lock();
    queue_request(s, rp, arrival_s);
    *ticket = rp->id;
    return HX_OK;
}

hx_status hx_serve_reserve(hx_server* s, int64_t h, int64_t w, float** h_slot,
                           uint64_t* ticket) {
    if (!s || !h_slot || !ticket) return fail(HX_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    Request* rp = nullptr;
    hx_status st = new_request(s, h, w, &rp);
    if (st != HX_OK) return st;
    *h_slot = reinterpret_cast<float*>(s->host + rp->host_off);
    *ticket = rp->id;
    return HX_OK;
}

hx_status hx_serve_commit(hx_server* s, uint64_t ticket, double arrival_s) {
    if (!s) return fail(HX_E_INVALID, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    Request* r = nullptr;
    hx_status st = find_request(s, ticket, RESERVED, &r);
    if (st != HX_OK) return st;
    if (s->sticky != HX_OK) return fail(s->sticky, "server failed: %s", s->sticky_msg.c_str());
    if (s->stop) return fail(HX_E_INVALID, "server is shutting down");
    queue_request(s, r, arrival_s);
    return HX_OK;
}

hx_status hx_serve_cancel(hx_server* s, uint64_t ticket) {
    if (!s) return fail(HX_E_INVALID, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    Request* r = nullptr;
    hx_status st = find_request(s, ticket, RESERVED, &r);
    if (st != HX_OK) return st;
    drop_request(s, r);
    return HX_OK;
}

hx_status hx_serve_view(hx_server* s, uint64_t ticket, const uint8_t** h_mask,
                        double* latency_s, double* service_s) {
    if (!s || !h_mask) return fail(HX_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    Request* r = nullptr;
    hx_status st = find_request(s, ticket, DONE, &r);
    if (st != HX_OK) return st;
    *h_mask = s->host + r->host_off + align_up(r->in_bytes());
    if (latency_s) *latency_s = r->done_t - r->arrival;
    if (service_s) *service_s = r->done_t - r->launch_t;
    return HX_OK;
}

hx_status hx_serve_release(hx_server* s, uint64_t ticket) {
    if (!s) return fail(HX_E_INVALID, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    Request* r = nullptr;
    hx_status st = find_request(s, ticket, DONE, &r);
    if (st != HX_OK) return st;
    drop_request(s, r);
    return HX_OK;
}

hx_status hx_serve_poll(hx_server* s, uint64_t ticket, uint8_t* h_mask, int64_t mask_pitch,
                        double* latency_s) {
    return hx_serve_poll_timed(s, ticket, h_mask, mask_pitch, latency_s, nullptr);
}

hx_status hx_serve_poll_timed(hx_server* s, uint64_t ticket, uint8_t* h_mask,
                              int64_t mask_pitch, double* latency_s, double* service_s) {
    if (!s) return fail(HX_E_INVALID, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    Request* r = nullptr;
    hx_status st = find_request(s, ticket, DONE, &r);
    if (st != HX_OK) return st;
    if (h_mask) {
        if (mask_pitch < r->w) return fail(HX_E_INVALID, "mask_pitch below width");
        s->copies->copy(h_mask, (size_t)mask_pitch,
                        s->host + r->host_off + align_up(r->in_bytes()), (size_t)r->w,
                        (size_t)r->w, r->h);
    }
    if (latency_s) *latency_s = r->done_t - r->arrival;
    if (service_s) *service_s = r->done_t - r->launch_t;
    drop_request(s, r);
    return HX_OK;
}

hx_status hx_serve_stats(const hx_server* s, uint64_t* completed, uint64_t* batches,
                         uint64_t* pixels, uint64_t* peak_bytes) {
    if (!s) return fail(HX_E_INVALID, "NULL server");
    hx_server* m = const_cast<hx_server*>(s);
    std::lock_guard<std::mutex> lk(m->mu);
    if (completed) *completed = s->completed;
    if (batches) *batches = s->batches;
    if (pixels) *pixels = s->pixels;
    if (peak_bytes) *peak_bytes = s->dev_alloc->peak();
    return HX_OK;
}

hx_status hx_serve_destroy(hx_server* s) {
    if (!s) return HX_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->sched.joinable()) s->sched.join();
    hx_status st = s->sticky;
    {
        DeviceGuard g(s->p->device);
        for (auto x : s->streams) {
            (void)hipStreamSynchronize(x);
            (void)hipStreamDestroy(x);
        }
        if (s->host) (void)hipHostFree(s->host);
    }
    delete s;
    return st == HX_OK ? HX_OK : fail(st, "server had failed");
}

}  // extern "C"
