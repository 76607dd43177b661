// hx_log.cpp -- diagnostics of libhx.so, off unless asked for.
//
//   HX_LOG=1   one line per API call outcome that matters to an operator:
//              pipeline creation (forms, contexts, bytes), each batched
//              call (images, pixels, pass structure, tile height and where
//              it came from, groups, graph capture or replay), the batch
//              autotuner's trials and choice, server creation, and every
//              failing call with its hx_last_error() text;
//   HX_LOG=2   also each per-image call's schedule and each serving batch.
//   HX_TRACE=1 brackets the API calls and the phases of a batched call in
//              roctx ranges, which rocprofv3 --marker-trace records beside
//              the kernels.  The roctx library is opened on first use; if
//              it cannot be, tracing stays off and HX_LOG says so.
// Lines go to stderr, prefixed "[hx]", one fprintf each (lines from
// several threads do not interleave within a line).
#include <dlfcn.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <mutex>

#include "hx_pipeline.h"

namespace hx {
namespace {

int env_int(const char* name) {
    const char* v = std::getenv(name);
    return v ? std::atoi(v) : 0;
}

struct Roctx {
    int (*push)(const char*) = nullptr;
    int (*pop)() = nullptr;
    bool on = false;
};

Roctx& roctx() {
    static Roctx r;
    static std::once_flag once;
    std::call_once(once, [] {
        if (env_int("HX_TRACE") <= 0) return;
        void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
        if (!h) h = dlopen("libroctx64.so.4", RTLD_NOW | RTLD_LOCAL);
        if (h) {
            r.push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
            r.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
        }
        r.on = r.push && r.pop;
        if (!r.on) logf(1, "HX_TRACE set but no roctx library could be opened");
    });
    return r;
}

}  // namespace

int log_level() {
    static const int level = env_int("HX_LOG");
    return level;
}

void logf(int level, const char* fmt, ...) {
    if (log_level() < level) return;
    char buf[768];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[hx] %s\n", buf);
}

TraceRange::TraceRange(const char* name) : on(roctx().on) {
    if (on) roctx().push(name);
}

TraceRange::~TraceRange() {
    if (on) roctx().pop();
}

}  // namespace hx
