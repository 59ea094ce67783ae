// Per-launch kernel timing for measurement (tsm2x_timing_* in include/tsm2x.h).
// Off by default: a launch then costs one relaxed atomic load more.  When on,
// every kernel launch of the library is bracketed by a HIP event pair recorded
// on the stream the kernel is launched on, and attributed to the kernel
// instance and to the tag the caller set last.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <cstdlib>
#include <cstring>
#include <cxxabi.h>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tsm2x.h"
#include "tsm2x_internal.h"

namespace {

struct Rec {
    const void* fn;
    int tag;
    hipStream_t st;
    hipEvent_t e0, e1;
    bool closed;             // end event recorded
};

struct Row {
    std::string name;
    int tag;
    int64_t launches;
    double total_ms;
};

std::mutex g_mu;
std::atomic<bool> g_on{false};
std::atomic<int> g_tag{0};
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::vector<Row> g_rows;
std::map<const void*, std::string> g_names;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// "tsm2l_bwd_kernel<double, 1, 1, 2, true, -1, false>": the demangled name
// without return type, namespace and parameter list
std::string kernel_name(const void* fn, hipStream_t st) {
    auto it = g_names.find(fn);
    if (it != g_names.end()) return it->second;
    const char* raw = hipKernelNameRefByPtr(fn, st);
    std::string name;
    if (raw) {
        int status = 0;
        char* dem = abi::__cxa_demangle(raw, nullptr, nullptr, &status);
        name = (status == 0 && dem) ? dem : raw;
        std::free(dem);
        if (name.compare(0, 5, "void ") == 0) name.erase(0, 5);
        // the kernels' namespace is left out, as tsm2x_kernel_name reports them
        if (name.compare(0, 5, "tsm::") == 0) name.erase(0, 5);
        int depth = 0;
        for (size_t i = 0; i < name.size(); ++i) {
            if (name[i] == '<') ++depth;
            else if (name[i] == '>') --depth;
            else if (name[i] == '(' && depth == 0) { name.resize(i); break; }
        }
    } else {
        char buf[40];
        std::snprintf(buf, sizeof buf, "kernel@%p", fn);
        name = buf;
    }
    g_names[fn] = name;
    return name;
}

void release_records() {
    for (Rec& r : g_recs) {
        g_pool.push_back(r.e0);
        g_pool.push_back(r.e1);
    }
    g_recs.clear();
}

}  // namespace

namespace tsm {

LaunchTimer::LaunchTimer(const void* fn, hipStream_t s) : slot(-1), st(s) {
    if (!g_on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b || hipEventRecord(a, s) != hipSuccess) {
        if (a) g_pool.push_back(a);
        if (b) g_pool.push_back(b);
        return;
    }
    g_recs.push_back(Rec{fn, g_tag.load(), s, a, b, false});
    slot = (int)g_recs.size() - 1;
}

LaunchTimer::~LaunchTimer() {
    if (slot < 0) return;
    // a failed launch leaves its error for the caller's check: record nothing
    // more (a successful event record would clear it)
    if (hipPeekAtLastError() != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (slot < (int)g_recs.size() && hipEventRecord(g_recs[slot].e1, st) == hipSuccess)
        g_recs[slot].closed = true;
}

}  // namespace tsm

extern "C" {

int tsm2x_timing_start(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    release_records();
    g_rows.clear();
    g_on.store(true);
    return TSM_SUCCESS;
}

int tsm2x_timing_stop(void) {
    g_on.store(false);
    return TSM_SUCCESS;
}

int tsm2x_timing_tag(int tag) {
    g_tag.store(tag);
    return TSM_SUCCESS;
}

int tsm2x_timing_collect(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    std::map<std::pair<std::string, int>, size_t> at;
    for (size_t i = 0; i < g_rows.size(); ++i) at[{g_rows[i].name, g_rows[i].tag}] = i;
    for (const Rec& r : g_recs) {
        if (!r.closed) continue;
        if (hipEventSynchronize(r.e1) != hipSuccess) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) continue;
        const std::pair<std::string, int> key(kernel_name(r.fn, r.st), r.tag);
        auto it = at.find(key);
        if (it == at.end()) {
            at[key] = g_rows.size();
            g_rows.push_back(Row{key.first, r.tag, 1, (double)ms});
        } else {
            g_rows[it->second].launches += 1;
            g_rows[it->second].total_ms += ms;
        }
    }
    release_records();
    return (int)g_rows.size();
}

int tsm2x_timing_row(int i, const char** kernel, int* tag, int64_t* launches,
                     double* total_ms) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (i < 0 || i >= (int)g_rows.size()) return -1;
    if (kernel) *kernel = g_rows[i].name.c_str();
    if (tag) *tag = g_rows[i].tag;
    if (launches) *launches = g_rows[i].launches;
    if (total_ms) *total_ms = g_rows[i].total_ms;
    return TSM_SUCCESS;
}

}  // extern "C"
