// The request server's host engine (paper_2503_16955_amd/csrc/server.cpp) on
// the CPU, against the fake HIP layer in fakehip/ (streams run on threads of
// their own): the serving "kernel" walks
// the round's items (one ray range per request) and, for every ray id,
// adds a deterministic hash of (seed, ray id) to the request's images and
// counters, so a test can recompute each request's expected result.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdarg>
#include <thread>
#include <cstdio>
#include <string>

#include "params.h"
#include "trace_params.h"

std::atomic<long> fake_alloc_budget{1L << 40};
std::atomic<int> fake_fail_launches{0};
fake_kernel_binder fake_bind_serve_kernel = nullptr;
std::atomic<int> g_gate{1};          // launches wait while 0
std::atomic<long> g_launches{0};

namespace {
thread_local std::string g_err;

uint64_t mix64(uint64_t x) {   // splitmix64 finaliser
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

// The serving kernel's work for one round (runs on the stream's thread).
void serve(const mrt::TraceParams *slots, const mrt::ServeItem *items, uint32_t n, uint64_t total) {
    g_launches.fetch_add(1);
    while (!g_gate.load()) std::this_thread::sleep_for(std::chrono::milliseconds(1));
    uint64_t start = 0;
    for (uint32_t c = 0; c < n; ++c) {
        const mrt::ServeItem &it = items[c];
        if (it.start != start || it.chunk < 64 || it.chunk % 64) abort();   // malformed round
        start += it.count;
        const mrt::TraceParams &P = slots[it.slot];
        const uint64_t px = (uint64_t)P.nx * (uint64_t)P.ny;
        for (uint64_t id = it.first; id < it.first + it.count; ++id) {
            const uint64_t h = mix64(P.seed * 0x9E3779B97F4A7C15ull + id);
            // atomics, as on the device: rounds in flight run concurrently
            __atomic_fetch_add(&P.counts[h % px], 1u, __ATOMIC_RELAXED);
            __atomic_fetch_add(&P.energy[h % px], (unsigned long long)id, __ATOMIC_RELAXED);
            __atomic_fetch_add(&P.dev_counters[mrt::kCMissed], (unsigned long long)((h >> 60) & 1),
                               __ATOMIC_RELAXED);
            __atomic_fetch_add(&P.dev_counters[mrt::kCEvents], (unsigned long long)(1 + ((h >> 50) & 3)),
                               __ATOMIC_RELAXED);
            __atomic_fetch_add(&P.dev_counters[mrt::kCDetected], 1ull, __ATOMIC_RELAXED);
        }
    }
    if (start != total) abort();
}

// Bind a launch's argument values (the args point to the caller's locals).
std::function<void()> bind_serve(void **args) {
    const mrt::TraceParams *slots = *(const mrt::TraceParams **)args[0];
    const mrt::ServeItem *items = *(const mrt::ServeItem **)args[1];
    const uint32_t n = *(const uint32_t *)args[2];
    const uint64_t total = *(const uint64_t *)args[3];
    return [=] { serve(slots, items, n, total); };
}
}  // namespace

namespace mrt {
mrt_status fail(mrt_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}
const char *last_error() { return g_err.c_str(); }
void clear_error() { g_err.clear(); }
int launch_zero(void *p, size_t words, void *stream) {
    ((hipStream_t)stream)->push([p, words] { memset(p, 0, words * 4); });
    return 0;
}
const void *serve_kernel_ptr(int, bool) { return (const void *)&serve; }
}  // namespace mrt

extern "C" {
void harness_init(long device_bytes, int fail_launches) {
    fake_bind_serve_kernel = bind_serve;
    fake_alloc_budget = device_bytes;
    fake_fail_launches = fail_launches;
    g_gate = 1;
    g_launches = 0;
}
long harness_free_bytes() { return fake_alloc_budget.load(); }
void harness_gate(int open) { g_gate = open; }
long harness_launches() { return g_launches.load(); }
const char *harness_last_error() { return g_err.c_str(); }
long harness_pinned_overruns() { return fake_pinned_overruns.load(); }
}
