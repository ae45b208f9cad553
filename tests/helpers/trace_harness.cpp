// The one-call host runtime (paper_2503_16955_amd/csrc/runtime.cpp, through
// its C-ABI) on the CPU against the fake HIP layer in fakehip/ (streams run on
// threads of their own, device memory is host memory).  The trace "kernel"
// copies what it finds in the tables the parameter block points at, so a
// test can check that each call's kernel read that call's tables, whatever
// the caller did to its own arrays after the call returned; a stream can be
// held shut to show that a call returns without waiting for it.
#include <hip/hip_runtime.h>

#include <vector>

#include "params.h"
#include "trace_params.h"

std::atomic<long> fake_alloc_budget{1L << 40};
std::atomic<int> fake_fail_launches{0};
fake_kernel_binder fake_bind_serve_kernel = nullptr;

namespace {
std::mutex g_mu;
std::vector<std::vector<double>> g_seen;   // per kernel run: lut values, then the CDF
std::atomic<int> g_gate{1};
char g_kernel_tag;                         // the address every "kernel" pointer takes

void run_trace(const mrt::TraceParams P) {
    std::vector<double> t;
    if (P.lut) t.insert(t.end(), P.lut, P.lut + P.lut_n);
    if (P.bin_cdf) t.insert(t.end(), P.bin_cdf, P.bin_cdf + P.n_bins + 1);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_seen.push_back(t);
    }
    // counters the caller can read back: the ray count and the table size
    __atomic_fetch_add(&P.dev_counters[mrt::kCEvents], (unsigned long long)P.n, __ATOMIC_RELAXED);
    __atomic_fetch_add(&P.dev_counters[mrt::kCDetected], (unsigned long long)t.size(), __ATOMIC_RELAXED);
}

std::function<void()> bind_trace(void **args) {
    const mrt::TraceParams P = *(const mrt::TraceParams *)args[0];
    return [P] { run_trace(P); };
}
}  // namespace

namespace mrt {
const void *trace_kernel_ptr(int, int, int, int, bool) { return &g_kernel_tag; }
const void *ext_kernel_ptr(int, int, int, int, bool) { return &g_kernel_tag; }
const void *mwg_kernel_ptr(int, bool, bool, bool) { return &g_kernel_tag; }
int launch_zero(void *p, size_t words, void *stream) {
    ((hipStream_t)stream)->push([p, words] { memset(p, 0, words * 4); });
    return 0;
}
int launch_calibration_map(const uint32_t *, const uint64_t *, size_t, double *, void *) { return 0; }
}  // namespace mrt

extern "C" {
void harness_init() {
    fake_bind_serve_kernel = bind_trace;
    std::lock_guard<std::mutex> lk(g_mu);
    g_seen.clear();
}
void *harness_stream() {
    hipStream_t s = nullptr;
    hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    return s;
}
// Hold the stream shut at this point of its queue until harness_open().
void harness_hold(void *stream) {
    g_gate = 0;
    ((hipStream_t)stream)->push([] {
        while (!g_gate.load()) std::this_thread::sleep_for(std::chrono::milliseconds(1));
    });
}
void harness_open() { g_gate = 1; }
void harness_sync(void *stream) { hipStreamSynchronize((hipStream_t)stream); }
// host waits, device allocations, pinned host allocations so far
void harness_counts(long *waits, long *dev_allocs, long *pinned) {
    *waits = fake_host_waits.load();
    *dev_allocs = fake_device_allocs.load();
    *pinned = fake_pinned_allocs.load();
}
int harness_runs() {
    std::lock_guard<std::mutex> lk(g_mu);
    return (int)g_seen.size();
}
// Tables kernel run `i` read; returns how many values (at most cap copied).
int harness_seen(int i, double *out, int cap) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (i < 0 || i >= (int)g_seen.size()) return -1;
    const std::vector<double> &t = g_seen[(size_t)i];
    for (size_t k = 0; k < t.size() && (int)k < cap; ++k) out[k] = t[k];
    return (int)t.size();
}
}
