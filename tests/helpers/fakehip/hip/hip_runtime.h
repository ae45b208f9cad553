// Host-only stand-in for the HIP runtime API the request server uses, so the
// server's engine (threads, admission, rounds in flight, completion) runs on
// the CPU in tests.  Device memory is host memory with a byte budget.  Each
// stream is a queue executed in order by a thread of its own: copies read
// their source when they execute, kernels run when their turn comes, events
// complete when the stream reaches them and carry that time, frees return
// memory when they execute.  So the engine meets the same asynchrony as on a
// device (a staging buffer rewritten too early, or a missing wait, changes
// what a test sees).  A kernel launch binds the launch's argument values at
// once (through the registered binder) and queues the bound call.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <thread>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorNotReady = 600, hipErrorLaunchFailure = 719 };
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 };
#define hipStreamNonBlocking 1
#define hipEventDisableTiming 2
#define hipHostMallocDefault 0
struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct hipDeviceProp_t {
    int multiProcessorCount;
    int clockRate;
    size_t sharedMemPerBlock;
    char name[256];
    char gcnArchName[256];
};
inline const char *hipGetErrorString(hipError_t e) { return e ? "fake HIP error" : "no error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }

// Device variables are host memory here; the symbol's address is the
// variable's own.
#define __device__
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) {
    *p = const_cast<void *>(sym);
    return hipSuccess;
}

// What the library under test did: host waits for a stream or an event,
// device allocations, pinned host allocations.
inline std::atomic<long> fake_host_waits{0};
inline std::atomic<long> fake_device_allocs{0};
inline std::atomic<long> fake_pinned_allocs{0};

struct ihipStream_t {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::function<void()>> q;
    bool stop = false;
    std::thread th;
    ihipStream_t() : th([this] { run(); }) {}
    ~ihipStream_t() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv.notify_all();
        th.join();
    }
    void push(std::function<void()> f) {
        {
            std::lock_guard<std::mutex> lk(mu);
            q.push_back(std::move(f));
        }
        cv.notify_all();
    }
    void run() {
        for (;;) {
            std::function<void()> f;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || !q.empty(); });
                if (q.empty()) return;
                f = std::move(q.front());
                q.pop_front();
            }
            f();
        }
    }
};
typedef ihipStream_t *hipStream_t;

struct ihipEvent_t {
    std::mutex mu;
    std::condition_variable cv;
    uint64_t recorded = 0, reached = 0;
    double t_ms = 0.0;
};
typedef ihipEvent_t *hipEvent_t;

// test controls (defined in the harness)
extern std::atomic<long> fake_alloc_budget;     // bytes the fake device may still allocate
extern std::atomic<int> fake_fail_launches;     // launches left to fail
typedef std::function<void()> (*fake_kernel_binder)(void **args);
extern fake_kernel_binder fake_bind_serve_kernel;

inline double fake_now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) {
    p->multiProcessorCount = 4;
    return hipSuccess;
}
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, const void *, int, size_t) {
    *n = 2;
    return hipSuccess;
}
inline hipError_t fake_alloc(void **p, size_t bytes) {
    fake_device_allocs.fetch_add(1);
    if (fake_alloc_budget.fetch_sub((long)bytes) < (long)bytes) {
        fake_alloc_budget.fetch_add((long)bytes);
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    *p = calloc(1, bytes + 16);
    ((size_t *)*p)[0] = bytes;
    *p = (char *)*p + 16;
    return hipSuccess;
}
inline void fake_free(void *p) {
    if (!p) return;
    char *b = (char *)p - 16;
    fake_alloc_budget.fetch_add((long)((size_t *)b)[0]);
    free(b);
}
inline hipError_t hipMalloc(void **p, size_t b) { return fake_alloc(p, b); }
inline hipError_t hipMallocAsync(void **p, size_t b, hipStream_t) { return fake_alloc(p, b); }
inline hipError_t hipFree(void *p) { fake_free(p); return hipSuccess; }
inline hipError_t hipFreeAsync(void *p, hipStream_t s) {
    s->push([p] { fake_free(p); });
    return hipSuccess;
}
// Pinned blocks by start address, so that a copy reading past the end of
// one is counted (fake_pinned_overruns).
inline std::mutex fake_pinned_mu;
inline std::map<const char *, size_t> fake_pinned_blocks;
inline std::atomic<long> fake_pinned_overruns{0};
inline hipError_t hipHostMalloc(void **p, size_t b, unsigned) {
    fake_pinned_allocs.fetch_add(1);
    *p = calloc(1, b);
    std::lock_guard<std::mutex> g(fake_pinned_mu);
    fake_pinned_blocks[(const char *)*p] = b;
    return hipSuccess;
}
inline hipError_t hipHostFree(void *p) {
    {
        std::lock_guard<std::mutex> g(fake_pinned_mu);
        fake_pinned_blocks.erase((const char *)p);
    }
    free(p);
    return hipSuccess;
}
inline void fake_check_pinned(const void *s, size_t n) {
    std::lock_guard<std::mutex> g(fake_pinned_mu);
    auto it = fake_pinned_blocks.upper_bound((const char *)s);
    if (it == fake_pinned_blocks.begin()) return;
    --it;
    const char *c = (const char *)s;
    if (c < it->first + it->second && c + n > it->first + it->second) fake_pinned_overruns.fetch_add(1);
}
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t st) {
    fake_check_pinned(s, n);
    fake_check_pinned(d, n);
    st->push([d, s, n] { memcpy(d, s, n); });
    return hipSuccess;
}
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
    memcpy(d, s, n);   // the null stream does not wait for non-blocking streams
    return hipSuccess;
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = new ihipStream_t();
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = new ihipEvent_t(); return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    uint64_t gen;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        gen = ++e->recorded;
    }
    s->push([e, gen] {
        // notify under the lock: a waiter may destroy the event once it sees it
        std::lock_guard<std::mutex> lk(e->mu);
        if (gen > e->reached) {
            e->reached = gen;
            e->t_ms = fake_now_ms();
        }
        e->cv.notify_all();
    });
    return hipSuccess;
}
inline hipError_t hipEventQuery(hipEvent_t e) {
    std::lock_guard<std::mutex> lk(e->mu);
    return e->reached >= e->recorded ? hipSuccess : hipErrorNotReady;
}
inline hipError_t hipEventSynchronize(hipEvent_t e) {
    fake_host_waits.fetch_add(1);
    std::unique_lock<std::mutex> lk(e->mu);
    const uint64_t want = e->recorded;
    e->cv.wait(lk, [&] { return e->reached >= want; });
    return hipSuccess;
}
// The stream waits, at this point of its queue, for the event's latest
// recording as of this call.
inline hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    uint64_t want;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        want = e->recorded;
    }
    s->push([e, want] {
        std::unique_lock<std::mutex> lk(e->mu);
        e->cv.wait(lk, [&] { return e->reached >= want; });
    });
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t s) {
    ihipEvent_t e;
    hipEventRecord(&e, s);
    return hipEventSynchronize(&e);   // counted there
}
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> la(a->mu);
    std::lock_guard<std::mutex> lb(b->mu);
    *ms = (float)(b->t_ms - a->t_ms);
    return hipSuccess;
}
inline hipError_t hipLaunchKernel(const void *, dim3, dim3, void **args, size_t, hipStream_t s) {
    if (fake_fail_launches.load() > 0) {
        fake_fail_launches.fetch_sub(1);
        return hipErrorLaunchFailure;
    }
    s->push(fake_bind_serve_kernel(args));
    return hipSuccess;
}
