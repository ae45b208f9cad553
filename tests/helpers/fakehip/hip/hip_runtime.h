// Host-only stand-in for the HIP runtime API the request server uses, so the
// server's engine (threads, admission, rounds, completion) runs on the CPU in
// tests.  Device memory is host memory; every stream operation executes at
// once in the calling thread; a kernel launch calls the registered host
// function with the launch's arguments.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorLaunchFailure = 719 };
typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2 };
#define hipStreamNonBlocking 1
struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct hipDeviceProp_t {
    int multiProcessorCount;
};

// test controls (defined in the harness)
extern std::atomic<long> fake_alloc_budget;     // bytes the fake device may still allocate
extern std::atomic<int> fake_fail_launches;     // launches left to fail
typedef void (*fake_kernel_fn)(void **args);
extern fake_kernel_fn fake_serve_kernel;

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
inline hipError_t fake_free(void *p) {
    if (!p) return hipSuccess;
    char *b = (char *)p - 16;
    fake_alloc_budget.fetch_add((long)((size_t *)b)[0]);
    free(b);
    return hipSuccess;
}
inline hipError_t hipMalloc(void **p, size_t b) { return fake_alloc(p, b); }
inline hipError_t hipMallocAsync(void **p, size_t b, hipStream_t) { return fake_alloc(p, b); }
inline hipError_t hipFree(void *p) { return fake_free(p); }
inline hipError_t hipFreeAsync(void *p, hipStream_t) { return fake_free(p); }
inline hipError_t hipHostMalloc(void **p, size_t b, unsigned) { *p = calloc(1, b); return hipSuccess; }
inline hipError_t hipHostFree(void *p) { free(p); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) {
    memcpy(d, s, n);
    return hipSuccess;
}
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
    memcpy(d, s, n);
    return hipSuccess;
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = (hipStream_t)malloc(8);
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) { free(s); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = (hipEvent_t)malloc(8); return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { free(e); return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 1.0f; return hipSuccess; }
inline hipError_t hipLaunchKernel(const void *, dim3, dim3, void **args, size_t, hipStream_t) {
    if (fake_fail_launches.load() > 0) {
        fake_fail_launches.fetch_sub(1);
        return hipErrorLaunchFailure;
    }
    fake_serve_kernel(args);
    return hipSuccess;
}
