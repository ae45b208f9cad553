// Serving kernel: one persistent launch traces a round of work for many
// resident requests at once (the loop itself is serve_waves in
// trace_impl.h), with each request's crystal, mosaic and rocking-curve kinds
// chosen at run time from its parameter block (wave-uniform scalar loads).
// Images and counters go to the request's own buffers, so every request's
// result is the one a separate mrt_trace call of the same rays would give.
#include "trace_impl.h"

namespace mrt {
namespace tk {

template <class R>
__global__ void __launch_bounds__(256)
    serve_kernel(const TraceParams *__restrict__ slots, const ServeItem *__restrict__ items,
                 uint32_t n_items, uint64_t total, unsigned long long *__restrict__ cursors) {
    const uint32_t waves_per_block = blockDim.x >> 6;
    const uint32_t w = uniform(threadIdx.x >> 6);
    __shared__ RayQueue<R, false> queues[4];   // one ray queue per wave
    serve_waves<Tracer<R, kAny, kAny, kAny, false>>(slots, items, n_items, total, cursors,
                                                    blockIdx.x * waves_per_block + w,
                                                    gridDim.x * waves_per_block, queues[w]);
}

// The same loop with the extended inputs (source spots, user ray arrays and
// polarisations, energy-dependent curves, further planes), for rounds that
// hold a request using them.
template <class R>
__global__ void __launch_bounds__(256)
    serve_kernel_ext(const TraceParams *__restrict__ slots, const ServeItem *__restrict__ items,
                     uint32_t n_items, uint64_t total, unsigned long long *__restrict__ cursors) {
    using T = Tracer<R, kAny, kAny, kAny, false, true>;
    const uint32_t waves_per_block = blockDim.x >> 6;
    const uint32_t w = uniform(threadIdx.x >> 6);
    __shared__ typename T::Queue queues[4];   // one ray queue per wave
    serve_waves<T>(slots, items, n_items, total, cursors, blockIdx.x * waves_per_block + w,
                   gridDim.x * waves_per_block, queues[w]);
}

}  // namespace tk

const void *serve_kernel_ptr(int precision, bool ext) {
    if (ext)
        return precision == MRT_FP64 ? (const void *)tk::serve_kernel_ext<double>
                                     : (const void *)tk::serve_kernel_ext<float>;
    return precision == MRT_FP64 ? (const void *)tk::serve_kernel<double>
                                 : (const void *)tk::serve_kernel<float>;
}

}  // namespace mrt
