// Serving kernels: one persistent launch traces a round of work for many
// resident requests at once (the loop itself is serve_waves in
// trace_impl.h); each request's rays run the loop specialised for its
// crystal, mosaic and rocking-curve kinds, chosen per item from its
// parameter block (wave-uniform scalar loads).  The extended serving kernel
// reads the kinds at run time.
// Images and counters go to the request's own buffers, so every request's
// result is the one a separate mrt_trace call of the same rays would give.
// Instantiated per precision in serve_f64.hip and serve_f32.hip.
#pragma once
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
    serve_waves(slots, items, n_items, total, cursors, blockIdx.x * waves_per_block + w,
                gridDim.x * waves_per_block, KindRun<R, false, RayQueue<R, false>>{queues[w]});
}

// The same loop with the extended inputs (user polarisations,
// energy-dependent curves, further planes), with the kinds read at run time,
// for rounds that hold a request using them.
template <class R>
__global__ void __launch_bounds__(256)
    serve_kernel_ext(const TraceParams *__restrict__ slots, const ServeItem *__restrict__ items,
                     uint32_t n_items, uint64_t total, unsigned long long *__restrict__ cursors) {
    using T = Tracer<R, kAny, kAny, kAny, false, true>;
    const uint32_t waves_per_block = blockDim.x >> 6;
    const uint32_t w = uniform(threadIdx.x >> 6);
    __shared__ typename T::Queue queues[4];   // one ray queue per wave
    serve_waves(slots, items, n_items, total, cursors, blockIdx.x * waves_per_block + w,
                gridDim.x * waves_per_block, LoopRun<T, false, typename T::Queue>{queues[w]});
}

}  // namespace tk

}  // namespace mrt
