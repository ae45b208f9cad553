// Serving kernel: one persistent launch traces a round of work for many
// resident requests at once.  Each wave claims one chunk of the round's work
// list at a time, reads that request's parameter block (wave-uniform scalar
// loads) and runs the persistent ray loop over the chunk's rays with the
// request's crystal, mosaic and rocking-curve kinds chosen at run time.
// Images and counters go to the request's own buffers, so every request's
// result is the one a separate mrt_trace call of the same rays would give.
#include "trace_impl.h"

namespace mrt {
namespace tk {

// The rays of one chunk, handed out once.
struct OneChunk {
    uint64_t first, end;
    bool used;
    __device__ __forceinline__ bool operator()(uint64_t &next, uint64_t &e) {
        if (used) return false;
        used = true;
        next = first;
        e = end;
        return true;
    }
};

template <class R>
__global__ void __launch_bounds__(256)
    serve_kernel(const TraceParams *__restrict__ slots, const ServeChunk *__restrict__ chunks,
                 uint32_t n_chunks, unsigned int *__restrict__ cursor) {
    using T = Tracer<R, kAny, kAny, kAny, false>;
    for (;;) {
        // Every lane takes part in the claim (lane 0 adds one, the others
        // zero) so that no lane-conditional block sits at the loop head: the
        // final counter flush of trace_loop is lane-0-only, and a claim
        // guarded by the same lane test right after the back-edge lets the
        // compiler thread the two branches and run lanes 1..63 round the loop
        // without lane 0, reading a stale chunk index forever.
        const unsigned int c = uniform(atomicAdd(cursor, __lane_id() == 0 ? 1u : 0u));
        if (c >= n_chunks) return;
        const ServeChunk ch = chunks[c];
        const TraceParams &P = slots[ch.slot];
        OneChunk claim{ch.first, ch.first + ch.count, false};
        trace_loop<T>(P, P.lut, P.bin_cdf, claim);
    }
}

}  // namespace tk

const void *serve_kernel_ptr(int precision) {
    return precision == MRT_FP64 ? (const void *)tk::serve_kernel<double>
                                 : (const void *)tk::serve_kernel<float>;
}

}  // namespace mrt
