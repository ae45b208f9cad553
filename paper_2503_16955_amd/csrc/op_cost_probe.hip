// Single-operation probe kernels.  Each applies one operation, exactly as the
// trace kernels evaluate it (the same device functions and flags), inside a
// loop of runtime length, the way the event loop runs it: loop-invariant
// constants are then hoisted out, as they are in the trace kernel.  The
// number of VALU instructions in the loop body of its gfx950 code, minus that
// of the glue-only loop of the same shape, is the instruction cost of the
// operation.  Used to price the per-event operation mix for the ALU
// roofline; never linked into the library.
#include <hip/hip_runtime.h>
#include <math.h>

#include "device_math.h"
#include "trace_impl.h"

using namespace mrt;

// x <- op(x), n times; the result depends on every iteration.
#define PROBE(name, T, expr)                                                              \
    extern "C" __global__ void probe_##name(const T *__restrict__ a, T *__restrict__ o, int n) { \
        const int i = threadIdx.x;                                                        \
        T x = a[i];                                                                       \
        for (int j = 0; j < n; ++j) x = (expr);                                           \
        o[i] = x;                                                                         \
    }

PROBE(glue_f64, double, x * 0.5)
PROBE(log_f64, double, dm::log_pos(x) * 0.5)
PROBE(exp_f64, double, dm::exp_nonpos(-x) * 0.5)
PROBE(expm1_f64, double, ::expm1(x) * 0.5)
PROBE(sqrt_f64, double, dm::sqrt(x) * 0.5)
PROBE(rsqrt_f64, double, dm::rsqrt(x) * 0.5)
PROBE(rcp_f64, double, dm::rcp(x) * 0.5)
PROBE(div_ieee_f64, double, (1.0 / x) * 0.5)
PROBE(sin_f64, double, ::sin(x) * 0.5)
PROBE(cos_f64, double, ::cos(x) * 0.5)
PROBE(asin_f64, double, ::asin(x) * 0.5)
PROBE(glue_f32, float, x * 0.5f)
PROBE(log_f32, float, dm::log_pos(x) * 0.5f)
PROBE(exp_f32, float, dm::exp_(x) * 0.5f)
PROBE(expm1_f32, float, ::expm1f(x) * 0.5f)
PROBE(sqrt_f32, float, dm::sqrt(x) * 0.5f)
PROBE(rsqrt_f32, float, dm::rsqrt(x) * 0.5f)
PROBE(rcp_f32, float, dm::rcp(x) * 0.5f)
PROBE(div_ieee_f32, float, (1.0f / x) * 0.5f)

__device__ __forceinline__ double sc64(double x) {
    double s, c;
    dm::sincos_turns(x, &s, &c);
    return s * c;
}
__device__ __forceinline__ float sc32(float x) {
    float s, c;
    dm::sincos_turns(x, &s, &c);
    return s * c;
}
PROBE(sincos_f64, double, sc64(x))
PROBE(glue2_f64, double, x * x)
PROBE(sincos_f32, float, sc32(x))
PROBE(glue2_f32, float, x * x)

// Philox4x32-10 with a wave-uniform key, as the trace kernel draws it.
extern "C" __global__ void probe_philox(const unsigned *__restrict__ a, unsigned *__restrict__ o,
                                        unsigned k0, unsigned k1, int n) {
    const int i = threadIdx.x;
    unsigned c0 = a[i], c1 = a[i + 64], c2 = a[i + 128], c3 = a[i + 192];
    for (int j = 0; j < n; ++j) {
        const dm::Words w = dm::philox(k0, k1, c0, c1, c2, c3);
        c0 = w.w0; c1 = w.w1; c2 = w.w2; c3 = w.w3;
    }
    o[i] = c0; o[i + 64] = c1; o[i + 128] = c2; o[i + 192] = c3;
}
extern "C" __global__ void probe_glue_u32(const unsigned *__restrict__ a, unsigned *__restrict__ o,
                                          unsigned k0, unsigned k1, int n) {
    const int i = threadIdx.x;
    unsigned c0 = a[i], c1 = a[i + 64], c2 = a[i + 128], c3 = a[i + 192];
    for (int j = 0; j < n; ++j) {
        const unsigned t = c0;
        c0 = c1; c1 = c2; c2 = c3; c3 = t;
    }
    o[i] = c0; o[i + 64] = c1; o[i + 128] = c2; o[i + 192] = c3;
}

// Acceptance filter of the trace kernel (fast path), per rocking-curve kind:
// the decision feeds back into the next argument.
#define FILTER_PROBE(name, IRC)                                                                \
    extern "C" __global__ void probe_##name(const TraceParams P, const double *__restrict__ a,   \
                                            double *__restrict__ o, int n) {                   \
        const int i = threadIdx.x;                                                             \
        double x = a[i];                                                                       \
        const float sa = (float)a[i + 64], ca = (float)a[i + 128], u = (float)a[i + 192];      \
        for (int j = 0; j < n; ++j)                                                            \
            x = x * 0.5 + (double)tk::Tracer<double, MRT_GEOMETRY_CYLINDER,                    \
                                             MRT_MOSAIC_PSEUDO_VOIGT, IRC, false>::filter(     \
                              P, x, sa, ca, u, P.f32.shift, 1.0f);                            \
        o[i] = x;                                                                              \
    }
FILTER_PROBE(filter_gaussian, MRT_IRC_GAUSSIAN)
FILTER_PROBE(filter_pseudo_voigt, MRT_IRC_PSEUDO_VOIGT)
FILTER_PROBE(filter_table, MRT_IRC_TABLE)
// The table curve's decision as priced: the FP32 estimate of x and the
// test against the table's range.  The envelope bounds the filter adds
// only spare most of the exact evaluations inside the range, which are
// not priced either.
extern "C" __global__ void probe_filter_table_range(const TraceParams P, const double *__restrict__ a,
                                                    double *__restrict__ o, int n) {
    const int i = threadIdx.x;
    double x = a[i];
    const float sa = (float)a[i + 64], ca = (float)a[i + 128];
    using T = tk::Tracer<double, MRT_GEOMETRY_CYLINDER, MRT_MOSAIC_PSEUDO_VOIGT, MRT_IRC_TABLE, false>;
    for (int j = 0; j < n; ++j) {
        float lo, hi, slo, shi;
        const bool b = T::x_bounds(x, sa, ca, P.f32.shift, 1.0f, lo, hi, slo, shi);
        x = x * 0.5 + (double)(b ? (T::outside_table(P, slo, shi) ? 0 : -1) : -1);
    }
    o[i] = x;
}
FILTER_PROBE(filter_lorentzian, MRT_IRC_LORENTZIAN)
FILTER_PROBE(filter_box, MRT_IRC_BOX)
extern "C" __global__ void probe_glue_filter(const TraceParams P, const double *__restrict__ a,
                                             double *__restrict__ o, int n) {
    const int i = threadIdx.x;
    double x = a[i];
    const float sa = (float)a[i + 64], ca = (float)a[i + 128], u = (float)a[i + 192];
    for (int j = 0; j < n; ++j) x = x * 0.5 + (double)(int)(sa + ca + u);
    o[i] = x;
}
