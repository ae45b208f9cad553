// Single-operation probe kernels.  Each reads one operand per lane, applies
// one operation and stores the result; the number of VALU instructions in
// its gfx950 code, minus that of the plain copy kernel of the same type, is
// the instruction cost of the operation as the trace kernels compile it
// (same flags).  Used to convert the per-event operation mix into VALU
// lane-operations for the ALU roofline; never linked into the library.
#include <hip/hip_runtime.h>
#include <math.h>

#define PROBE(name, T, expr)                                                            \
    extern "C" __global__ void probe_##name(const T *__restrict__ a, T *__restrict__ o) { \
        const int i = threadIdx.x;                                                      \
        const T x = a[i];                                                               \
        o[i] = (expr);                                                                  \
    }

PROBE(copy_f64, double, x)
PROBE(log_f64, double, log(x))
PROBE(exp_f64, double, exp(x))
PROBE(asin_f64, double, asin(x))
PROBE(sqrt_f64, double, sqrt(x))
PROBE(rcp_f64, double, 1.0 / x)
PROBE(expm1_f64, double, expm1(x))
PROBE(copy_f32, float, x)
PROBE(log_f32, float, __logf(x))
PROBE(exp_f32, float, __expf(x))
PROBE(sqrt_f32, float, __fsqrt_rn(x))
PROBE(rcp_f32, float, 1.0f / x)
PROBE(expm1_f32, float, expm1f(x))

extern "C" __global__ void probe_sincos_f64(const double *__restrict__ a, double *__restrict__ o) {
    const int i = threadIdx.x;
    double s, c;
    sincos(a[i], &s, &c);
    o[i] = s;
    o[i + 64] = c;
}
extern "C" __global__ void probe_sincos_f32(const float *__restrict__ a, float *__restrict__ o) {
    const int i = threadIdx.x;
    float s, c;
    __sincosf(a[i], &s, &c);
    o[i] = s;
    o[i + 64] = c;
}
extern "C" __global__ void probe_copy2_f64(const double *__restrict__ a, double *__restrict__ o) {
    const int i = threadIdx.x;
    o[i] = a[i];
    o[i + 64] = a[i];
}
extern "C" __global__ void probe_copy2_f32(const float *__restrict__ a, float *__restrict__ o) {
    const int i = threadIdx.x;
    o[i] = a[i];
    o[i + 64] = a[i];
}

// Philox4x32-10 with the round keys in memory, as the trace kernel has them.
extern "C" __global__ void probe_philox(const unsigned *__restrict__ a, unsigned *__restrict__ o,
                                        const unsigned *__restrict__ key) {
    const int i = threadIdx.x;
    unsigned c0 = a[i], c1 = a[i + 64], c2 = a[i + 128], c3 = a[i + 192];
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const unsigned lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const unsigned n0 = hi1 ^ c1 ^ key[r], n2 = hi0 ^ c3 ^ key[10 + r];
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    o[i] = c0; o[i + 64] = c1; o[i + 128] = c2; o[i + 192] = c3;
}
extern "C" __global__ void probe_copy4_u32(const unsigned *__restrict__ a, unsigned *__restrict__ o,
                                           const unsigned *__restrict__ key) {
    const int i = threadIdx.x;
    o[i] = a[i]; o[i + 64] = a[i + 64]; o[i + 128] = a[i + 128]; o[i + 192] = a[i + 192];
}
