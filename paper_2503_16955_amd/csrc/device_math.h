// Device arithmetic of the trace kernels (gfx950).
//
// Philox4x32-10 and the uniform maps, plus the FP64 elementary functions the
// per-event path needs, written for the arguments that path produces
// (positive normal logarithm arguments, angles given in turns) instead of
// the general-purpose library versions.  Each is
// accurate to one or two units in the last place; the accuracy is checked
// against the host C library by the parity tests of the whole path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrt {
namespace dm {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11).  Each round forms the
// two 32x32 -> 64-bit products of words 0 and 2 (one v_mad_u64_u32 each),
// xors their high halves with words 3 and 1 and the round key, and permutes;
// the key advances by the Weyl constants.  The key stays wave-uniform, so
// its schedule runs on the scalar unit.
// ---------------------------------------------------------------------------
struct Words {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                        uint32_t c2, uint32_t c3) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words{c0, c1, c2, c3};
}

// Uniforms in the open interval (0, 1).
__device__ __forceinline__ double u01_f64(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }
// 23 random bits, exact in float: ((w >> 9) + 1/2) 2^-23.
__device__ __forceinline__ float u01_f32(uint32_t w) {
    return (float)(((w >> 9) << 1) | 1u) * 0x1p-24f;
}

// Polynomial step p z + c as the three-operand v_fma_f64 with the constant
// coefficient c in scalar registers (built by the scalar unit next to its
// use).  The compiler otherwise materialises 64-bit coefficients with two
// VALU moves each and uses the two-address v_fmac_f64, which overwrites its
// addend and so needs a further copy at every use.  c must be wave-uniform.
__device__ __forceinline__ double poly_step(double p, double z, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(z), "s"(c));
    return r;
}

// ---------------------------------------------------------------------------
// FP64 reciprocal, quotient, square root and reciprocal square root from the
// hardware seeds (v_rcp_f64, v_rsq_f64) by Newton-Raphson and Goldschmidt
// iterations (Markstein, "IA-64 and Elementary Functions", ch. 8), with a
// final residual correction.  Arguments are positive normal numbers; sqrt
// also returns 0 for 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rcp(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double div(double n, double d) {
    const double r = rcp(d);
    const double q = n * r;
    const double rem = fma(-d, q, n);
    return fma(rem, r, q);
}

__device__ __forceinline__ double sqrt(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    g = fma(d, h, g);
    return x == 0.0 ? 0.0 : g;
}

__device__ __forceinline__ double rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-h * y, y, 0.5);
    return fma(y, e, y);
}

// ---------------------------------------------------------------------------
// Natural logarithm of a positive normal double.  x = 2^e m with m in
// [sqrt(1/2), sqrt(2)); with f = m - 1 and s = f / (2 + f),
//   log(1 + f) = 2 atanh(s) = f - s f + 2 s (s^2/3 + s^4/5 + ...)
// (the atanh series of the logarithm, Abramowitz and Stegun 4.1.27), |s| <=
// 0.1716, truncated after s^23; ln 2 is split so that e ln2_hi is exact.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double log_pos(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    int e = (int)(b >> 52) - 1023;
    double m = __longlong_as_double((long long)((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    if (m > 1.4142135623730951) {
        m *= 0.5;
        e += 1;
    }
    const double f = m - 1.0;
    const double s = div(f, 2.0 + f);
    const double z = s * s;
    double p = 2.0 / 23.0;
    p = poly_step(p, z, 2.0 / 21.0);
    p = poly_step(p, z, 2.0 / 19.0);
    p = poly_step(p, z, 2.0 / 17.0);
    p = poly_step(p, z, 2.0 / 15.0);
    p = poly_step(p, z, 2.0 / 13.0);
    p = poly_step(p, z, 2.0 / 11.0);
    p = poly_step(p, z, 2.0 / 9.0);
    p = poly_step(p, z, 2.0 / 7.0);
    p = poly_step(p, z, 2.0 / 5.0);
    p = poly_step(p, z, 2.0 / 3.0);
    const double l1p = fma(-s, f, f) + s * z * p;
    const double de = (double)e;
    return fma(de, 0.6931467056274414, fma(de, 4.7493250390316726e-07, l1p));
}

// ---------------------------------------------------------------------------
// sin(2 pi u) and cos(2 pi u) for an angle given in turns (|u| < 2^30).  The
// reduction to the nearest quarter turn is exact in turns; the remainder
// (|a| <= pi/4 after scaling by 2 pi) goes through the Taylor series of sin
// to a^17 and of cos to a^18, and the quadrant permutes and negates.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sincos_turns(double u, double *sn, double *cs) {
    const double q = __builtin_rint(4.0 * u);
    const double r = fma(-0.25, q, u);
    const double a = r * 6.283185307179586;
    const double z = a * a;
    double P = 1.0 / 355687428096000.0;
    P = poly_step(P, z, -1.0 / 1307674368000.0);
    P = poly_step(P, z, 1.0 / 6227020800.0);
    P = poly_step(P, z, -1.0 / 39916800.0);
    P = poly_step(P, z, 1.0 / 362880.0);
    P = poly_step(P, z, -1.0 / 5040.0);
    P = poly_step(P, z, 1.0 / 120.0);
    P = poly_step(P, z, -1.0 / 6.0);
    const double s = fma(a * z, P, a);
    double Q = -1.0 / 6402373705728000.0;
    Q = poly_step(Q, z, 1.0 / 20922789888000.0);
    Q = poly_step(Q, z, -1.0 / 87178291200.0);
    Q = poly_step(Q, z, 1.0 / 479001600.0);
    Q = poly_step(Q, z, -1.0 / 3628800.0);
    Q = poly_step(Q, z, 1.0 / 40320.0);
    Q = poly_step(Q, z, -1.0 / 720.0);
    Q = poly_step(Q, z, 1.0 / 24.0);
    const double c = fma(z * z, Q, fma(-0.5, z, 1.0));
    const int qi = (int)q & 3;
    const double ss = (qi & 1) ? c : s;
    const double cc = (qi & 1) ? s : c;
    *sn = (qi & 2) ? -ss : ss;
    *cs = (qi == 1 || qi == 2) ? -cc : cc;
}

// ---------------------------------------------------------------------------
// FP32 forms for the mixed-precision path: the hardware transcendental
// instructions (v_log_f32 = log2, v_exp_f32 = exp2, v_sin_f32 / v_cos_f32 of
// turns, v_sqrt_f32, v_rsq_f32, v_rcp_f32), each about one ulp.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float log_pos(float x) {
    return __builtin_amdgcn_logf(x) * 0.69314718055994531f;
}
__device__ __forceinline__ float exp_(float x) {
    return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
}
__device__ __forceinline__ void sincos_turns(float u, float *sn, float *cs) {
    *sn = __builtin_amdgcn_sinf(u);
    *cs = __builtin_amdgcn_cosf(u);
}
__device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float div(float n, float d) { return n * __builtin_amdgcn_rcpf(d); }

}  // namespace dm
}  // namespace mrt
