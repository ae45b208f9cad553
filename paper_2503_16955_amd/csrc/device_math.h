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

#include "math_tables.h"

// Pointer qualifier for read-only device tables read at wave-uniform
// indices: the constant address space, whose uniform loads the compiler
// issues as scalar loads.  (Host builds of the device code for tests define
// it empty.)
#ifndef MRT_CONST_AS
#define MRT_CONST_AS __attribute__((address_space(4)))
#endif

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
        // three-input XORs as one v_bitop3_b32 each (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words{c0, c1, c2, c3};
}

// Uniforms in the open interval (0, 1): (w + 1/2) 2^-32 = (2w + 1) 2^-33,
// the odd integer 2w + 1 from one FMA with the inline constants 2 and 1, and
// the power of two by ldexp (both exact: 33 significant bits).  (The single
// FMA w 2^-32 + 2^-33 needs its two 64-bit constants moved into vector
// registers at every use.)
__device__ __forceinline__ double odd_u01(uint32_t w) { return __builtin_fma((double)w, 2.0, 1.0); }
__device__ __forceinline__ double u01_f64(uint32_t w) { return __builtin_ldexp(odd_u01(w), -33); }
// 23 random bits, exact in float: ((w >> 9) + 1/2) 2^-23.  One funnel
// shift places w >> 9 under the exponent of 1.0 (the float 1 + (w >> 9)
// 2^-23), and subtracting 1 - 2^-24 leaves (2 (w >> 9) + 1) 2^-24 exactly
// (the operands are within a factor 2, and the result has 24 significant
// bits): two instructions for the shift, conversion and FMA.
__device__ __forceinline__ float u01_f32(uint32_t w) {
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9u)) - 0x1.fffffep-1f;
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
// FP64 reciprocal, quotient and square root from the hardware seeds
// (v_rcp_f64, v_rsq_f64) by Newton-Raphson and Goldschmidt iterations
// (Markstein, "IA-64 and Elementary Functions", ch. 8), with a final
// residual correction; the reciprocal square root by one third-order step
// (below).  Arguments are positive normal numbers; sqrt also returns 0 for 0.
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

// 1/sqrt(x) from the hardware seed y (about 2^-24 off) by one third-order
// step: with e = 1 - x y^2, 1/sqrt(x) = y (1 - e)^(-1/2) = y (1 + e/2 +
// 3e^2/8 + ...), the e^3 term below 2^-70.  Five operations and a chain of
// four, where two Newton steps take seven and six.
__device__ __forceinline__ double rsqrt(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// ---------------------------------------------------------------------------
// Natural logarithm of a positive normal double, by the table method: x =
// 2^e m with m in [1, 2); inv is the table's float near 1 / m (128 intervals)
// and r = m inv - 1, |r| <= 2^-8, from one FMA; then
//   log x = e ln 2 + (-log inv) + log1p(r),
// log1p by its series to r^8, the high parts e ln2_hi (exact: ln2_hi has 32
// significant bits) and -log(inv)_hi summed first.  The first interval has
// inv = 1 and -log(inv) = 0, the last inv = 1/2 and -log(inv) = ln2_hi +
// ln2_lo, the same split as e ln 2: within 2^-8 of 1 (e = 0 above 1, e = -1
// below) r = x - 1 exactly and the high and low parts cancel to zero, so
// small logarithms keep their relative accuracy without a separate branch
// (there r reaches 2^-7, and the series' truncation stays below 2^-56
// relative).  About 1 ulp.
// ---------------------------------------------------------------------------
// log of x 2^-bias (bias 0: log x): the scale enters only the exponent.
__device__ __forceinline__ double log_scaled(double x, int bias) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const int e = (int)(b >> 52) - (1023 + bias);
    const double m = __longlong_as_double((long long)((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    const LogEntry t = kLogTable[(b >> 45) & 127];
    const double r = fma(m, (double)t.inv, -1.0);
    double p = -1.0 / 8.0;
    p = poly_step(p, r, 1.0 / 7.0);
    p = poly_step(p, r, -1.0 / 6.0);
    p = poly_step(p, r, 1.0 / 5.0);
    p = poly_step(p, r, -1.0 / 4.0);
    p = poly_step(p, r, 1.0 / 3.0);
    p = poly_step(p, r, -1.0 / 2.0);
    const double l1p = fma(r * r, p, r);
    const double de = (double)e;
    const double hi = fma(de, 0x1.62e42feep-1, t.nlog_hi);
    const double lo = fma(de, 0x1.a39ef35793c76p-33, t.nlog_lo);
    return hi + (lo + l1p);
}
__device__ __forceinline__ double log_pos(double x) { return log_scaled(x, 0); }
// log u01_f64(w), bit for bit: the same mantissa as 2w + 1, the exponent 33
// lower, so the power of two never needs applying.
__device__ __forceinline__ double log_u01(uint32_t w) { return log_scaled(odd_u01(w), 33); }

// ---------------------------------------------------------------------------
// exp(x) for x <= 0 (the mosaic densities, the rocking curves' Gaussians), by
// the table method: k = rint(128 x / ln 2), r = x - k ln2 / 128 in two FMAs
// (ln2_hi / 128 has 32 significant bits, so k ln2_hi / 128 is exact for
// |k| < 2^21), |r| <= ln 2 / 256; exp(r) - 1 by its series to r^5 (truncation
// below 2^-60); the table's 2^(j / 128) = hi + lo for j = k mod 128; the
// power 2^(k div 128) by ldexp, which also gives the subnormal and zero
// results.  Arguments below -1100 give 0.  About 1 ulp.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double exp_nonpos(double x) {
    x = x > -1100.0 ? x : -1100.0;
    const double kd = __builtin_rint(x * 0x1.71547652b82fep+7);   // 128 / ln 2
    const int k = (int)kd;
    double r = fma(-kd, 0x1.62e42feep-8, x);
    r = fma(-kd, 0x1.a39ef35793c76p-40, r);
    double p = 1.0 / 120.0;
    p = poly_step(p, r, 1.0 / 24.0);
    p = poly_step(p, r, 1.0 / 6.0);
    p = poly_step(p, r, 0.5);
    const double em1 = fma(r * r, p, r);   // exp(r) - 1
    const ExpEntry t = kExpTable[k & 127];
    return __builtin_ldexp(t.hi + fma(t.hi, em1, t.lo), k >> 7);
}

// ---------------------------------------------------------------------------
// sin and cos of 2 pi u (u in turns, u in [0, 1)).  u = q / 256 + r exactly
// (|r| <= 1/512); with a = 2 pi r, |a| <= 0.0123, sin a and cos a by their
// series to a^7 and a^6, then the angle-addition formulas with the table's
// sin and cos of 2 pi q / 256 (exact at the quadrant points).  About 1 ulp.
// ---------------------------------------------------------------------------
// The series and the table step for a = 2 pi r and the table index q mod 256.
__device__ __forceinline__ void sincos_reduced(double a, int qi, double *sn, double *cs) {
    const double z = a * a;
    double ps = -1.0 / 5040.0;
    ps = poly_step(ps, z, 1.0 / 120.0);
    ps = poly_step(ps, z, -1.0 / 6.0);
    const double sa = fma(a * z, ps, a);
    double pc = -1.0 / 720.0;
    pc = poly_step(pc, z, 1.0 / 24.0);
    pc = poly_step(pc, z, -0.5);
    const double cm = z * pc;   // cos a - 1
    const SinCosEntry t = kSinCosTable[qi & 255];
    // the table value is added last, to the small corrections
    *sn = t.s + fma(t.s, cm, t.c * sa);
    *cs = t.c + fma(t.c, cm, -(t.s * sa));
}
__device__ __forceinline__ void sincos_turns(double u, double *sn, double *cs) {
    const double q = __builtin_rint(256.0 * u);
    const double r = fma(-0x1p-8, q, u);
    sincos_reduced(fma(r, 0x1.921fb54442d18p+2, r * 0x1.1a62633145c07p-52), (int)q, sn, cs);
}
// sincos_turns(u01_f64(w)), bit for bit, with the reduction in integers: u =
// (2w + 1) 2^-33 lies within 1/512 of q / 256 for q = round(256 u), never
// halfway (2w + 1 is odd), so q = (w >> 24) + bit 23 of w, the table index
// is (w + 2^23) >> 24 mod 256, and r = u - q / 256 = (2d + 1) 2^-33 with d
// the low 24 bits of w read as a signed integer.  2 pi r is then formed from
// t = 2d + 1 and the constants scaled by 2^-33, which rounds exactly as the
// products with r do.
__device__ __forceinline__ void sincos_u01(uint32_t w, double *sn, double *cs) {
    const int d = (int)(w << 8) >> 8;
    const double t = (double)(2 * d + 1);
    sincos_reduced(fma(t, 0x1.921fb54442d18p-31, t * 0x1.1a62633145c07p-85),
                   (int)((w + 0x800000u) >> 24), sn, cs);
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
