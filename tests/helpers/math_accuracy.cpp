// Accuracy of the FP64 device math (device_math.h compiled for the host)
// against long-double references: worst error in ulps of log over uniform
// words, over 80 binades and densely near 1, of exp over non-positive
// arguments (normal and subnormal results), and of sin/cos of turns (the reference reduced
// exactly in quarter turns as well).  Also every FP32 uniform u01_f32(w)
// against its definition ((w >> 9) 2 + 1) 2^-24 in exact arithmetic, over all
// 2^23 values of w >> 9, and the FP64 uniform (w + 1/2) 2^-32 on 2^24 words.
// And log_u01 and sincos_u01 (the forms fed by the word) bit for bit equal
// to log_pos and sincos_turns of the word's uniform.  And rcp, div, sqrt and
// rsqrt from seeds 2^-23 off.  Prints "log L sin S cos C exp X
// u01_f32_mismatches M u01_identity_mismatches I rcp R sqrt Q rsqrt T" (M
// counts both uniforms, R covers rcp and div).
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <initializer_list>
#include "device_math.h"
using namespace mrt;
static double ulp_err(double got, long double ref) {
    if (ref == 0) return got == 0 ? 0 : 1e30;
    double r = (double)ref;
    double u = std::nextafter(std::fabs(r), INFINITY) - std::fabs(r);
    return (double)std::fabs((long double)got - ref) / u;
}
int main() {
    uint64_t s = 88172645463325252ull;
    double worst_log = 0, worst_sin = 0, worst_cos = 0; double wl_x = 0, ws_x = 0;
    const long n_uni = 2000000, n_wide = 1000000;
    for (long i = 0; i < n_uni; ++i) {
        s ^= s << 13; s ^= s >> 7; s ^= s << 17;
        const uint32_t w = (uint32_t)s;
        const double u = ((double)w + 0.5) * 0x1p-32;
        double e = ulp_err(dm::log_pos(u), logl((long double)u));
        if (e > worst_log) { worst_log = e; wl_x = u; }
        double sn, cs; dm::sincos_turns(u, &sn, &cs);
        const long double q = rintl(4.0L * (long double)u);
        long double a = 6.2831853071795864769252867665590058L * ((long double)u - q / 4.0L) + 1.5707963267948966192313216916397514L * q;
        // exact quarter-turn reduction for the reference too
        const long double ar = 6.2831853071795864769252867665590058L * ((long double)u - q / 4.0L);
        const int qi = ((int)q) & 3;
        long double rs = qi == 0 ? sinl(ar) : qi == 1 ? cosl(ar) : qi == 2 ? -sinl(ar) : -cosl(ar);
        long double rc = qi == 0 ? cosl(ar) : qi == 1 ? -sinl(ar) : qi == 2 ? -cosl(ar) : sinl(ar);
        (void)a;
        double es = ulp_err(sn, rs), ec = ulp_err(cs, rc);
        if (es > worst_sin) { worst_sin = es; ws_x = u; }
        if (ec > worst_cos) worst_cos = ec;
    }
    // log over other ranges (vMF argument u + (1-u) floor, energies, etc.)
    for (long i = 0; i < n_wide; ++i) {
        s ^= s << 13; s ^= s >> 7; s ^= s << 17;
        double x = std::ldexp(1.0 + (double)(s >> 11) * 0x1p-53, (int)(s % 80) - 40);
        double e = ulp_err(dm::log_pos(x), logl((long double)x));
        if (e > worst_log) { worst_log = e; wl_x = x; }
    }
    // log near 1, where its value is small and must keep its relative
    // accuracy: every binade of |x - 1| from 2^-1 to 2^-53 on both sides, and
    // the first thousand doubles on either side of 1
    for (int j = 1; j <= 53; ++j) {
        for (int i = 0; i < 2000; ++i) {
            s ^= s << 13; s ^= s >> 7; s ^= s << 17;
            const double d = std::ldexp(1.0 + (double)(s >> 11) * 0x1p-53, -j);
            for (double x : {1.0 + d, 1.0 - d}) {
                if (!(x > 0.0) || x == 1.0) continue;
                double e = ulp_err(dm::log_pos(x), logl((long double)x));
                if (e > worst_log) { worst_log = e; wl_x = x; }
            }
        }
    }
    for (int k = 1; k <= 1000; ++k)
        for (double x : {1.0 + k * 0x1p-52, 1.0 - k * 0x1p-53}) {
            double e = ulp_err(dm::log_pos(x), logl((long double)x));
            if (e > worst_log) { worst_log = e; wl_x = x; }
        }
    if (dm::log_pos(1.0) != 0.0) worst_log = 1e30;
    // exp for non-positive arguments: uniform over [-708, 0] (normal
    // results), every binade of |x| from 2^-60 to 2^9, and the subnormal
    // range in absolute terms; exp(0) = 1, exp(-1100) = 0
    double worst_exp = 0;
    for (long i = 0; i < n_wide; ++i) {
        s ^= s << 13; s ^= s >> 7; s ^= s << 17;
        const double x = -708.0 * (double)(s >> 11) * 0x1p-53;
        double e = ulp_err(dm::exp_nonpos(x), expl((long double)x));
        if (e > worst_exp) worst_exp = e;
    }
    for (int j = -60; j <= 9; ++j)
        for (int i = 0; i < 2000; ++i) {
            s ^= s << 13; s ^= s >> 7; s ^= s << 17;
            const double x = -std::ldexp(1.0 + (double)(s >> 11) * 0x1p-53, j);
            if (x < -708.0) continue;
            double e = ulp_err(dm::exp_nonpos(x), expl((long double)x));
            if (e > worst_exp) worst_exp = e;
        }
    for (int i = 0; i < 100000; ++i) {
        const double x = -708.4 - 37.0 * i / 100000.0;
        const long double ref = expl((long double)x);
        const long double err = fabsl((long double)dm::exp_nonpos(x) - ref);
        if (err > 2.0L * 0x1p-1074L + ref * 0x1p-52L) worst_exp = 1e30;
    }
    if (dm::exp_nonpos(0.0) != 1.0 || dm::exp_nonpos(-1100.0) != 0.0 ||
        dm::exp_nonpos(-1e300) != 0.0)
        worst_exp = 1e30;
    // exactly +0 from -746 on (the quadrature skips it there), nonzero just above
    for (int i = 0; i <= 200000; ++i) {
        const double x = -746.0 - 400.0 * i / 200000.0;
        const double e = dm::exp_nonpos(x);
        if (e != 0.0 || std::signbit(e)) worst_exp = 1e30;
    }
    if (!(dm::exp_nonpos(-745.0) > 0.0)) worst_exp = 1e30;
    long mismatches = 0;
    for (uint32_t k = 0; k < (1u << 23); ++k) {
        const uint32_t w = (k << 9) | (k & 0x1ffu);   // low bits do not matter
        const double want = (double)(2u * k + 1u) * 0x1p-24;
        const float got = dm::u01_f32(w);
        if ((double)got != want || !(got > 0.0f && got < 1.0f)) ++mismatches;
    }
    // and the FP64 uniform (w + 1/2) 2^-32, on 2^24 words spread over the range
    for (uint64_t k = 0; k < (1u << 24); ++k) {
        const uint32_t w = (uint32_t)(k * 257u + (k >> 12));
        const long double want = ((long double)w + 0.5L) * 0x1p-32L;
        if ((long double)dm::u01_f64(w) != want) ++mismatches;
    }
    for (uint32_t w : {0u, 1u, 0xffffffffu, 0x80000000u})
        if ((long double)dm::u01_f64(w) != ((long double)w + 0.5L) * 0x1p-32L) ++mismatches;
    // reciprocal, quotient, square root and reciprocal square root from
    // seeds exact and 2^-23 off either way (twice the hardware's), over 80
    // binades
    double worst_rcp = 0, worst_sqrt = 0, worst_rsqrt = 0;
    for (double rel : {0.0, 0x1p-23, -0x1p-23}) {
        simt_seed_rel = rel;
        for (long i = 0; i < n_wide; ++i) {
            s ^= s << 13; s ^= s >> 7; s ^= s << 17;
            const double x = std::ldexp(1.0 + (double)(s >> 11) * 0x1p-53, (int)(s % 80) - 40);
            const double y = std::ldexp(1.0 + (double)(s >> 23) * 0x1p-41, (int)((s >> 7) % 40) - 20);
            worst_rcp = std::fmax(worst_rcp, ulp_err(dm::rcp(x), 1.0L / (long double)x));
            worst_rcp = std::fmax(worst_rcp, ulp_err(dm::div(y, x), (long double)y / (long double)x));
            worst_sqrt = std::fmax(worst_sqrt, ulp_err(dm::sqrt(x), sqrtl((long double)x)));
            worst_rsqrt = std::fmax(worst_rsqrt, ulp_err(dm::rsqrt(x), 1.0L / sqrtl((long double)x)));
        }
    }
    simt_seed_rel = 0.0;
    // the uniform-fed forms against the general ones on the uniform, bit for
    // bit: 2^24 words spread over the range, every word within 64 of the
    // points where the integer reduction changes (bit 23 set or clear, the
    // top byte wrapping), and the ends
    long identity = 0;
    auto same = [](double a, double b) { return std::memcmp(&a, &b, sizeof a) == 0; };
    auto check = [&](uint32_t w) {
        const double u = dm::u01_f64(w);
        if (!same(dm::log_u01(w), dm::log_pos(u))) ++identity;
        double s1, c1, s2, c2;
        dm::sincos_u01(w, &s1, &c1);
        dm::sincos_turns(u, &s2, &c2);
        if (!same(s1, s2) || !same(c1, c2)) ++identity;
    };
    for (uint64_t k = 0; k < (1u << 24); ++k) check((uint32_t)(k * 257u + (k >> 12)));
    for (uint32_t top = 0; top < 256; ++top)
        for (uint32_t edge : {0u, 0x7fffffu, 0x800000u, 0xffffffu})
            for (int d = -64; d <= 64; ++d) check((top << 24) + edge + (uint32_t)d);
    printf("log %.4f sin %.4f cos %.4f exp %.4f u01_f32_mismatches %ld u01_identity_mismatches %ld "
           "rcp %.4f sqrt %.4f rsqrt %.4f\n",
           worst_log, worst_sin, worst_cos, worst_exp, mismatches, identity, worst_rcp, worst_sqrt,
           worst_rsqrt);
    (void)wl_x;
    (void)ws_x;
}
