// Per-ray mosaic-crystal transport kernels for gfx950 (MI355X).
//
// One lane traces one ray at a time.  Waves are persistent: each wave claims
// chunks of ray ids from a global counter, lanes whose ray has ended are
// refilled from the chunk, and per-ray state lives in registers.  A ray's
// random numbers come from Philox4x32-10 keyed by (seed, ray id, draw
// index), so the result does not depend on which lane or wave traced it.
//
// The physics per ray (HEART, arXiv 2503.16955):
//   source (sec. 2.1) -> front-face entry (sec. 2.2) -> events at the
//   majorant rate mu0 + R_max / h (Eq. AnyEvent): absorb with probability
//   mu0 / mu_tot, otherwise draw a crystallite normal from the mosaic
//   distribution (sec. 2.2.2), take Delta = asin|k.n| - alpha_B (Eq.
//   BraggLaw) and reflect (sec. 2.2.4) with probability r(Delta - Delta_M)
//   / R_max (sec. 2.2.1) -> detector binning (sec. 2.3).
//
// Two precisions share this source: R = double (everything FP64) and
// R = float (geometry, free paths, tilts, detector in FP32; the Bragg
// deviation, its rocking-curve argument and the photon energy in FP64).
#include <hip/hip_runtime.h>
#include <math.h>

#include "trace_params.h"

namespace mrt {
namespace {

constexpr int kWave = 64;
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kHC = 12.398419843320026;   // h c in keV Angstrom (SI 2019 exact)

enum LaneState : int { kIdle = 0, kActive = 1, kDone = 2 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// on words 0 and 2, xor with words 1 and 3 and the round key, permutation.
// Round keys are precomputed on the host (seed halves plus Weyl increments).
// ---------------------------------------------------------------------------
struct Words { uint32_t w[4]; };

__device__ __forceinline__ Words philox(const TraceParams &P, uint32_t c0, uint32_t c1,
                                        uint32_t c2, uint32_t c3) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ P.key0[r];
        const uint32_t n2 = hi0 ^ c3 ^ P.key1[r];
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    Words o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

__device__ __forceinline__ double u01_f64(uint32_t w) {   // open (0, 1), 32 bits
    return ((double)w + 0.5) * 0x1p-32;
}
__device__ __forceinline__ float u01_f32(uint32_t w) {    // open (0, 1), 23 bits, exact
    return (float)(((w >> 9) << 1) | 1u) * 0x1p-24f;
}

// ---------------------------------------------------------------------------
// Precision policy.
// ---------------------------------------------------------------------------
template <class R> struct Pol;

template <> struct Pol<double> {
    static __device__ __forceinline__ double uni(uint32_t w) { return u01_f64(w); }
    static __device__ __forceinline__ double log_(double x) { return log(x); }
    static __device__ __forceinline__ double exp_(double x) { return exp(x); }
    static __device__ __forceinline__ double expm1_(double x) { return expm1(x); }
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
    static __device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
    static __device__ __forceinline__ void sincos_(double x, double *s, double *c) { sincos(x, s, c); }
    static __device__ __forceinline__ double cv(double x) { return x; }
};

template <> struct Pol<float> {
    static __device__ __forceinline__ float uni(uint32_t w) { return u01_f32(w); }
    static __device__ __forceinline__ float log_(float x) { return __logf(x); }
    static __device__ __forceinline__ float exp_(float x) { return __expf(x); }
    static __device__ __forceinline__ float expm1_(float x) { return expm1f(x); }
    static __device__ __forceinline__ float sqrt_(float x) { return __fsqrt_rn(x); }
    static __device__ __forceinline__ float rsqrt_(float x) { return __frsqrt_rn(x); }
    static __device__ __forceinline__ void sincos_(float x, float *s, float *c) { __sincosf(x, s, c); }
    static __device__ __forceinline__ float cv(double x) { return (float)x; }
};

template <class R> struct V3 { R x, y, z; };

template <class R> __device__ __forceinline__ V3<R> ld3(const double *a) {
    return V3<R>{Pol<R>::cv(a[0]), Pol<R>::cv(a[1]), Pol<R>::cv(a[2])};
}
template <class R> __device__ __forceinline__ R dot(V3<R> a, V3<R> b) {
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <class R> __device__ __forceinline__ V3<R> axpy(V3<R> p, R t, V3<R> k) {
    return V3<R>{p.x + t * k.x, p.y + t * k.y, p.z + t * k.z};
}
template <class R> __device__ __forceinline__ V3<R> sub(V3<R> a, V3<R> b) {
    return V3<R>{a.x - b.x, a.y - b.y, a.z - b.z};
}
template <class R> __device__ __forceinline__ V3<R> cross(V3<R> a, V3<R> b) {
    return V3<R>{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class R> __device__ __forceinline__ R fminr(R a, R b) { return a < b ? a : b; }

// ---------------------------------------------------------------------------
// Per-lane ray state.
// ---------------------------------------------------------------------------
template <class R, bool REC> struct Ray {
    V3<R> p, k;          // local position, direction
    R dist;              // distance to the crystal boundary along k from p
    double E;            // keV
    double alpha_b;      // Bragg angle, < 0 when none
    uint64_t id;
    uint32_t nev, nrefl;
    int status;
    V3<R> entry;         // only read when REC
};

struct Counts {
    uint32_t missed, absorbed, exit_refl, exit_trans, truncated, detected, reflections;
    unsigned long long events;
};

// ---------------------------------------------------------------------------
// Source (sec. 2.1): cone direction uniform in solid angle; spectrum as PDF.
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void sample_source(const TraceParams &P, const double *bin_cdf,
                                              uint64_t ray, V3<R> &o, V3<R> &k, double &E) {
    const uint32_t rlo = (uint32_t)ray, rhi = (uint32_t)(ray >> 32);
    const Words a = philox(P, 0u, rlo, rhi, 0u);
    const Words b = philox(P, 1u, rlo, rhi, 0u);
    using M = Pol<R>;
    const R v = M::uni(a.w[0]) * M::cv(P.vmax);
    const R ct = R(1) - v;
    const R st = M::sqrt_(v * (R(2) - v));
    R sp, cp;
    M::sincos_(M::cv(kTwoPi) * M::uni(a.w[1]), &sp, &cp);
    const V3<R> ax = ld3<R>(P.sa), b1 = ld3<R>(P.sb1), b2 = ld3<R>(P.sb2);
    k.x = ct * ax.x + st * (cp * b1.x + sp * b2.x);
    k.y = ct * ax.y + st * (cp * b1.y + sp * b2.y);
    k.z = ct * ax.z + st * (cp * b1.z + sp * b2.z);
    o = ld3<R>(P.so);

    // energies in FP64 in both precisions
    const double s2 = u01_f64(a.w[2]), s3 = u01_f64(a.w[3]), s4 = u01_f64(b.w[0]);
    if (P.spectrum == MRT_SPECTRUM_UNIFORM) {
        E = P.e_min + s2 * P.e_span;
    } else if (P.spectrum == MRT_SPECTRUM_LINES) {
        int pick = P.n_lines;
        for (int j = 0; j < P.n_lines; ++j)
            if (s2 < P.line_cum[j]) { pick = j; break; }
        if (pick < P.n_lines) {
            double sg, cg;
            sincos(kTwoPi * s4, &sg, &cg);
            E = P.line_e[pick] + P.line_sig[pick] * sqrt(-2.0 * log(s3)) * cg;
        } else {
            E = P.e_min + s3 * P.e_span;
        }
    } else {
        // largest bin b with cdf[b] <= s2 (binary search over n_bins entries)
        int lo = 0, hi = P.n_bins - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (bin_cdf[mid] <= s2) lo = mid; else hi = mid - 1;
        }
        E = P.e_min + ((double)lo + s3) * P.e_span / (double)P.n_bins;
    }
}

// ---------------------------------------------------------------------------
// Crystal geometry (sec. 2.2).  The local origin lies on the cylinder axis.
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ bool entry_distance(const TraceParams &P, V3<R> o, V3<R> k, R &t) {
    if (P.geometry == MRT_GEOMETRY_FLAT) {
        const V3<R> N = ld3<R>(P.N);
        const R zeta = dot(o, N), kn = dot(k, N);
        if (!(kn < R(0))) return false;
        t = -zeta / kn;
        if (!(t > R(0))) return false;
        const V3<R> h = axpy(o, t, k);
        const R xi = dot(h, ld3<R>(P.e1)), eta = dot(h, ld3<R>(P.e2));
        return fabs(xi) <= Pol<R>::cv(P.hl) && fabs(eta) <= Pol<R>::cv(P.hw);
    }
    const V3<R> ax = ld3<R>(P.ax);
    const R ka = dot(k, ax);
    const V3<R> kp = axpy(k, -ka, ax);
    const R zo = dot(o, ax);
    const V3<R> rho = axpy(o, -zo, ax);
    const R a = dot(kp, kp), b = dot(rho, kp);
    const R cc = dot(rho, rho) - Pol<R>::cv(P.R2);
    if (!(cc < R(0)) || !(a > R(0))) return false;
    const R disc = b * b - a * cc;
    t = b >= R(0) ? -cc / (b + Pol<R>::sqrt_(disc)) : (-b + Pol<R>::sqrt_(disc)) / a;
    const V3<R> h = axpy(o, t, k);
    const R zh = dot(h, ax);
    const V3<R> rh = axpy(h, -zh, ax);
    return fabs(zh) <= Pol<R>::cv(P.hl) && dot(rh, ld3<R>(P.op)) <= R(0) &&
           dot(rh, ld3<R>(P.om)) <= R(0);
}

template <class R>
__device__ __forceinline__ R exit_distance(const TraceParams &P, V3<R> p, V3<R> k) {
    R t = R(INFINITY);
    if (P.geometry == MRT_GEOMETRY_FLAT) {
        const V3<R> N = ld3<R>(P.N), e1 = ld3<R>(P.e1), e2 = ld3<R>(P.e2);
        const R zeta = dot(p, N), xi = dot(p, e1), eta = dot(p, e2);
        const R kn = dot(k, N), k1 = dot(k, e1), k2 = dot(k, e2);
        const R hl = Pol<R>::cv(P.hl), hw = Pol<R>::cv(P.hw), T = Pol<R>::cv(P.T);
        if (kn > R(0)) t = fminr(t, -zeta / kn);
        if (kn < R(0)) t = fminr(t, (-T - zeta) / kn);
        if (k1 > R(0)) t = fminr(t, (hl - xi) / k1);
        if (k1 < R(0)) t = fminr(t, (-hl - xi) / k1);
        if (k2 > R(0)) t = fminr(t, (hw - eta) / k2);
        if (k2 < R(0)) t = fminr(t, (-hw - eta) / k2);
    } else {
        const V3<R> ax = ld3<R>(P.ax);
        const R z = dot(p, ax), ka = dot(k, ax);
        const V3<R> rho = axpy(p, -z, ax), kp = axpy(k, -ka, ax);
        const R a = dot(kp, kp), b = dot(rho, kp), r2 = dot(rho, rho);
        if (a > R(0)) {
            const R co = r2 - Pol<R>::cv(P.Ro2);
            R disc = b * b - a * co;
            if (disc < R(0)) disc = R(0);
            const R to = b >= R(0) ? -co / (b + Pol<R>::sqrt_(disc)) : (-b + Pol<R>::sqrt_(disc)) / a;
            t = fminr(t, to);
            if (b < R(0)) {
                const R ci = r2 - Pol<R>::cv(P.R2);
                const R di = b * b - a * ci;
                if (di >= R(0)) t = fminr(t, ci / (-b + Pol<R>::sqrt_(di)));
            }
        }
        const R hl = Pol<R>::cv(P.hl);
        if (ka > R(0)) t = fminr(t, (hl - z) / ka);
        if (ka < R(0)) t = fminr(t, (-hl - z) / ka);
        const V3<R> op = ld3<R>(P.op), om = ld3<R>(P.om);
        const R kop = dot(k, op), kom = dot(k, om);
        if (kop > R(0)) t = fminr(t, -dot(rho, op) / kop);
        if (kom > R(0)) t = fminr(t, -dot(rho, om) / kom);
    }
    return t > R(0) ? t : R(0);
}

// Local surface frame at p: N toward the source side, e1 along the length
// axis (flat) or the cylinder axis, e2 = N x e1.
template <class R>
__device__ __forceinline__ void local_frame(const TraceParams &P, V3<R> p, V3<R> &N, V3<R> &e1,
                                            V3<R> &e2) {
    if (P.geometry == MRT_GEOMETRY_FLAT) {
        N = ld3<R>(P.N); e1 = ld3<R>(P.e1); e2 = ld3<R>(P.e2);
        return;
    }
    const V3<R> ax = ld3<R>(P.ax);
    const V3<R> rho = axpy(p, -dot(p, ax), ax);
    const R inv = R(1) / Pol<R>::sqrt_(dot(rho, rho));
    N = V3<R>{-rho.x * inv, -rho.y * inv, -rho.z * inv};
    e1 = ax;
    e2 = cross(N, e1);
}

// ---------------------------------------------------------------------------
// Mosaic tilt (sec. 2.2.2): v = 1 - cos(theta) by inverse CDF, azimuth
// uniform.  Returns the crystallite normal.
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ R vmf_v(const TraceParams &P, R u) {
    using M = Pol<R>;
    const R v = -M::cv(P.vmf_s2) * M::log_(u + (R(1) - u) * M::cv(P.vmf_floor));
    return v < R(2) ? v : R(2);
}

template <class R>
__device__ __forceinline__ void lorentz_tilt(const TraceParams &P, R q, R &ct, R &st) {
    using M = Pol<R>;
    const R T = M::cv(P.lor_g) * M::sqrt_(R(1) - q * q) / q;
    const R c = M::rsqrt_(R(1) + T * T);
    ct = c;
    st = T * c;
}

template <class R>
__device__ __forceinline__ V3<R> mosaic_normal(const TraceParams &P, R u2, R u3, V3<R> N,
                                               V3<R> e1, V3<R> e2) {
    using M = Pol<R>;
    R ct = R(1), st = R(0);
    if (P.fwhm > 0.0) {
        R v = R(-1);
        switch (P.mdf) {
        case MRT_MOSAIC_GAUSSIAN_VMF:
            v = vmf_v<R>(P, u2);
            break;
        case MRT_MOSAIC_LORENTZIAN:
            lorentz_tilt<R>(P, R(1) - u2, ct, st);
            break;
        case MRT_MOSAIC_PSEUDO_VOIGT: {
            const R eta = M::cv(P.m_eta);
            if (u2 < eta) lorentz_tilt<R>(P, (eta - u2) * M::cv(P.inv_eta), ct, st);
            else v = vmf_v<R>(P, (u2 - eta) * M::cv(P.inv_1meta));
            break;
        }
        case MRT_MOSAIC_WRAPPED_LORENTZIAN:
            v = M::cv(P.wl_half_g2) * M::expm1_(u2 * M::cv(P.wl_z));
            v = v < R(2) ? v : R(2);
            break;
        default:
            v = M::cv(P.swl_k) * u2 / (M::cv(P.swl_d) - R(2) * u2);
            v = v < R(2) ? v : R(2);
            break;
        }
        if (v >= R(0)) {
            ct = R(1) - v;
            st = M::sqrt_(v * (R(2) - v));
        }
    }
    R sx, cx;
    M::sincos_(M::cv(kTwoPi) * u3, &sx, &cx);
    return V3<R>{ct * N.x + st * (cx * e1.x + sx * e2.x),
                 ct * N.y + st * (cx * e1.y + sx * e2.y),
                 ct * N.z + st * (cx * e1.z + sx * e2.z)};
}

// ---------------------------------------------------------------------------
// Rocking curve (sec. 2.2.1): acceptance ratio r(x) / R_max, x in FP64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double irc_ratio(const TraceParams &P, const double *lut, double x) {
    switch (P.irc) {
    case MRT_IRC_GAUSSIAN:
        return exp(-P.g_k * x * x);
    case MRT_IRC_PSEUDO_VOIGT: {
        const double x2 = x * x;
        return (P.pv_eta * P.pv_ln / (P.pv_h2 + x2) + (1.0 - P.pv_eta) * P.pv_gn * exp(-P.g_k * x2)) *
               P.pv_inv_r0;
    }
    case MRT_IRC_TABLE: {
        if (!(x >= P.lut_x0 && x <= P.lut_x1)) return 0.0;   // also rejects NaN
        const int n = P.lut_n;
        if (x == P.lut_x1) return lut[n - 1] * P.lut_inv_max;
        const double f = (x - P.lut_x0) * P.lut_scale;
        const int j = (int)floor(f);
        if (j >= n - 1) return lut[n - 1] * P.lut_inv_max;
        const double t = f - (double)j;
        return ((1.0 - t) * lut[j] + t * lut[j + 1]) * P.lut_inv_max;
    }
    case MRT_IRC_LORENTZIAN:
        return P.lor_h2 / (P.lor_h2 + x * x);
    default:
        return fabs(x) <= P.box_half ? 1.0 : 0.0;
    }
}

// FP32 rocking-curve evaluation of an FP64 argument (the mixed path keeps the
// argument in FP64 and needs the value only to float accuracy).
__device__ __forceinline__ float irc_ratio_f32(const TraceParams &P, const double *lut, double x) {
    switch (P.irc) {
    case MRT_IRC_GAUSSIAN:
        return __expf((float)(-P.g_k * x * x));
    case MRT_IRC_PSEUDO_VOIGT: {
        const double x2 = x * x;
        const float l = (float)(P.pv_h2 / (P.pv_h2 + x2));
        const float g = __expf((float)(-P.g_k * x2));
        return ((float)(P.pv_eta * P.pv_ln / P.pv_h2) * l + (float)((1.0 - P.pv_eta) * P.pv_gn) * g) *
               (float)P.pv_inv_r0;
    }
    default:
        return (float)irc_ratio(P, lut, x);
    }
}

// ---------------------------------------------------------------------------
// One event of a ray (sec. 2.2.3 and 2.2.4).  Returns true when the ray ends.
// ---------------------------------------------------------------------------
template <class R, bool REC>
__device__ __forceinline__ bool step(const TraceParams &P, const double *lut, Ray<R, REC> &ry) {
    using M = Pol<R>;
    if (ry.nev == P.max_events) { ry.status = MRT_TRUNCATED; return true; }
    const Words w = philox(P, ry.nev, (uint32_t)ry.id, (uint32_t)(ry.id >> 32), 1u);
    ++ry.nev;

    if ((int)ry.nrefl >= P.max_refl) {
        // reflection budget spent: Beer-Lambert absorption only
        const R l = -M::log_(M::uni(w.w[0])) * M::cv(P.inv_mu0);
        if (l < ry.dist) { ry.p = axpy(ry.p, l, ry.k); ry.status = MRT_ABSORBED; }
        else { ry.p = axpy(ry.p, ry.dist, ry.k);
               ry.status = ry.nrefl ? MRT_EXIT_REFLECTED : MRT_EXIT_TRANSMITTED; }
        return true;
    }
    // free path to the next event at the majorant rate (Eq. AnyEvent)
    const R l = -M::log_(M::uni(w.w[0])) * M::cv(P.inv_mu_tot);
    if (l >= ry.dist) {
        ry.p = axpy(ry.p, ry.dist, ry.k);
        ry.status = ry.nrefl ? MRT_EXIT_REFLECTED : MRT_EXIT_TRANSMITTED;
        return true;
    }
    ry.p = axpy(ry.p, l, ry.k);
    ry.dist -= l;
    const R u1 = M::uni(w.w[1]);
    const R pa = M::cv(P.p_a);
    if (u1 < pa) { ry.status = MRT_ABSORBED; return true; }
    if (ry.alpha_b < 0.0) return false;
    const R u_acc = (u1 - pa) * M::cv(P.inv_1mpa);

    V3<R> N, e1, e2;
    local_frame<R>(P, ry.p, N, e1, e2);
    const V3<R> n = mosaic_normal<R>(P, M::uni(w.w[2]), M::uni(w.w[3]), N, e1, e2);
    // Bragg deviation in FP64 (k.n accumulated in FP64 from the components)
    const double kn = (double)ry.k.x * (double)n.x + (double)ry.k.y * (double)n.y +
                      (double)ry.k.z * (double)n.z;
    double akn = fabs(kn);
    akn = akn < 1.0 ? akn : 1.0;
    const double x = (asin(akn) - ry.alpha_b) - P.shift;
    bool accept;
    if constexpr (sizeof(R) == 8) accept = u_acc < irc_ratio(P, lut, x);
    else accept = u_acc < irc_ratio_f32(P, lut, x);
    if (accept) {
        const R two_kn = R(2) * (R)kn;
        V3<R> ks = V3<R>{ry.k.x - two_kn * n.x, ry.k.y - two_kn * n.y, ry.k.z - two_kn * n.z};
        const R nr = M::sqrt_(dot(ks, ks));
        ry.k = V3<R>{ks.x / nr, ks.y / nr, ks.z / nr};
        ++ry.nrefl;
        ry.dist = exit_distance<R>(P, ry.p, ry.k);
    }
    return false;
}

// ---------------------------------------------------------------------------
// End of a ray: detector (sec. 2.3), counters, record.
// ---------------------------------------------------------------------------
template <class R, bool REC>
__device__ __forceinline__ void finish(const TraceParams &P, Ray<R, REC> &ry, Counts &c) {
    int pi = -1, pj = -1;
    V3<R> end = ry.p;
    bool detected = false;
    switch (ry.status) {
    case MRT_MISS: ++c.missed; break;
    case MRT_ABSORBED: ++c.absorbed; break;
    case MRT_EXIT_REFLECTED: ++c.exit_refl; break;
    case MRT_EXIT_TRANSMITTED: ++c.exit_trans; break;
    default: ++c.truncated; break;
    }
    c.events += ry.nev;
    c.reflections += ry.nrefl;
    if (ry.status == MRT_EXIT_REFLECTED || ry.status == MRT_EXIT_TRANSMITTED) {
        const V3<R> dn = ld3<R>(P.dn);
        const R kn = dot(ry.k, dn);
        if (kn < R(0)) {
            const V3<R> dP = ld3<R>(P.dP);
            const R t = dot(sub(dP, ry.p), dn) / kn;
            if (t > R(0)) {
                const V3<R> h = axpy(ry.p, t, ry.k);
                const V3<R> d = sub(h, dP);
                const R fu = dot(d, ld3<R>(P.du)) / Pol<R>::cv(P.pitch) + Pol<R>::cv(P.half_nx);
                const R fv = dot(d, ld3<R>(P.dv)) / Pol<R>::cv(P.pitch) + Pol<R>::cv(P.half_ny);
                const R fi = floor(fu), fj = floor(fv);
                if (fi >= R(0) && fj >= R(0) && fi < (R)P.nx && fj < (R)P.ny) {
                    pi = (int)fi;
                    pj = (int)fj;
                    detected = true;
                    end = h;
                    const size_t px = (size_t)pj * (size_t)P.nx + (size_t)pi;
                    atomicAdd(&P.counts[px], 1u);
                    if (P.energy)
                        atomicAdd(&P.energy[px], (unsigned long long)rint(ry.E * 1e6));
                    ++c.detected;
                }
            }
        }
    }
    if constexpr (REC) {
        int64_t idx = -1;
        if (P.records_mode == MRT_RECORDS_ALL) {
            idx = (int64_t)(ry.id - P.first);
        } else if (detected) {
            const unsigned long long slot = atomicAdd(&P.dev_counters[kCRecords], 1ull);
            if (slot < P.rec_cap) idx = (int64_t)slot;
        }
        if (idx >= 0) {
            mrt_hit_record *r = &P.records[idx];
            const bool miss = ry.status == MRT_MISS;
            const double nan = __builtin_nan("");
            r->ray_id = ry.id;
            r->energy_kev = ry.E;
            r->entry[0] = miss ? nan : (double)ry.entry.x + P.origin[0];
            r->entry[1] = miss ? nan : (double)ry.entry.y + P.origin[1];
            r->entry[2] = miss ? nan : (double)ry.entry.z + P.origin[2];
            r->end[0] = miss ? nan : (double)end.x + P.origin[0];
            r->end[1] = miss ? nan : (double)end.y + P.origin[1];
            r->end[2] = miss ? nan : (double)end.z + P.origin[2];
            r->dir[0] = ry.k.x; r->dir[1] = ry.k.y; r->dir[2] = ry.k.z;
            r->pix_i = pi; r->pix_j = pj;
            r->n_events = ry.nev;
            r->n_refl = (uint16_t)ry.nrefl;
            r->status = (uint8_t)ry.status;
            r->detected = detected ? 1 : 0;
        }
    }
}

// Start a ray: source, entry, Bragg angle, first exit distance.  Returns
// false on a miss (status MISS).
template <class R, bool REC>
__device__ __forceinline__ bool start(const TraceParams &P, const double *bin_cdf, uint64_t ray,
                                      Ray<R, REC> &ry) {
    V3<R> o, k;
    double E;
    sample_source<R>(P, bin_cdf, ray, o, k, E);
    ry.id = ray;
    ry.E = E;
    ry.k = k;
    ry.nev = 0;
    ry.nrefl = 0;
    R t;
    if (!entry_distance<R>(P, o, k, t)) {
        ry.status = MRT_MISS;
        ry.p = o;
        return false;
    }
    ry.p = axpy(o, t, k);
    if constexpr (REC) ry.entry = ry.p;
    const double s = kHC / (P.two_d * E);   // Eq. BraggLaw
    ry.alpha_b = s < 1.0 ? asin(s) : -1.0;
    ry.dist = exit_distance<R>(P, ry.p, ry.k);
    return true;
}

__device__ __forceinline__ uint32_t wave_reduce_u32(uint32_t v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ unsigned long long wave_reduce_u64(unsigned long long v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ void flush_counts(const TraceParams &P, Counts &c) {
    const uint32_t vals[7] = {c.missed, c.absorbed, c.exit_refl, c.exit_trans, c.truncated,
                              c.detected, c.reflections};
    const int slots[7] = {kCMissed, kCAbsorbed, kCExitReflected, kCExitTransmitted, kCTruncated,
                          kCDetected, kCReflections};
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const uint32_t s = wave_reduce_u32(vals[i]);
        if (__lane_id() == 0 && s) atomicAdd(&P.dev_counters[slots[i]], (unsigned long long)s);
    }
    const unsigned long long ev = wave_reduce_u64(c.events);
    if (__lane_id() == 0 && ev) atomicAdd(&P.dev_counters[kCEvents], ev);
    c = Counts{};
}

__device__ __forceinline__ uint32_t lane_rank(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---------------------------------------------------------------------------
// Persistent trace kernel.
// ---------------------------------------------------------------------------
template <class R, bool REC>
__global__ void __launch_bounds__(256) trace_kernel(const TraceParams P) {
    extern __shared__ double lds[];
    // stage the rocking-curve table and the spectrum CDF in LDS
    const int nl = P.irc == MRT_IRC_TABLE ? P.lut_n : 0;
    const int nc = P.spectrum == MRT_SPECTRUM_TABLE ? P.n_bins + 1 : 0;
    for (int i = threadIdx.x; i < nl; i += blockDim.x) lds[i] = P.lut[i];
    for (int i = threadIdx.x; i < nc; i += blockDim.x) lds[nl + i] = P.bin_cdf[i];
    __syncthreads();
    const double *lut = lds;
    const double *cdf = lds + nl;

    Ray<R, REC> ry;
    ry.status = MRT_MISS;
    int state = kIdle;
    Counts cnt{};
    uint64_t next = 0, end = 0;     // wave-uniform chunk cursor (offsets into [0, n))
    bool more = true;               // wave-uniform: unclaimed rays remain

    for (;;) {
        if (state == kDone) { finish<R, REC>(P, ry, cnt); state = kIdle; }

        // refill idle lanes from the wave's chunk, claiming chunks as needed
        while (more) {
            const unsigned long long idle = __ballot(state == kIdle);
            if (idle == 0) break;
            if (next == end) {
                flush_counts(P, cnt);
                unsigned long long base = 0;
                if (__lane_id() == 0) base = atomicAdd(P.chunk_counter, (unsigned long long)P.chunk);
                base = __shfl(base, 0, kWave);
                if (base >= P.n) { more = false; break; }
                next = base;
                end = base + P.chunk < P.n ? base + P.chunk : P.n;
            }
            const uint64_t avail = end - next;
            const uint32_t nidle = (uint32_t)__popcll(idle);
            const uint32_t take = avail < nidle ? (uint32_t)avail : nidle;
            if (state == kIdle) {
                const uint32_t r = lane_rank(idle);
                if (r < take) {
                    state = start<R, REC>(P, cdf, P.first + next + r, ry) ? kActive : kDone;
                }
            }
            next += take;
        }
        if (!__any(state != kIdle)) break;   // no ray in flight and none left

        // events: run while enough lanes are busy (drain once rays run out)
        const uint32_t keep = more ? 40u : 1u;
        for (;;) {
            if (state == kActive && step<R, REC>(P, lut, ry)) state = kDone;
            const unsigned long long act = __ballot(state == kActive);
            if ((uint32_t)__popcll(act) < keep) break;
        }
    }
    flush_counts(P, cnt);
}

__global__ void zero_kernel(uint32_t *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

}  // namespace

int launch_trace(const TraceParams &p, int precision, bool records, int grid, int block,
                 size_t lds_bytes, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (precision == MRT_FP64) {
        if (records) hipLaunchKernelGGL((trace_kernel<double, true>), dim3(grid), dim3(block), lds_bytes, s, p);
        else hipLaunchKernelGGL((trace_kernel<double, false>), dim3(grid), dim3(block), lds_bytes, s, p);
    } else {
        if (records) hipLaunchKernelGGL((trace_kernel<float, true>), dim3(grid), dim3(block), lds_bytes, s, p);
        else hipLaunchKernelGGL((trace_kernel<float, false>), dim3(grid), dim3(block), lds_bytes, s, p);
    }
    return (int)hipGetLastError();
}

int occupancy(int precision, bool records, int block, size_t lds_bytes, int *blocks_per_cu) {
    const void *f;
    if (precision == MRT_FP64)
        f = records ? (const void *)trace_kernel<double, true> : (const void *)trace_kernel<double, false>;
    else
        f = records ? (const void *)trace_kernel<float, true> : (const void *)trace_kernel<float, false>;
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, block, lds_bytes);
}

int launch_zero(void *ptr, size_t n_words, void *stream) {
    if (n_words == 0) return 0;
    size_t blocks = (n_words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (uint32_t *)ptr, n_words);
    return (int)hipGetLastError();
}

}  // namespace mrt
