// Per-ray mosaic-crystal transport kernel for gfx950 (MI355X), templated on
// precision, crystal geometry, mosaic distribution and rocking curve, so that
// each instance keeps only its own parameters live across the event loop.
//
// One lane traces one ray at a time.  Waves are persistent: each claims
// chunks of ray ids from a global counter, lanes whose ray has ended are
// refilled from the chunk (a ray that misses the crystal is retired inside
// the refill loop), and per-ray state lives in registers.  Random numbers
// come from Philox4x32-10 keyed by (seed, ray id, draw index), so a ray's
// result does not depend on the lane, wave or launch shape that traced it.
//
// The physics per ray (HEART, arXiv 2503.16955):
//   source (sec. 2.1) -> front-face entry (sec. 2.2) -> events at the
//   majorant rate mu0 + R_max / h (Eq. AnyEvent): absorb with probability
//   mu0 / mu_tot, otherwise draw a crystallite normal from the mosaic
//   distribution (sec. 2.2.2), take Delta = asin|k.n| - alpha_B (Eq.
//   BraggLaw) and reflect (reflection equation, sec. 2.2.4) with probability
//   r(Delta - Delta_M) / R_max (sec. 2.2.1) -> detector binning (sec. 2.3).
//
// R = double: everything in FP64.  R = float (mixed): geometry, free paths,
// tilts and detector in FP32; photon energy, Bragg angle, k.n (accumulated
// in FP64 from the FP32 components), Delta and the rocking-curve argument in
// FP64.
#pragma once
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "trace_params.h"

// Bounds assertions of the loop's indices: compiled out for the device; the
// CPU emulation of the kernels defines it to check every index it computes.
#ifndef MRT_DEV_CHECK
#define MRT_DEV_CHECK(cond) ((void)0)
#endif

namespace mrt {
namespace tk {

constexpr int kWave = 64;
constexpr double kHC = 12.398419843320026;   // h c in keV Angstrom (SI 2019 exact)

template <class R> struct V3 { R x, y, z; };

template <class R> __device__ __forceinline__ R cvt(double x) { return (R)x; }
template <class R> __device__ __forceinline__ V3<R> ld3(const double *a) {
    return V3<R>{cvt<R>(a[0]), cvt<R>(a[1]), cvt<R>(a[2])};
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
// A parameter in the path's precision: the FP64 value, or its FP32 copy.
template <class R> __device__ __forceinline__ R par(double d, float f) {
    if constexpr (sizeof(R) == 8) return d;
    else return f;
}
template <class R> __device__ __forceinline__ V3<R> par3(const double *d, const float *f) {
    if constexpr (sizeof(R) == 8) return V3<R>{d[0], d[1], d[2]};
    else return V3<R>{f[0], f[1], f[2]};
}
template <class R> __device__ __forceinline__ R uni(uint32_t w);
template <> __device__ __forceinline__ double uni<double>(uint32_t w) { return dm::u01_f64(w); }
template <> __device__ __forceinline__ float uni<float>(uint32_t w) { return dm::u01_f32(w); }
// log uni<R>(w), and sin and cos of the turn uni<R>(w); FP64 without forming
// the uniform (the same values bit for bit)
template <class R> __device__ __forceinline__ R log_uni(uint32_t w) {
    if constexpr (sizeof(R) == 8) return dm::log_u01(w);
    else return dm::log_pos(dm::u01_f32(w));
}
template <class R> __device__ __forceinline__ void sincos_uni(uint32_t w, R *sn, R *cs) {
    if constexpr (sizeof(R) == 8) dm::sincos_u01(w, sn, cs);
    else dm::sincos_turns(dm::u01_f32(w), sn, cs);
}

// Per-lane ray state.
template <class R, bool REC> struct RayEntry {};
template <class R> struct RayEntry<R, true> {
    V3<R> entry;     // front-face entry point (records)
};
template <class R, bool POL> struct RayPol {};
template <class R> struct RayPol<R, true> {
    V3<R> pol;       // unit polarisation vector (sec. 2.1, 2.2.4)
};
template <class R, bool REC, bool POL = false> struct Ray : RayEntry<R, REC>, RayPol<R, POL> {
    V3<R> p, k;      // crystal-local position, unit direction
    R dist;          // distance to the crystal boundary along k from p
    double E;        // photon energy, keV
    double sa;       // sin(alpha_B) = hc / (2d E); >= 1: no Bragg angle
    float saf, caf;  // sin and cos of alpha_B in FP32, for the acceptance filter
    uint64_t id;
    uint32_t nev, nrefl;
};

// Wave-uniform counters (scalar registers), flushed with one atomic each.
struct WaveCounts {
    uint64_t missed, absorbed, exit_refl, exit_trans, truncated, detected, events, reflections,
        refined;
};

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
           (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ uint32_t popc(uint64_t m) { return (uint32_t)__popcll(m); }
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
// Orders one wave's LDS writes before its later reads by other lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wave queue of rays that have entered the crystal, in LDS (one array
// per field, so the lanes of a wave touch consecutive addresses).  A wave
// starts a batch of candidate rays on all its lanes at once and queues those
// that enter; lanes whose ray has ended take queued rays.  The queue is only
// refilled when empty, so its entries are [head, head + queued) with no
// wrap-around.  While a batch is started, the queue's (then free) slots also
// hold the running rays (slot = lane), so that the candidates can use the
// same registers.
constexpr uint32_t kQueue = 64;
template <class R, bool REC> struct QueueEntry {};   // entry points: record kernels only
template <class R> struct QueueEntry<R, true> {
    R ex[kQueue], ey[kQueue], ez[kQueue];
};
template <class R, bool POL> struct QueuePol {};     // polarisations: extended kernels only
template <class R> struct QueuePol<R, true> {
    R qx[kQueue], qy[kQueue], qz[kQueue];
};
template <class R, bool REC, bool POL = false>
struct RayQueue : QueueEntry<R, REC>, QueuePol<R, POL> {
    using RayT = Ray<R, REC, POL>;
    R px[kQueue], py[kQueue], pz[kQueue], kx[kQueue], ky[kQueue], kz[kQueue], dist[kQueue];
    double E[kQueue], sa[kQueue];
    uint64_t id[kQueue];
    float saf[kQueue], caf[kQueue];
    uint32_t nev[kQueue], nrefl[kQueue];

    // f(array, field) for every field of a ray
    template <class F> __device__ __forceinline__ void fields(RayT &r, F f) {
        f(px, r.p.x); f(py, r.p.y); f(pz, r.p.z);
        f(kx, r.k.x); f(ky, r.k.y); f(kz, r.k.z);
        f(dist, r.dist); f(E, r.E); f(sa, r.sa); f(id, r.id); f(saf, r.saf); f(caf, r.caf);
        f(nev, r.nev); f(nrefl, r.nrefl);
        if constexpr (REC) {
            f(this->ex, r.entry.x); f(this->ey, r.entry.y); f(this->ez, r.entry.z);
        }
        if constexpr (POL) {
            f(this->qx, r.pol.x); f(this->qy, r.pol.y); f(this->qz, r.pol.z);
        }
    }
    __device__ __forceinline__ void put(uint32_t i, RayT &r) {
        MRT_DEV_CHECK(i < kQueue);
        fields(r, [&](auto *a, auto &v) { a[i] = v; });
    }
    __device__ __forceinline__ void take(uint32_t i, RayT &r) {
        MRT_DEV_CHECK(i < kQueue);
        fields(r, [&](auto *a, auto &v) { v = a[i]; });
    }
    // After a batch: lanes with `parked` set take back their ray from slot
    // `lane` while lanes with `queue` set store their candidate `r` at slot
    // `rank`, field by field, all lanes' reads of a field before any write
    // of it.  Only one field of the parked ray is held beside the
    // candidate at a time.
    __device__ __forceinline__ void unpark(uint32_t lane, bool parked, bool queue, uint32_t rank,
                                           RayT &r) {
        MRT_DEV_CHECK(lane < kQueue && (!queue || rank < kQueue));
        fields(r, [&](auto *a, auto &v) {
            const auto t = a[lane];
            wave_sync();
            if (queue) a[rank] = v;
            v = parked ? t : v;
        });
    }
};

// A kind template argument of kAny means: read the kind from the parameter
// block at run time (one wave always traces rays of one parameter block, so
// the branches stay wave-uniform).
constexpr int kAny = -1;

// EXT: the extended inputs (run-time kinds only): a rocking curve whose shift
// and width depend on the photon energy (tables interpolated per event), a
// finite source spot, user-supplied origins, directions or energies, and
// further reflecting planes.  POL: rays carry a polarisation vector, used
// when the user supplies initial polarisations.
template <class R, int GEOM, int MDF, int IRC, bool REC, bool EXT = false, bool POL = EXT>
struct Tracer {
    using RayT = Ray<R, REC, POL>;
    using Queue = RayQueue<R, REC, POL>;
    static constexpr bool kF64 = sizeof(R) == 8;

    static __device__ __forceinline__ bool is_flat(const TraceParams &P) {
        if constexpr (GEOM == kAny) return P.geometry == MRT_GEOMETRY_FLAT;
        else return GEOM == MRT_GEOMETRY_FLAT;
    }
    static __device__ __forceinline__ bool mdf_is(const TraceParams &P, int k) {
        if constexpr (MDF == kAny) return P.mdf == k;
        else return MDF == k;
    }
    static __device__ __forceinline__ bool irc_is(const TraceParams &P, int k) {
        if constexpr (IRC == kAny) return P.irc == k;
        else return IRC == k;
    }

    // ---- crystal geometry (sec. 2.2), in the crystal-local frame ----------
    // Flat: front face z = 0 with the normal +z toward the source, length
    // along x, width along y.  Cylinder: axis z, radius rho = |(x, y)|.
    // (x, y)-plane dot product with an edge normal (whose z is 0).
    static __device__ __forceinline__ R dot_xy(V3<R> a, const double *d, const float *f) {
        const V3<R> b = par3<R>(d, f);
        return a.x * b.x + a.y * b.y;
    }
    // Front-face entry; false on a miss.
    static __device__ __forceinline__ bool entry(const TraceParams &P, V3<R> o, V3<R> k, R &t) {
        if (is_flat(P)) {
            if (!(k.z < R(0))) return false;
            t = -o.z / k.z;
            if (!(t > R(0))) return false;
            const R hx = o.x + t * k.x, hy = o.y + t * k.y;
            return __builtin_fabs(hx) <= par<R>(P.hl, P.f32.hl) && __builtin_fabs(hy) <= par<R>(P.hw, P.f32.hw);
        } else {
            const R a = k.x * k.x + k.y * k.y, b = o.x * k.x + o.y * k.y;
            const R cc = o.x * o.x + o.y * o.y - par<R>(P.R2, P.f32.R2);
            if (!(cc < R(0)) || !(a > R(0))) return false;
            const R disc = b * b - a * cc;
            const R sq = dm::sqrt(disc);
            t = b >= R(0) ? -cc / (b + sq) : (-b + sq) / a;
            const V3<R> h = axpy(o, t, k);
            return __builtin_fabs(h.z) <= par<R>(P.hl, P.f32.hl) && dot_xy(h, P.op, P.f32.op) <= R(0) &&
                   dot_xy(h, P.om, P.f32.om) <= R(0);
        }
    }

    // Distance to the boundary from an inside point along k: the minimum
    // positive crossing over the faces k moves toward.
    static __device__ __forceinline__ R exit_distance(const TraceParams &P, V3<R> p, V3<R> k) {
        R t = R(INFINITY);
        if (is_flat(P)) {
            const R zeta = p.z, xi = p.x, eta = p.y;
            const R kn = k.z, k1 = k.x, k2 = k.y;
            const R hl = par<R>(P.hl, P.f32.hl), hw = par<R>(P.hw, P.f32.hw), T = par<R>(P.T, P.f32.T);
            if (kn > R(0)) t = fminr(t, -zeta / kn);
            if (kn < R(0)) t = fminr(t, (-T - zeta) / kn);
            if (k1 > R(0)) t = fminr(t, (hl - xi) / k1);
            if (k1 < R(0)) t = fminr(t, (-hl - xi) / k1);
            if (k2 > R(0)) t = fminr(t, (hw - eta) / k2);
            if (k2 < R(0)) t = fminr(t, (-hw - eta) / k2);
        } else {
            const R z = p.z, ka = k.z;
            const R a = k.x * k.x + k.y * k.y, b = p.x * k.x + p.y * k.y, r2 = p.x * p.x + p.y * p.y;
            if (a > R(0)) {
                const R co = r2 - par<R>(P.Ro2, P.f32.Ro2);
                R disc = b * b - a * co;
                if (disc < R(0)) disc = R(0);
                const R sq = dm::sqrt(disc);
                const R to = b >= R(0) ? -co / (b + sq) : (-b + sq) / a;
                t = fminr(t, to);
                if (b < R(0)) {
                    const R ci = r2 - par<R>(P.R2, P.f32.R2);
                    const R di = b * b - a * ci;
                    if (di >= R(0)) t = fminr(t, ci / (-b + dm::sqrt(di)));
                }
            }
            const R hl = par<R>(P.hl, P.f32.hl);
            if (ka > R(0)) t = fminr(t, (hl - z) / ka);
            if (ka < R(0)) t = fminr(t, (-hl - z) / ka);
            const R kop = dot_xy(k, P.op, P.f32.op), kom = dot_xy(k, P.om, P.f32.om);
            if (kop > R(0)) t = fminr(t, -dot_xy(p, P.op, P.f32.op) / kop);
            if (kom > R(0)) t = fminr(t, -dot_xy(p, P.om, P.f32.om) / kom);
        }
        return t > R(0) ? t : R(0);
    }

    // ---- mosaic tilt (sec. 2.2.2) ----------------------------------------
    // Radial part: (cos theta, sin theta) of the crystallite normal from the
    // uniform u2, by the inverse of the distribution's radial CDF.
    static __device__ __forceinline__ void vmf(const TraceParams &P, R u, R &ct, R &st) {
        // Eq. MF: v = 1 - cos(theta) = -s^2 log(u + (1 - u) e^{-2/s^2})
        R v = -par<R>(P.vmf_s2, P.f32.vmf_s2) * dm::log_pos(u + (R(1) - u) * par<R>(P.vmf_floor, P.f32.vmf_floor));
        v = v < R(2) ? v : R(2);
        ct = R(1) - v;
        st = dm::sqrt(v * (R(2) - v));
    }
    static __device__ __forceinline__ void lorentz(const TraceParams &P, R q, R &ct, R &st) {
        // bivariate Cauchy in the tangent plane: tan(theta) = g sqrt(1 - q^2) / q
        const R g = par<R>(P.lor_g, P.f32.lor_g);
        const R om = (R(1) - q) * (R(1) + q);
        const R rs = dm::rsqrt(g * g * om + q * q);
        ct = q * rs;
        st = g * dm::sqrt(om) * rs;
    }
    // Local surface frame at a point: N toward the source side, e1 along
    // the length axis (flat) or the cylinder axis, e2 = N x e1.  Flat: the
    // coordinate axes z, x, y.  Cylinder: N = (nx, ny, 0) points to the
    // axis, e1 = z, e2 = (ny, -nx, 0).
    struct Frame {
        R nx, ny;   // the cylinder's N (unused for the flat crystal)
    };
    static __device__ __forceinline__ Frame frame(const TraceParams &P, V3<R> p) {
        if (is_flat(P)) return Frame{R(0), R(0)};
        const R inv = dm::rsqrt(p.x * p.x + p.y * p.y);
        return Frame{-p.x * inv, -p.y * inv};
    }
    // The surface normal alone, as a vector.
    static __device__ __forceinline__ V3<R> normal_at(const TraceParams &P, V3<R> p) {
        if (is_flat(P)) return V3<R>{R(0), R(0), R(1)};
        const Frame f = frame(P, p);
        return V3<R>{f.nx, f.ny, R(0)};
    }
    static __device__ __forceinline__ V3<R> mosaic_normal(const TraceParams &P, R u2, uint32_t w3,
                                                          Frame f) {
        R ct, st;
        if (mdf_is(P, MRT_MOSAIC_GAUSSIAN_VMF)) {
            vmf(P, u2, ct, st);
        } else if (mdf_is(P, MRT_MOSAIC_LORENTZIAN)) {
            lorentz(P, R(1) - u2, ct, st);
        } else if (mdf_is(P, MRT_MOSAIC_PSEUDO_VOIGT)) {
            // Lorentzian with probability eta, else von Mises-Fisher; the two
            // branches share the square root of sin(theta)
            const R eta = par<R>(P.m_eta, P.f32.m_eta);
            R arg, scale;
            if (u2 < eta) {
                const R q = (eta - u2) * par<R>(P.inv_eta, P.f32.inv_eta);
                const R g = par<R>(P.lor_g, P.f32.lor_g);
                const R om = (R(1) - q) * (R(1) + q);
                const R rs = dm::rsqrt(g * g * om + q * q);
                ct = q * rs;
                arg = om;
                scale = g * rs;
            } else {
                const R u = (u2 - eta) * par<R>(P.inv_1meta, P.f32.inv_1meta);
                R v = -par<R>(P.vmf_s2, P.f32.vmf_s2) * dm::log_pos(u + (R(1) - u) * par<R>(P.vmf_floor, P.f32.vmf_floor));
                v = v < R(2) ? v : R(2);
                ct = R(1) - v;
                arg = v * (R(2) - v);
                scale = R(1);
            }
            st = scale * dm::sqrt(arg);
        } else if (mdf_is(P, MRT_MOSAIC_GAUSSIAN)) {
            // regular Gaussian (Eq. Gaussian) as a tangent-plane bivariate
            // normal: tan^2(theta) = 2 s^2 (-ln u), Rayleigh in the radius
            const R t2 = -par<R>(P.gau_2s2, P.f32.gau_2s2) * dm::log_pos(u2);
            ct = dm::rsqrt(R(1) + t2);
            st = dm::sqrt(t2) * ct;
        } else if (mdf_is(P, MRT_MOSAIC_WRAPPED_LORENTZIAN)) {
            // Eq. WL: density in v proportional to 1 / (g^2 + 2 v)
            R v;
            if constexpr (kF64) v = P.wl_half_g2 * ::expm1(u2 * P.wl_z);
            else v = P.f32.wl_half_g2 * ::expm1f(u2 * P.f32.wl_z);
            v = v < R(2) ? v : R(2);
            ct = R(1) - v;
            st = dm::sqrt(v * (R(2) - v));
        } else {
            // Eq. SWL: density in v proportional to 1 / (cosh(G/2) - 1 + v)^2
            R v = dm::div(par<R>(P.swl_k, P.f32.swl_k) * u2, par<R>(P.swl_d, P.f32.swl_d) - R(2) * u2);
            v = v < R(2) ? v : R(2);
            ct = R(1) - v;
            st = dm::sqrt(v * (R(2) - v));
        }
        if (!(P.fwhm > 0.0)) {   // perfect alignment
            ct = R(1);
            st = R(0);
        }
        R sx, cx;
        sincos_uni<R>(w3, &sx, &cx);   // azimuth uniform in turns
        // n = ct N + st (cx e1 + sx e2)
        if (is_flat(P)) return V3<R>{st * cx, st * sx, ct};
        const R ss = st * sx;
        return V3<R>{ct * f.nx + ss * f.ny, ct * f.ny - ss * f.nx, st * cx};
    }

    // ---- rocking curve (sec. 2.2.1): r(x) / R_max at x = Delta - Delta_M ---
    static __device__ __forceinline__ R irc_ratio(const TraceParams &P, const double *lut, double x) {
        if (irc_is(P, MRT_IRC_GAUSSIAN)) {
            if constexpr (kF64) return dm::exp_nonpos(-P.g_k * x * x);
            else return dm::exp_((float)(-P.g_k * x * x));
        } else if (irc_is(P, MRT_IRC_PSEUDO_VOIGT)) {
            // eta L(x)/R(0) + (1 - eta) G(x)/R(0) = A h^2/(h^2 + x^2) + B exp(-k x^2)
            const double x2 = x * x;
            if constexpr (kF64) {
                return P.pv_a * dm::div(P.pv_h2, P.pv_h2 + x2) + P.pv_b * dm::exp_nonpos(-P.g_k * x2);
            } else {
                const float h2 = P.f32.pv_h2, xf = (float)x2;
                return P.f32.pv_a * h2 * dm::rcp(h2 + xf) +
                       P.f32.pv_b * dm::exp_(-P.f32.g_k * xf);
            }
        } else if (irc_is(P, MRT_IRC_LORENTZIAN)) {
            if constexpr (kF64) return dm::div(P.lor_h2, P.lor_h2 + x * x);
            else return P.f32.lor_h2 * dm::rcp((float)(P.lor_h2 + x * x));
        } else if (irc_is(P, MRT_IRC_BOX)) {
            return __builtin_fabs(x) <= P.box_half ? R(1) : R(0);
        } else {
            // table: linear interpolation on equally spaced nodes, 0 outside
            if (!(x >= P.lut_x0 && x <= P.lut_x1)) return R(0);   // also rejects NaN
            const int n = P.lut_n;
            if (x == P.lut_x1) return cvt<R>(lut[n - 1] * P.lut_inv_max);
            const double f = (x - P.lut_x0) * P.lut_scale;
            const int j = (int)__builtin_floor(f);
            if (j >= n - 1) return cvt<R>(lut[n - 1] * P.lut_inv_max);
            const double t = f - (double)j;
            return cvt<R>(((1.0 - t) * lut[j] + t * lut[j + 1]) * P.lut_inv_max);
        }
    }

    // ---- acceptance filter ------------------------------------------------
    // The decision u_acc < r(x) / R_max with x = Delta - Delta_M is first
    // taken from an FP32 estimate of x whose error is below kFilterErr.  The
    // estimate (sin(Delta) = c cos(alpha_B) - sqrt(1 - c^2) sin(alpha_B) in
    // float, then the arcsine series) errs by at most 3.2e-7 rad: the
    // rounding of c = |k.n| to float (3e-8) is multiplied by
    // cos(alpha_B) + c sin(alpha_B) / sqrt(1 - c^2), up to ~10 at the
    // sqrt(1 - c^2) >= 0.1 cutoff, which steep Bragg angles reach; v_sqrt_f32
    // and the truncated series add little.  Measured over Bragg angles of
    // 1-84 deg with the hardware estimates moved by an ulp either way: 3.1e-7.
    // It bounds r over
    // [|x| - kFilterErr, |x| + kFilterErr] with a relative margin for the
    // FP32 curve.  Returns 1 (accept), 0 (reject) or -1 when u_acc falls in
    // that band, in which case the exact FP64 evaluation decides; the result
    // is therefore always the exact one.
    static constexpr float kFilterErr = 2e-6f;
    static __device__ __forceinline__ float ratio_f32(const TraceParams &P, float a) {
        const float a2 = a * a;
        if (irc_is(P, MRT_IRC_GAUSSIAN)) {
            return __builtin_amdgcn_exp2f(-P.f32.g_k_log2e * a2);
        } else if (irc_is(P, MRT_IRC_PSEUDO_VOIGT)) {
            const float h2 = P.f32.pv_h2;
            return P.f32.pv_a * h2 * __builtin_amdgcn_rcpf(__builtin_fmaf(a, a, h2)) +
                   P.f32.pv_b * __builtin_amdgcn_exp2f(-P.f32.g_k_log2e * a2);
        } else {
            const float h2 = P.f32.lor_h2;
            return h2 * __builtin_amdgcn_rcpf(__builtin_fmaf(a, a, h2));
        }
    }
    // Bounds of x (lo, hi of |x|; slo, shi of x) from the FP32 estimate;
    // false when there is none.  With EXT the curve is read at x / s: the
    // bounds are scaled by 1/s (inv_s, rounded to float) and widened by 2^-20
    // relative, which covers the float roundings of inv_s and of the products.
    // sin(Delta) = c cos(alpha_B) - sqrt(1 - c^2) sin(alpha_B) in FP32 from
    // c = |k.n|; false when the normal lies within ~6 deg of k (no bound).
    static __device__ __forceinline__ bool sin_delta_f32(double akn, float saf, float caf,
                                                         float &z) {
        const float c = (float)akn;
        const float cw = __builtin_amdgcn_sqrtf(__builtin_fmaf(-c, c, 1.0f));
        if (!(cw >= 0.1f)) return false;
        z = __builtin_fmaf(c, caf, -cw * saf);
        return true;
    }
    // asin(z) for |z| <= 1/4: its series to z^9 (truncation below 6e-9)
    static __device__ __forceinline__ float asin_small_f32(float z) {
        const float w = z * z;
        float p = 35.0f / 1152.0f;
        p = __builtin_fmaf(p, w, 5.0f / 112.0f);
        p = __builtin_fmaf(p, w, 3.0f / 40.0f);
        p = __builtin_fmaf(p, w, 1.0f / 6.0f);
        return __builtin_fmaf(z * w, p, z);
    }
    static __device__ __forceinline__ bool x_bounds(double akn, float saf, float caf, float shift,
                                                    float inv_s, float &lo, float &hi, float &slo,
                                                    float &shi) {
        float z;
        if (!sin_delta_f32(akn, saf, caf, z)) return false;
        if (__builtin_fabsf(z) <= 0.25f) {
            const float x = asin_small_f32(z) - shift;
            slo = x - kFilterErr;
            shi = x + kFilterErr;
            const float ax = __builtin_fabsf(x);
            lo = ax - kFilterErr;
            hi = ax + kFilterErr;
        } else {
            // |Delta| > asin(1/4)
            const float d = 0.25268025514207865f - kFilterErr;
            slo = z > 0.0f ? d - shift : -INFINITY;
            shi = z > 0.0f ? INFINITY : -d - shift;
            lo = d - __builtin_fabsf(shift);
            hi = INFINITY;
        }
        lo = lo > 0.0f ? lo : 0.0f;
        // (inv_s == 1 scales nothing and needs no margin)
        if (EXT && inv_s != 1.0f) {
            const float up = 1.0f + 0x1p-20f, dn = 1.0f - 0x1p-20f;
            lo *= inv_s * dn;
            hi *= inv_s * up;   // INFINITY stays
            slo *= inv_s;
            shi *= inv_s;
            slo -= __builtin_fabsf(slo) * 0x1p-20f;
            shi += __builtin_fabsf(shi) * 0x1p-20f;
        }
        return true;
    }
    static __device__ __forceinline__ bool outside_table(const TraceParams &P, float slo, float shi) {
        // the table curve is zero outside [x_min, x_max]
        const float x0 = P.f32.lut_x0, x1 = P.f32.lut_x1;
        return shi < x0 - __builtin_fabsf(x0) * 0x1p-20f - 1e-12f ||
               slo > x1 + __builtin_fabsf(x1) * 0x1p-20f + 1e-12f;
    }
    // Bounds [r_lo, r_hi] of the table curve r / R_max over x in [slo, shi]
    // from its envelope: the linear interpolation between two nodes lies
    // between them, so r over the interval lies between the minimum and the
    // maximum of the nodes it reaches, and those lie within the envelope of
    // the buckets holding the first and the last of them.  The node
    // coordinates are widened by 1/16 node, far beyond the float rounding of
    // (x - x_min) x scale (below 1e-3 nodes up to 8192 nodes), and the
    // values by 2^-20 relative, beyond the roundings of the interpolation
    // and of its conversion to float.  false when the interval reaches more
    // than two buckets or lies outside the table.
    static __device__ __forceinline__ bool table_bounds(const TraceParams &P, float slo, float shi,
                                                        float &r_lo, float &r_hi) {
        const float x0 = P.f32.lut_x0, sc = P.f32.lut_scale;
        const int last = P.lut_n - 1;
        const float fa = (slo - x0) * sc - 0.0625f, fb = (shi - x0) * sc + 0.0625f;
        if (!(fa < (float)last) || !(fb >= 0.0f)) return false;
        const int ja = fa > 0.0f ? (int)fa : 0;
        const int jb = fb < (float)last ? (int)fb + 1 : last;
        const int ba = ja >> P.env_shift, bb = jb >> P.env_shift;
        if (bb - ba > 1) return false;
        // each word: (min, max) of a bucket as r / R_max, rounded outward to float
        const uint64_t wa = (uint64_t)__double_as_longlong(P.lut_env[ba]);
        const uint64_t wb = (uint64_t)__double_as_longlong(P.lut_env[bb]);
        const float vlo = __builtin_fminf(__uint_as_float((uint32_t)wa), __uint_as_float((uint32_t)wb));
        const float vhi = __builtin_fmaxf(__uint_as_float((uint32_t)(wa >> 32)),
                                          __uint_as_float((uint32_t)(wb >> 32)));
        r_hi = vhi * (1.0f + 0x1p-20f) + 1e-30f;
        // zero where the interval leaves the table
        r_lo = fa > 0.0f && fb < (float)last ? vlo * (1.0f - 0x1p-20f) : 0.0f;
        return true;
    }
    // The acceptance decision u_acc < r(x) / R_max from the bounds: 1
    // (accept), 0 (reject) or -1 (the exact FP64 evaluation decides).
    static __device__ __forceinline__ int filter(const TraceParams &P, double akn, float saf,
                                                 float caf, float u_acc, float shift,
                                                 float inv_s) {
        if constexpr (EXT) {
            if (P.exact) return -1;   // every decision by the FP64 evaluation
        }
        float lo, hi, slo, shi;
        if (!x_bounds(akn, saf, caf, shift, inv_s, lo, hi, slo, shi)) return -1;
        if (irc_is(P, MRT_IRC_TABLE)) {
            if (outside_table(P, slo, shi)) return 0;
            float r_lo, r_hi;
            if (!table_bounds(P, slo, shi, r_lo, r_hi)) return -1;
            if (u_acc >= r_hi) return 0;
            return u_acc < r_lo ? 1 : -1;
        } else if (irc_is(P, MRT_IRC_BOX)) {
            const float half = P.f32.box_half;
            if (hi < half * (1.0f - 0x1p-20f)) return 1;
            if (lo > half * (1.0f + 0x1p-20f)) return 0;
            return -1;
        } else {
            // r / R_max is even and decreasing in |x|; most candidates are
            // rejected by the upper bound alone, before the lower one
            const float r_hi = ratio_f32(P, lo) * 1.0001f + 1e-30f;
            if (u_acc >= r_hi) return 0;
            const float r_lo = hi < INFINITY ? ratio_f32(P, hi) * 0.9999f : 0.0f;
            return u_acc < r_lo ? 1 : -1;
        }
    }
    // Bounds [r_lo, r_hi] of r(x) / R_max, which lies in [0, 1] ([0, 1]
    // when there is no bound), for sums of curves.
    static __device__ __forceinline__ void ratio_bounds(const TraceParams &P, double akn,
                                                        float saf, float caf, float shift,
                                                        float inv_s, float &r_lo, float &r_hi) {
        r_lo = 0.0f;
        r_hi = 1.0f;
        if constexpr (EXT) {
            // no bound: a plane sum is then always evaluated exactly
            if (P.exact) {
                r_hi = INFINITY;
                return;
            }
        }
        float lo, hi, slo, shi;
        if (!x_bounds(akn, saf, caf, shift, inv_s, lo, hi, slo, shi)) return;
        if (irc_is(P, MRT_IRC_TABLE)) {
            if (outside_table(P, slo, shi)) r_hi = 0.0f;
            else table_bounds(P, slo, shi, r_lo, r_hi);
        } else if (irc_is(P, MRT_IRC_BOX)) {
            const float half = P.f32.box_half;
            if (hi < half * (1.0f - 0x1p-20f)) r_lo = 1.0f;
            else if (lo > half * (1.0f + 0x1p-20f)) r_hi = 0.0f;
        } else {
            r_hi = ratio_f32(P, lo) * 1.0001f + 1e-30f;
            r_lo = hi < INFINITY ? ratio_f32(P, hi) * 0.9999f : 0.0f;
        }
    }

    // Reflection equation of sec. 2.2.4: k - 2 (k.n) n, renormalised.
    static __device__ __forceinline__ V3<R> reflect_dir(const V3<R> &k, double kn, const V3<R> &n) {
        const R two_kn = R(2) * (R)kn;
        const V3<R> ks{k.x - two_kn * n.x, k.y - two_kn * n.y, k.z - two_kn * n.z};
        const R nr = dm::rsqrt(dot(ks, ks));
        return V3<R>{ks.x * nr, ks.y * nr, ks.z * nr};
    }

    // ---- one event (sec. 2.2.3, 2.2.4).  Returns the end status, or -1. ----
    static __device__ __forceinline__ int step(const TraceParams &P, const double *lut, RayT &ry,
                                               bool &reflected, bool &refined) {
        if (ry.nev == P.max_events) return MRT_TRUNCATED;
        const dm::Words w = dm::philox(P.key0, P.key1, ry.nev, (uint32_t)ry.id,
                                       (uint32_t)(ry.id >> 32), 1u);
        ++ry.nev;
        const int exit_status = ry.nrefl ? MRT_EXIT_REFLECTED : MRT_EXIT_TRANSMITTED;
        // free path to the next event at the majorant rate (Eq. AnyEvent),
        // or once the reflection budget is spent to the absorption at mu0
        const bool spent = (int)ry.nrefl >= P.max_refl;
        const R nlog = -log_uni<R>(w.w0);
        if (spent) {
            // Beer-Lambert absorption only
            const R l = nlog * par<R>(P.inv_mu0, P.f32.inv_mu0);
            if (l < ry.dist) {
                ry.p = axpy(ry.p, l, ry.k);
                return MRT_ABSORBED;
            }
            ry.p = axpy(ry.p, ry.dist, ry.k);
            return exit_status;
        }
        const R l = nlog * par<R>(P.inv_mu_tot, P.f32.inv_mu_tot);
        if (l >= ry.dist) {
            ry.p = axpy(ry.p, ry.dist, ry.k);
            return exit_status;
        }
        ry.p = axpy(ry.p, l, ry.k);
        ry.dist -= l;
        const R u1 = uni<R>(w.w1);
        const R pa = par<R>(P.p_a, P.f32.p_a);
        if (u1 < pa) return MRT_ABSORBED;      // absorbed when u < mu0 / mu_tot
        if (!(ry.sa < 1.0)) return -1;         // no Bragg angle: never reflects
        const R u_acc = (u1 - pa) * par<R>(P.inv_1mpa, P.f32.inv_1mpa);

        const V3<R> n = mosaic_normal(P, uni<R>(w.w2), w.w3, frame(P, ry.p));
        // Bragg deviation in FP64, k.n accumulated in FP64 from the components
        const double kn = (double)ry.k.x * (double)n.x + (double)ry.k.y * (double)n.y +
                          (double)ry.k.z * (double)n.z;
        double akn = __builtin_fabs(kn);
        akn = akn < 1.0 ? akn : 1.0;
        int dec;
        bool dep = false;      // the curve depends on the energy (wave-uniform)
        bool planes = false;   // further plane sets or an H-bar ratio (wave-uniform)
        bool polar = false;    // rays carry polarisations (wave-uniform)
        if constexpr (EXT) {
            dep = P.dep_n > 0;
            planes = P.has_planes != 0;
        }
        // with polarisations the reflected direction is needed before the
        // decision (G depends on it)
        V3<R> ksn{};
        if constexpr (POL) {
            polar = P.user_p != nullptr;
            ksn = reflect_dir(ry.k, kn, n);
        }
        // the polarisation factor G = 1 - (p.k_s)^2 (sec. 2.2.3) multiplies
        // the reflection probability when polarisations are tracked
        double pk = 0.0, G = 1.0;
        if constexpr (POL) {
            if (polar) {
                pk = (double)ry.pol.x * (double)ksn.x + (double)ry.pol.y * (double)ksn.y +
                     (double)ry.pol.z * (double)ksn.z;
                G = 1.0 - pk * pk;
            }
        }
        if (planes) {
            // every plane set j and side (sec. 2.2.3): reflect when
            // u sum_j a_j max(1, hbar) < G h(k.n) sum_j a_j r_j(Delta_j) / R_max,
            // h = 1 against the normal (H), hbar along it (H-bar).  The FP32
            // bounds of each r_j / R_max bound the sum; the exact FP64 sum
            // decides only when u falls between them.
            const double h = kn < 0.0 ? 1.0 : P.hbar;
            const double hg = G * h;
            const double lhs = (double)u_acc * P.plane_tot;
            if (!(hg > 0.0)) {
                dec = 0;
            } else {
                float s_lo = 0.0f, s_hi = 0.0f;
                for (int j = 0; j < P.n_planes; ++j) {
                    // sin(alpha_B,j) = sin(alpha_B) 2d / 2d_j; within 1e-9 of 1
                    // the set is taken as unbounded, so the bounds never
                    // disagree with the exact sum about which sets reflect
                    float rl = 0.0f, rh = 0.0f;
                    if (j == 0) {
                        ratio_bounds(P, akn, ry.saf, ry.caf, P.f32.shift, 1.0f, rl, rh);
                    } else {
                        const double sj = ry.sa * P.plane_ratio[j];
                        if (sj < 1.0 - 1e-9) {
                            const float sf = (float)sj;
                            ratio_bounds(P, akn, sf, __builtin_amdgcn_sqrtf(__builtin_fmaf(-sf, sf, 1.0f)),
                                         (float)P.plane_shift[j], (float)P.plane_inv_scale[j], rl, rh);
                        } else if (sj <= 1.0 + 1e-9) {
                            rh = 1.0f;
                        }
                    }
                    const float aj = (float)P.plane_a[j];
                    s_lo += aj * rl;
                    s_hi += aj * rh;
                }
                if (lhs >= hg * ((double)s_hi * (1.0 + 0x1p-20))) {
                    dec = 0;
                } else if (lhs < hg * ((double)s_lo * (1.0 - 0x1p-20))) {
                    dec = 1;
                } else {
                    refined = true;
                    const double a = ::asin(akn);
                    double sum = 0.0;
                    for (int j = 0; j < P.n_planes; ++j) {
                        const double sj = j ? kHC / (P.plane_2d[j] * ry.E) : ry.sa;
                        if (sj < 1.0) {
                            const double x = ((a - ::asin(sj)) - P.plane_shift[j]) / P.plane_scale[j];
                            sum += P.plane_a[j] * irc_ratio(P, lut, x);
                        }
                    }
                    dec = lhs < G * (h * sum) ? 1 : 0;
                }
            }
        } else if (polar) {
            // u < G r / R_max is u / G < r / R_max: the FP32 filter decides on
            // u / G (its 1e-4 relative margins cover the rounding of u / G to
            // float), G <= 0 never reflects, and a box curve's certain accept
            // (r = R_max there) becomes u < G
            double shift = P.shift, scale = 1.0;
            float shf = P.f32.shift, inv_sf = 1.0f;
            if (dep) {
                shift = interp(P.dep, P.dep + P.dep_n, P.dep_n, ry.E);
                scale = interp(P.dep, P.dep + 2 * P.dep_n, P.dep_n, ry.E);
                shf = (float)shift;
                inv_sf = (float)(1.0 / scale);
            }
            if (!(G > 0.0)) {
                dec = 0;
            } else {
                // (FP32-mixed: u / G in float, a reciprocal within an ulp
                // or two, far inside the margins)
                float ug;
                if constexpr (kF64) ug = (float)((double)u_acc / G);
                else ug = (float)u_acc * __builtin_amdgcn_rcpf((float)G);
                dec = filter(P, akn, ry.saf, ry.caf, ug, shf, inv_sf);
                if (dec == 1 && irc_is(P, MRT_IRC_BOX)) dec = (double)u_acc < G ? 1 : 0;
                if (dec < 0) {
                    refined = true;
                    const double x = ((::asin(akn) - ::asin(ry.sa)) - shift) / scale;
                    dec = u_acc < G * irc_ratio(P, lut, x) ? 1 : 0;
                }
            }
        } else if (dep) {
            // Delta_M(E) and the width scale s(E) (sec. 2.2.1): r read at
            // (Delta - Delta_M(E)) / s(E)
            const double shift = interp(P.dep, P.dep + P.dep_n, P.dep_n, ry.E);
            const double scale = interp(P.dep, P.dep + 2 * P.dep_n, P.dep_n, ry.E);
            dec = filter(P, akn, ry.saf, ry.caf, (float)u_acc, (float)shift, (float)(1.0 / scale));
            if (dec < 0) {
                refined = true;
                const double x = ((::asin(akn) - ::asin(ry.sa)) - shift) / scale;
                dec = u_acc < irc_ratio(P, lut, x) ? 1 : 0;
            }
        } else {
            dec = filter(P, akn, ry.saf, ry.caf, (float)u_acc, P.f32.shift, 1.0f);
            if (dec < 0) {
                // exact: Delta = asin|k.n| - alpha_B in FP64 (Eq. BraggLaw)
                refined = true;
                const double x = (::asin(akn) - ::asin(ry.sa)) - P.shift;
                dec = u_acc < irc_ratio(P, lut, x) ? 1 : 0;
            }
        }
        if (dec) {
            if constexpr (POL) {
                ry.k = ksn;
                if (polar) {
                    // polarisation after the reflection (sec. 2.2.4): the
                    // old one with its component along k_s removed, unit
                    const R f = (R)pk, g = dm::rsqrt((R)(1.0 - pk * pk));
                    ry.pol = V3<R>{(ry.pol.x - f * ksn.x) * g, (ry.pol.y - f * ksn.y) * g,
                                   (ry.pol.z - f * ksn.z) * g};
                }
            } else {
                ry.k = reflect_dir(ry.k, kn, n);
            }
            ++ry.nrefl;
            ry.dist = exit_distance(P, ry.p, ry.k);
            reflected = true;
        }
        return -1;
    }

    // ---- source (sec. 2.1) -------------------------------------------------
    // Direction uniform in solid angle inside the cone.
    static __device__ __forceinline__ V3<R> direction(const TraceParams &P, const dm::Words &a) {
        const R v = uni<R>(a.w0) * par<R>(P.vmax, P.f32.vmax);
        const R ct = R(1) - v;
        const R st = dm::sqrt(v * (R(2) - v));
        R sp, cp;
        sincos_uni<R>(a.w1, &sp, &cp);
        const V3<R> ax = par3<R>(P.sa, P.f32.sa), b1 = par3<R>(P.sb1, P.f32.sb1), b2 = par3<R>(P.sb2, P.f32.sb2);
        return V3<R>{ct * ax.x + st * (cp * b1.x + sp * b2.x),
                     ct * ax.y + st * (cp * b1.y + sp * b2.y),
                     ct * ax.z + st * (cp * b1.z + sp * b2.z)};
    }
    // Energy from the spectrum used as a PDF (FP64 in both precisions).
    static __device__ __forceinline__ double energy(const TraceParams &P, const double *cdf,
                                                    const dm::Words &a, uint64_t ray) {
        const double s2 = dm::u01_f64(a.w2), s3 = dm::u01_f64(a.w3);
        if (P.spectrum == MRT_SPECTRUM_UNIFORM) return P.e_min + s2 * P.e_span;
        if (P.spectrum == MRT_SPECTRUM_LINES) {
            int pick = P.n_lines;
            for (int j = 0; j < P.n_lines; ++j)
                if (s2 < P.line_cum[j]) { pick = j; break; }
            if (pick >= P.n_lines) return P.e_min + s3 * P.e_span;
            const dm::Words b = dm::philox(P.key0, P.key1, 1u, (uint32_t)ray, (uint32_t)(ray >> 32), 0u);
            double sg, cg;
            dm::sincos_u01(b.w0, &sg, &cg);
            return P.line_e[pick] + P.line_sig[pick] * dm::sqrt(-2.0 * dm::log_u01(a.w3)) * cg;
        }
        // largest bin b with cdf[b] <= s2, uniform inside the bin
        int lo = 0, hi = P.n_bins - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (cdf[mid] <= s2) lo = mid;
            else hi = mid - 1;
        }
        return P.e_min + ((double)lo + s3) * P.e_span / (double)P.n_bins;
    }

    // ---- records (sec. 3: saved ray data) ------------------------------------
    static __device__ __forceinline__ void write_record(const TraceParams &P, const RayT &ry,
                                                        int status, bool miss, V3<R> end,
                                                        bool detected, int pi, int pj) {
        if constexpr (REC) {
            int64_t idx = -1;
            if (P.records_mode == MRT_RECORDS_ALL) {
                idx = (int64_t)(ry.id - P.first);
            } else if (detected) {
                const unsigned long long slot = atomicAdd(&P.dev_counters[kCRecords], 1ull);
                if (slot < P.rec_cap) idx = (int64_t)slot;
            }
            if (idx < 0) return;
            MRT_DEV_CHECK((uint64_t)idx < P.rec_cap);
            mrt_hit_record *r = &P.records[idx];
            const double nan = __builtin_nan("");
            r->ray_id = ry.id;
            r->energy_kev = ry.E;
            // global coordinates: origin + local vector through the rotation
            const double ex = ry.entry.x, ey = ry.entry.y, ez = ry.entry.z;
            const double qx = end.x, qy = end.y, qz = end.z;
            const double kx = ry.k.x, ky = ry.k.y, kz = ry.k.z;
            for (int c = 0; c < 3; ++c) {
                const double rx = P.rot[0][c], ryy = P.rot[1][c], rz = P.rot[2][c];
                r->entry[c] = miss ? nan : P.origin[c] + (rx * ex + ryy * ey + rz * ez);
                r->end[c] = miss ? nan : P.origin[c] + (rx * qx + ryy * qy + rz * qz);
                r->dir[c] = rx * kx + ryy * ky + rz * kz;
            }
            r->pix_i = pi;
            r->pix_j = pj;
            r->n_events = ry.nev;
            r->n_refl = (uint16_t)ry.nrefl;
            r->status = (uint8_t)status;
            r->detected = detected ? 1 : 0;
        }
    }

    // ---- tables of the photon energy: nodes e (increasing), values q,
    // interpolated linearly at E with the end values held outside, as
    // q_j + (q_{j+1} - q_j) / (e_{j+1} - e_j) * (E - e_j) with separately
    // rounded operations (no fused multiply-add), j the last node <= E.
    static __device__ __forceinline__ double interp(const double *e, const double *q, int n,
                                                    double E) {
        if (n == 1 || !(E > e[0])) return q[0];
        if (!(E < e[n - 1])) return q[n - 1];
        int lo = 0, hi = n - 1;   // e[lo] <= E < e[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (e[mid] <= E) lo = mid;
            else hi = mid;
        }
        const double slope = __ddiv_rn(__dsub_rn(q[lo + 1], q[lo]), __dsub_rn(e[lo + 1], e[lo]));
        return __dadd_rn(q[lo], __dmul_rn(slope, __dsub_rn(E, e[lo])));
    }
    // detector quantum efficiency (sec. 3)
    static __device__ __forceinline__ double qe_weight(const TraceParams &P, double E) {
        return interp(P.qe, P.qe + P.qe_n, P.qe_n, E);
    }

    // ---- end of a ray: detector (sec. 2.3) and images -------------------------
    // Returns true when the ray lands on a pixel.
    static __device__ __forceinline__ bool finish(const TraceParams &P, const RayT &ry, int status) {
        int pi = -1, pj = -1;
        bool detected = false;
        V3<R> end = ry.p;
        if (status == MRT_EXIT_REFLECTED || status == MRT_EXIT_TRANSMITTED) {
            const V3<R> dn = par3<R>(P.dn, P.f32.dn);
            const R kn = dot(ry.k, dn);
            if (kn < R(0)) {
                const V3<R> dP = par3<R>(P.dP, P.f32.dP);
                const R t = dot(sub(dP, ry.p), dn) / kn;
                if (t > R(0)) {
                    const V3<R> h = axpy(ry.p, t, ry.k);
                    const V3<R> d = sub(h, dP);
                    const R fu = dot(d, par3<R>(P.du, P.f32.du)) / par<R>(P.pitch, P.f32.pitch) + par<R>(P.half_nx, P.f32.half_nx);
                    const R fv = dot(d, par3<R>(P.dv, P.f32.dv)) / par<R>(P.pitch, P.f32.pitch) + par<R>(P.half_ny, P.f32.half_ny);
                    const R fi = __builtin_floor(fu), fj = __builtin_floor(fv);
                    if (fi >= R(0) && fj >= R(0) && fi < (R)P.nx && fj < (R)P.ny) {
                        pi = (int)fi;
                        pj = (int)fj;
                        detected = true;
                        end = h;
                        const size_t px = (size_t)pj * (size_t)P.nx + (size_t)pi;
                        MRT_DEV_CHECK(pi < P.nx && pj < P.ny && P.counts != nullptr);
                        atomicAdd(&P.counts[px], 1u);
                        if (P.energy) {
                            const double ew = P.qe_n > 0 ? __dmul_rn(ry.E, qe_weight(P, ry.E)) : ry.E;
                            atomicAdd(&P.energy[px], (unsigned long long)__builtin_rint(ew * 1e6));
                        }
                    }
                }
            }
        }
        write_record(P, ry, status, false, end, detected, pi, pj);
        return detected;
    }

    // Local components of a global direction (rows of the frame's rotation).
    static __device__ __forceinline__ void local(const TraceParams &P, const double *g, double *l) {
        for (int r = 0; r < 3; ++r) l[r] = P.rot[r][0] * g[0] + P.rot[r][1] * g[1] + P.rot[r][2] * g[2];
    }

    // The photon energy: the user's array, else drawn from the spectrum.
    static __device__ __forceinline__ double ray_energy(const TraceParams &P, const double *cdf,
                                                        const dm::Words &a, uint64_t ray) {
        if (P.user_e) return P.user_e[ray - P.first];
        return energy(P, cdf, a, ray);
    }
    // Offset (x, y) of a ray's origin in the spot plane from the uniforms u,
    // v of words wu, wv: Gaussian, sigma_x sqrt(-2 ln u) (cos, sin)(2 pi v)
    // (Box-Muller), or uniform over the disk of radius sigma_x, sigma_x
    // sqrt(u) (cos, sin)(2 pi v).
    static __device__ __forceinline__ void spot_offset(const TraceParams &P, uint32_t wu,
                                                       uint32_t wv, double &x, double &y) {
        double s, c;
        dm::sincos_u01(wv, &s, &c);
        if (P.spot_kind == MRT_SPOT_GAUSSIAN) {
            const double r = dm::sqrt(-2.0 * dm::log_u01(wu));
            x = P.spot_sigma[0] * r * c;
            y = P.spot_sigma[1] * r * s;
        } else {
            const double r = P.spot_sigma[0] * dm::sqrt(dm::u01_f64(wu));
            x = r * c;
            y = r * s;
        }
    }

    // Start a ray: source direction and front-face entry.  On a hit, the
    // energy, Bragg angle and first exit distance follow and true is
    // returned; a miss is retired here (record written) and false returned.
    // Every instance takes the source spot and the user's origins and
    // directions, by a wave-uniform branch once per ray start: they change
    // nothing after it.
    static __device__ __forceinline__ bool start(const TraceParams &P, const double *cdf,
                                                 uint64_t ray, RayT &ry) {
        const dm::Words a = dm::philox(P.key0, P.key1, 0u, (uint32_t)ray, (uint32_t)(ray >> 32), 0u);
        V3<R> o, k;
        if (P.user_o || P.user_k || P.spot_kind != MRT_SPOT_POINT) {
            const size_t i = (size_t)(ray - P.first);
            double od[3] = {P.so[0], P.so[1], P.so[2]};
            if (P.user_o) {
                // user origins, global coordinates
                const double g[3] = {P.user_o[3 * i] - P.origin[0], P.user_o[3 * i + 1] - P.origin[1],
                                     P.user_o[3 * i + 2] - P.origin[2]};
                local(P, g, od);
            } else if (P.spot_kind != MRT_SPOT_POINT) {
                // finite source spot (sec. 4.2): words 1, 2 of the source's second draw
                const dm::Words b = dm::philox(P.key0, P.key1, 1u, (uint32_t)ray, (uint32_t)(ray >> 32), 0u);
                double x, y;
                spot_offset(P, b.w1, b.w2, x, y);
                for (int c = 0; c < 3; ++c) od[c] += x * P.spot_u[c] + y * P.spot_v[c];
            }
            o = V3<R>{cvt<R>(od[0]), cvt<R>(od[1]), cvt<R>(od[2])};
            if (P.user_k) {
                double kd[3];
                local(P, &P.user_k[3 * i], kd);
                k = V3<R>{cvt<R>(kd[0]), cvt<R>(kd[1]), cvt<R>(kd[2])};
            } else {
                k = direction(P, a);
            }
        } else {
            o = par3<R>(P.so, P.f32.so);
            k = direction(P, a);
        }
        ry.id = ray;
        ry.k = k;
        ry.nev = 0;
        ry.nrefl = 0;
        if constexpr (POL) {
            if (P.user_p) {
                const size_t i = (size_t)(ray - P.first);
                double pd[3];
                local(P, &P.user_p[3 * i], pd);
                ry.pol = V3<R>{cvt<R>(pd[0]), cvt<R>(pd[1]), cvt<R>(pd[2])};
            } else {
                ry.pol = V3<R>{R(0), R(0), R(0)};
            }
        }
        R t;
        const bool hit = entry(P, o, k, t);
        if (!hit) {
            if constexpr (REC) {
                ry.E = ray_energy(P, cdf, a, ray);
                ry.p = o;
                write_record(P, ry, MRT_MISS, true, o, false, -1, -1);
            }
            return false;
        }
        ry.p = axpy(o, t, k);
        if constexpr (REC) ry.entry = ry.p;
        ry.E = ray_energy(P, cdf, a, ray);
        const double s = kHC / (P.two_d * ry.E);   // Eq. BraggLaw: sin(alpha_B)
        ry.sa = s < 1.0 ? s : 2.0;
        ry.saf = (float)s;
        ry.caf = s < 1.0 ? (float)dm::sqrt(fma(-s, s, 1.0)) : 0.0f;
        ry.dist = exit_distance(P, ry.p, ry.k);
        return true;
    }
};

__device__ __forceinline__ void flush(const TraceParams &P, WaveCounts &c) {
    if (__lane_id() == 0) {
        unsigned long long *d = P.dev_counters;
        if (c.missed) atomicAdd(&d[kCMissed], (unsigned long long)c.missed);
        if (c.absorbed) atomicAdd(&d[kCAbsorbed], (unsigned long long)c.absorbed);
        if (c.exit_refl) atomicAdd(&d[kCExitReflected], (unsigned long long)c.exit_refl);
        if (c.exit_trans) atomicAdd(&d[kCExitTransmitted], (unsigned long long)c.exit_trans);
        if (c.truncated) atomicAdd(&d[kCTruncated], (unsigned long long)c.truncated);
        if (c.detected) atomicAdd(&d[kCDetected], (unsigned long long)c.detected);
        if (c.events) atomicAdd(&d[kCEvents], (unsigned long long)c.events);
        if (c.reflections) atomicAdd(&d[kCReflections], (unsigned long long)c.reflections);
        if (c.refined) atomicAdd(&d[kCRefined], (unsigned long long)c.refined);
    }
    c = WaveCounts{};
}

// ---------------------------------------------------------------------------
// The persistent ray loop of one wave.  Lanes whose ray has ended take rays
// from the wave's queue `q` (RayQueue).  When the queue is empty, all 64
// lanes start the next 64 ray ids of the wave's current chunk [next, end) at
// once, which `claim(next, end)` renews (false when no rays are left); rays
// that miss the crystal are counted and retired there, and those that enter
// are queued.  So starting a ray costs one lane of a full-width batch, and
// the lanes that take queued rays are never left idle by misses.  Events run
// until refill_at lanes are idle, then the wave refills; once the rays run
// out the remaining lanes drain.  With the FP32-mixed kernels the detector
// and record work of the rays that ended also runs at the refill.  The
// wave's counters (64-bit, in scalar registers) are added to P.dev_counters
// once, at the end: flushing them at every chunk claim put nine atomics on
// the same nine addresses per chunk, which throttled workloads whose chunks
// go fast (most rays missing).
// ---------------------------------------------------------------------------
template <class T, bool kDefer, class Claim, class Q>
__device__ __forceinline__ void trace_loop(const TraceParams &P, const double *lut,
                                           const double *cdf, Claim &claim, Q &q) {
    typename T::RayT ry;
    bool active = false;
    bool pending = false;         // the lane's ray has ended and awaits finish()
    int pend_status = 0;
    WaveCounts cnt{};
    uint64_t next = 0, end = 0;   // wave-uniform cursor of ray ids
    bool more = true;             // wave-uniform: unclaimed rays remain
    uint32_t head = 0, queued = 0;   // wave-uniform: the queue holds [head, head + queued)
    const uint32_t refill_at = P.refill_idle < 1u ? 1u : (P.refill_idle > 64u ? 64u : P.refill_idle);
    const uint32_t lane = __lane_id();

    // kDefer: the detector and record work of an ended ray waits for the
    // next refill, where it runs for all the rays that ended since, rather
    // than at each step for the one or two lanes whose ray ends there.
    for (;;) {
        if constexpr (kDefer) {
            bool det = false;
            if (pending) {
                det = T::finish(P, ry, pend_status);
                pending = false;
            }
            cnt.detected += popc(ballot(det));
        }
        for (;;) {
            const uint64_t idle = ballot(!active);
            const uint32_t nidle = popc(idle);
            if (nidle == 0 || (nidle < refill_at && idle != ~0ull)) break;
            if (queued == 0) {
                if (!more) break;
                if (next == end && !claim(next, end)) {
                    more = false;
                    break;
                }
                const uint64_t avail = end - next;
                const uint32_t width = avail < kQueue ? (uint32_t)avail : kQueue;
                // the running rays wait in the empty queue while every lane
                // starts a candidate in the same registers
                if (active) q.put(lane, ry);
                bool hit = false, missed = false;
                if (lane < width) {
                    hit = T::start(P, cdf, next + lane, ry);
                    missed = !hit;
                }
                const uint64_t hits = ballot(hit);
                q.unpark(lane, active, hit, lane_rank(hits), ry);
                cnt.missed += popc(ballot(missed));
                head = 0;
                queued = popc(hits);
                next += width;
                wave_sync();
                continue;
            }
            if (!active) {
                const uint32_t r = lane_rank(idle);
                if (r < queued) {
                    q.take(head + r, ry);
                    active = true;
                }
            }
            const uint32_t take = queued < nidle ? queued : nidle;
            head += take;
            queued -= take;
            MRT_DEV_CHECK(head + queued <= kQueue);
        }
        const uint64_t act0 = ballot(active);
        if (act0 == 0) {
            if (!more && queued == 0) break;
            continue;
        }

        // refill_at is in [1, 64], so keep is at least 1
        const uint32_t keep = more || queued ? 65u - refill_at : 1u;
        for (;;) {
            bool reflected = false, refined = false;
            int status = -1;
            const bool was_active = active;
            if (active) status = T::step(P, lut, ry, reflected, refined);
            const bool ended = status >= 0;
            bool det = false;
            if (ended) {
                if constexpr (kDefer) {
                    pending = true;
                    pend_status = status;
                } else {
                    det = T::finish(P, ry, status);
                }
                active = false;
            }
            // every step draws one event except a truncation, which ends the ray first
            cnt.events += popc(ballot(was_active && status != MRT_TRUNCATED));
            if (ballot(reflected)) cnt.reflections += popc(ballot(reflected));
            cnt.refined += popc(ballot(refined));
            const uint64_t endm = ballot(ended);
            if (endm) {
                cnt.absorbed += popc(ballot(ended && status == MRT_ABSORBED));
                cnt.exit_refl += popc(ballot(ended && status == MRT_EXIT_REFLECTED));
                cnt.exit_trans += popc(ballot(ended && status == MRT_EXIT_TRANSMITTED));
                cnt.truncated += popc(ballot(ended && status == MRT_TRUNCATED));
                if constexpr (!kDefer) cnt.detected += popc(ballot(det));
            }
            if (popc(ballot(active)) < keep) break;
        }
    }
    flush(P, cnt);
}

// Chunks of a ray range, claimed from a global cursor.  kPeek (serving):
// the cursor only grows, so a plain read at or past the end proves the range
// exhausted without the atomic.  A serving wave visits every item of its
// round, and the read-modify-writes of waves arriving at finished items
// serialised on the items' cursors (FP32-mixed serving 8% faster without
// them).  The one-call kernels claim without it: their ranges run out once,
// and the extra read changed the scheduling of their event loop (FP32-mixed
// 5% slower).
template <bool kPeek>
struct ClaimRange {
    unsigned long long *cursor;
    uint64_t first, n;
    uint32_t chunk;
    __device__ __forceinline__ bool operator()(uint64_t &next, uint64_t &end) {
        unsigned long long base = 0;
        if (__lane_id() == 0) {
            if constexpr (kPeek) {
                base = __hip_atomic_load(cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (base < n) base = atomicAdd(cursor, (unsigned long long)chunk);
            } else {
                base = atomicAdd(cursor, (unsigned long long)chunk);
            }
        }
        base = uniform64(base);
        if (base >= n) return false;
        next = first + base;
        end = first + (base + chunk < n ? base + chunk : n);
        return true;
    }
};
using RangeClaim = ClaimRange<false>;   // one call's range
using ItemClaim = ClaimRange<true>;     // a serving item's range

// ---------------------------------------------------------------------------
// Serving: the waves of one launch trace a round's items (one per request,
// each with its own chunk cursor).  Wave `wave` of `n_waves` starts at the
// item that holds ray position wave * total / n_waves of the round, so each
// item starts with a share of the waves proportional to its rays; the wave
// claims chunks of that item exactly as the one-call kernel claims chunks of
// its range (no drain between chunks), and when the item is exhausted it
// moves on to the following items in turn, helping wherever rays are left,
// until it has visited every item.  The wave index must be wave-uniform.
// The loop head holds no lane-conditional code before trace_loop's first
// wave operation, so the compiler cannot split the wave across the
// back-edge (the counter flush that ends trace_loop is lane-0-only).
// ---------------------------------------------------------------------------
template <class Run>
__device__ __forceinline__ void serve_waves(const TraceParams *__restrict__ slots,
                                            const ServeItem *__restrict__ items, uint32_t n_items,
                                            uint64_t total, unsigned long long *__restrict__ cursors,
                                            uint32_t wave, uint32_t n_waves, const Run &run) {
    if (n_items == 0 || n_waves == 0) return;
    // first item: the last one whose start is at or before the position
    const uint64_t pos = (uint64_t)wave * total / n_waves;
    uint32_t lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (items[mid].start <= pos) lo = mid;
        else hi = mid - 1;
    }
    for (uint32_t k = 0; k < n_items; ++k) {
        const uint32_t i = lo + k < n_items ? lo + k : lo + k - n_items;
        const ServeItem it = items[i];
        MRT_DEV_CHECK(i < n_items && it.slot >= 0);
        const TraceParams &P = slots[it.slot];
        ItemClaim claim{&cursors[i], it.first, it.count, it.chunk};
        run(P, claim);
    }
}

// The loop of one Tracer T (kinds as T fixes them) over an item's rays.
template <class T, bool kDefer, class Q>
struct LoopRun {
    Q &q;
    __device__ __forceinline__ void operator()(const TraceParams &P, ItemClaim &claim) const {
        trace_loop<T, kDefer>(P, P.lut, P.bin_cdf, claim, q);
    }
};

// The loop specialised for an item's geometry, mosaic and rocking-curve
// kinds (wave-uniform scalar loads from its parameter block), chosen by a
// uniform switch per item: the serving kernel then runs the plain kernels'
// code for every request.
template <class R, bool kDefer, int G, int M, int I, class Q>
__device__ __forceinline__ void run_kinds(const TraceParams &P, ItemClaim &c, Q &q) {
    trace_loop<Tracer<R, G, M, I, false>, kDefer>(P, P.lut, P.bin_cdf, c, q);
}
template <class R, bool kDefer, int G, int M, class Q>
__device__ __forceinline__ void run_irc(const TraceParams &P, ItemClaim &c, Q &q) {
    switch (P.irc) {
    case 0: run_kinds<R, kDefer, G, M, 0>(P, c, q); break;
    case 1: run_kinds<R, kDefer, G, M, 1>(P, c, q); break;
    case 2: run_kinds<R, kDefer, G, M, 2>(P, c, q); break;
    case 3: run_kinds<R, kDefer, G, M, 3>(P, c, q); break;
    default: run_kinds<R, kDefer, G, M, 4>(P, c, q); break;
    }
}
template <class R, bool kDefer, int G, class Q>
__device__ __forceinline__ void run_mdf(const TraceParams &P, ItemClaim &c, Q &q) {
    switch (P.mdf) {
    case 0: run_irc<R, kDefer, G, 0>(P, c, q); break;
    case 1: run_irc<R, kDefer, G, 1>(P, c, q); break;
    case 2: run_irc<R, kDefer, G, 2>(P, c, q); break;
    case 3: run_irc<R, kDefer, G, 3>(P, c, q); break;
    case 4: run_irc<R, kDefer, G, 4>(P, c, q); break;
    default: run_irc<R, kDefer, G, 5>(P, c, q); break;
    }
}
template <class R, bool kDefer, class Q>
struct KindRun {
    Q &q;
    __device__ __forceinline__ void operator()(const TraceParams &P, ItemClaim &claim) const {
        if (P.geometry == MRT_GEOMETRY_FLAT) run_mdf<R, kDefer, MRT_GEOMETRY_FLAT>(P, claim, q);
        else run_mdf<R, kDefer, MRT_GEOMETRY_CYLINDER>(P, claim, q);
    }
};

// ---------------------------------------------------------------------------
// Persistent trace kernel of one call (sec. 2; rays [P.first, P.first + P.n)).
//
// The parameter block is the kernel's by-value argument, read through the
// kernel-argument segment pointer so that each field is a scalar load where
// it is used.  Read as a by-value argument, the whole block is loaded into
// scalar registers at entry and the pressure spills them into vector
// register lanes (FP64 von Hamos kernel: 111 -> 87 VGPRs).  The rocking-curve
// table and the spectrum CDF are read from device memory, where they stay
// cache-resident (at most 32 + 8 KB): staging them in LDS capped occupancy
// at 4 waves per SIMD (40 KB per workgroup), and LDS reads share the wait
// counter of the scalar parameter loads; the stress workload ran 10-11%
// faster without it in both precisions.
// ---------------------------------------------------------------------------
// At least 6 waves per SIMD for the FP64 flat-crystal instances (about 80
// VGPRs, a few spilled): flat HOPG and the stress workload 2-3% faster; the
// FP64 cylinder instances ran 2% slower so bound, and keep 5.
template <class R, int GEOM>
constexpr int kTraceMinWaves = sizeof(R) == 8 && GEOM == MRT_GEOMETRY_FLAT ? 6 : 1;
template <class R, int GEOM, int MDF, int IRC, bool REC>
__global__ void __launch_bounds__(256, (kTraceMinWaves<R, GEOM>)) trace_kernel(const TraceParams P) {
    using T = Tracer<R, GEOM, MDF, IRC, REC>;
    const TraceParams &Q = *(const TraceParams *)__builtin_amdgcn_kernarg_segment_ptr();
    RangeClaim claim{Q.chunk_counter, Q.first, Q.n, Q.chunk};
    // one ray queue per wave (at most 4 waves per workgroup)
    __shared__ RayQueue<R, REC> queues[4];
    RayQueue<R, REC> &q = queues[uniform(threadIdx.x >> 6)];
    // The ended rays' detector and record work waits for the refill
    // (FP32-mixed: 2-16% faster; FP64: 2-10% faster).
    trace_loop<T, true>(Q, Q.lut, Q.bin_cdf, claim, q);
}

// The same loop with the extended inputs (energy-dependent rocking curve,
// polarisations, further plane sets), specialised for the kinds like the
// plain kernels (reading the kinds at run time made these kernels 6-17%
// slower).
// One wave per SIMD more than the compiler's choice: 5 in FP64 (at most 96
// VGPRs), 6 in FP32-mixed (at most 80).  Plane sets run 5% (FP64) and 3.5%
// faster, polarisation 0.5% and 3.3%, the energy-dependent curve 2.9%
// slower in FP64 and 0.6% faster in FP32-mixed (von Hamos, 5e7 rays).
template <class R>
constexpr int kExtMinWaves = sizeof(R) == 8 ? 5 : 6;
template <class R, int GEOM, int MDF, int IRC, bool REC>
__global__ void __launch_bounds__(256, (kExtMinWaves<R>)) trace_kernel_ext(const TraceParams P) {
    using T = Tracer<R, GEOM, MDF, IRC, REC, true>;
    const TraceParams &Q = *(const TraceParams *)__builtin_amdgcn_kernarg_segment_ptr();
    RangeClaim claim{Q.chunk_counter, Q.first, Q.n, Q.chunk};
    __shared__ typename T::Queue queues[4];
    typename T::Queue &q = queues[uniform(threadIdx.x >> 6)];
    trace_loop<T, !T::kF64>(Q, Q.lut, Q.bin_cdf, claim, q);
}

}  // namespace tk

// Kernel lookup of one translation unit: precision and geometry fixed,
// mosaic kind x rocking-curve kind x records; K is trace_kernel or
// trace_kernel_ext.
#define MRT_KERNEL_TABLE(FN, K, R, GEOM)                                                      \
    const void *FN(int mdf, int irc, bool rec) {                                               \
        using namespace tk;                                                                   \
        static const void *const t[6][5][2] = {                                               \
            MRT_ROW(K, R, GEOM, 0), MRT_ROW(K, R, GEOM, 1), MRT_ROW(K, R, GEOM, 2),           \
            MRT_ROW(K, R, GEOM, 3), MRT_ROW(K, R, GEOM, 4), MRT_ROW(K, R, GEOM, 5)};          \
        if (mdf < 0 || mdf > 5 || irc < 0 || irc > 4) return nullptr;                         \
        return t[mdf][irc][rec ? 1 : 0];                                                      \
    }
#define MRT_TRACE_TABLE(FN, R, GEOM) MRT_KERNEL_TABLE(FN, trace_kernel, R, GEOM)
#define MRT_EXT_TABLE(FN, R, GEOM) MRT_KERNEL_TABLE(FN, trace_kernel_ext, R, GEOM)
#define MRT_PAIR(K, R, GEOM, M, I) {(const void *)K<R, GEOM, M, I, false>, (const void *)K<R, GEOM, M, I, true>}
#define MRT_ROW(K, R, GEOM, M)                                                                \
    {MRT_PAIR(K, R, GEOM, M, 0), MRT_PAIR(K, R, GEOM, M, 1), MRT_PAIR(K, R, GEOM, M, 2),       \
     MRT_PAIR(K, R, GEOM, M, 3), MRT_PAIR(K, R, GEOM, M, 4)}

}  // namespace mrt
