// The paper's own event model (sec. 2.2.3, 2.2.4), FP64: free paths at
// mu0 + gamma0 sigma_H(alpha) + gamma0 sigma_anti-H(-alpha) (Eq. AnyEvent)
// with gamma0 sigma from the psi quadrature of Eq. SimpleReflXsection,
// absorption with probability mu0 / mu_eff, and reflections off a crystallite
// whose (psi, Delta) is drawn by a Metropolis-within-Gibbs sampler from the
// integrand of Eq. ReflXsection and oriented by the two rotations of sec.
// 2.2.2.  The reflection strength is the stepping model's:
// Q R(Delta) = r(Delta - Delta_M) / h, with the polarisation factor folded
// into r's peak.  Source, entry, exit distances, local frame, rocking curve
// and detector are the stepping kernels' (Tracer).
//
// The sampler's burn-in (hundreds of sweeps) costs far more than an event,
// so a lane whose event is a reflection parks, and the parked lanes of a
// wave run the sampler together once mwg_batch of them wait or no lane can
// take another event.
#include "trace_impl.h"

namespace mrt {
namespace tk {

template <int GEOM, bool REC, bool POL = false, bool PLANES = false>
struct MwgTracer : Tracer<double, GEOM, kAny, kAny, REC, true, POL> {
    // the base's start() with the extended inputs (source spot, user ray
    // arrays); its event code, which the energy-dependent curve would
    // change, is not used here.  POL: rays carry polarisations (the user's),
    // and the cross-section and the sampler's target carry the polarisation
    // factor (Eqs. SimpleReflXsectionPol, ReflXsectionPol).  PLANES: the
    // antiparallel planes' strength and further plane sets (sec. 2.2.3,
    // closing paragraphs): the attenuation sums every set and side, and the
    // reflecting set and side are drawn by their shares; also the
    // energy-dependent curve, as the main set's per-photon shift and scale.
    using B = Tracer<double, GEOM, kAny, kAny, REC, true, POL>;
    using RayT = typename B::RayT;

    // sin and cos of an angle within a turn, by the table-driven sin/cos of
    // turns (22 issue slots for both; the radian library forms cost ~128 each)
    static __device__ __forceinline__ double sin_(double x) {
        double s, c;
        dm::sincos_turns(x * kInv2Pi, &s, &c);
        return s;
    }
    static __device__ __forceinline__ double cos_(double x) {
        double s, c;
        dm::sincos_turns(x * kInv2Pi, &s, &c);
        return c;
    }
    static __device__ __forceinline__ void sincos_(double x, double *s, double *c) {
        dm::sincos_turns(x * kInv2Pi, s, c);
    }

    // ---- mosaic densities per steradian at v = 1 - cos(theta) ----------
    template <int K> static __device__ __forceinline__ double density(const TraceParams &P, double v) {
        if constexpr (K == MRT_MOSAIC_GAUSSIAN_VMF) {
            return P.vmf_norm * dm::exp_nonpos(-P.vmf_kappa * v);
        } else if constexpr (K == MRT_MOSAIC_LORENTZIAN) {
            const double c = 1.0 - v;
            if (!(c > 0.0)) return 0.0;
            // q^(-3/2) from one reciprocal square root
            const double q = v * (2.0 - v) + P.cau_g2 * c * c;
            const double rq = dm::rsqrt(q);
            return P.cau_norm * (rq * rq * rq);
        } else if constexpr (K == MRT_MOSAIC_PSEUDO_VOIGT) {
            return P.m_eta * density<MRT_MOSAIC_LORENTZIAN>(P, v) +
                   (1.0 - P.m_eta) * density<MRT_MOSAIC_GAUSSIAN_VMF>(P, v);
        } else if constexpr (K == MRT_MOSAIC_WRAPPED_LORENTZIAN) {
            return P.wl_norm / (P.wl_g2 + 2.0 * v);
        } else if constexpr (K == MRT_MOSAIC_GAUSSIAN) {
            // the tangent-plane Gaussian at tan^2(theta) = v (2 - v) / c^2,
            // times the gnomonic area ratio 1 / c^3; zero on the far side
            const double c = 1.0 - v;
            if (!(c > 0.0)) return 0.0;
            const double ic = dm::rcp(c);
            return P.gau_norm * (ic * ic * ic) *
                   dm::exp_nonpos(-P.gau_inv2s2 * (v * (2.0 - v)) * (ic * ic));
        } else {
            const double d = P.swl_a + v;
            return P.swl_norm / (d * d);
        }
    }
    static __device__ __forceinline__ double density_any(const TraceParams &P, double v) {
        switch (P.mdf) {
        case MRT_MOSAIC_GAUSSIAN_VMF: return density<MRT_MOSAIC_GAUSSIAN_VMF>(P, v);
        case MRT_MOSAIC_LORENTZIAN: return density<MRT_MOSAIC_LORENTZIAN>(P, v);
        case MRT_MOSAIC_PSEUDO_VOIGT: return density<MRT_MOSAIC_PSEUDO_VOIGT>(P, v);
        case MRT_MOSAIC_WRAPPED_LORENTZIAN: return density<MRT_MOSAIC_WRAPPED_LORENTZIAN>(P, v);
        case MRT_MOSAIC_GAUSSIAN: return density<MRT_MOSAIC_GAUSSIAN>(P, v);
        default: return density<MRT_MOSAIC_SPHERICAL_WRAPPED_LORENTZIAN>(P, v);
        }
    }

    // ---- psi integrals of Eq. SimpleReflXsection for alpha and -alpha ----
    // Trapezoid rule over psi_j = pi (j / M)^3 on [0, pi], doubled (the
    // integrand is even); v = 2 sin^2((a - beta)/2) + 2 cos(a) cos(beta)
    // sin^2(psi/2) by Eq. ThetaPsi.  The table holds (sin^2(psi_j / 2), w_j)
    // per node, w_j the node's trapezoid weight (half the sum of its two
    // intervals); its index is wave-uniform (scalar loads).  The von
    // Mises-Fisher density exp(-kappa v) at v = v0 + b is exp(-kappa v0)
    // exp(-kappa b): one exponential per node serves the H and the anti-H
    // planes (also for the pseudo-Voigt mosaic's vMF part).  With
    // polarisation (C2) the same rule also sums W cos(2 psi) on [0, pi] (i2h,
    // i2a; the table w_j cos(2 psi_j) follows the node table): W is even, so
    // int W G over [-pi, pi] with G = 1 - S cos^2(phi' - psi) is (1 - S/2)
    // int W - S cos(2 phi') int_0^pi W cos(2 psi).
    template <int K, bool C2>
    static __device__ __forceinline__ void psi_pair(const TraceParams &P, double alpha, double beta,
                                                    double &ih, double &ia, double &i2h,
                                                    double &i2a) {
        constexpr bool kVmf = K == MRT_MOSAIC_GAUSSIAN_VMF || K == MRT_MOSAIC_PSEUDO_VOIGT;
        const double sh = sin_((alpha - beta) / 2.0), sa = sin_((-alpha - beta) / 2.0);
        const double v0h = 2.0 * sh * sh, v0a = 2.0 * sa * sa;
        const double cc = 2.0 * cos_(alpha) * cos_(beta);
        double eh = 0.0, ea = 0.0;   // the vMF parts at v0h, v0a
        if constexpr (kVmf) {
            const double c = K == MRT_MOSAIC_PSEUDO_VOIGT ? (1.0 - P.m_eta) * P.vmf_norm : P.vmf_norm;
            eh = c * dm::exp_nonpos(-P.vmf_kappa * v0h);
            ea = c * dm::exp_nonpos(-P.vmf_kappa * v0a);
        }
        // The Lorentzian density cau_norm q^(-3/2), zero from v = 1 on, with
        // q(v) = v (2 - v) + g^2 (1 - v)^2 = g^2 + (1 - g^2)(2v - v^2): at v =
        // v0 + cc t, t = sin^2(psi_j / 2), a quadratic q = l0 + l1 t + l2 t^2
        // with l0 = q(v0), l1 = 2 (1 - g^2) cc (1 - v0), l2 = -(1 - g^2) cc^2
        // (the two terms in t differ in sign by at most a factor 2 below v =
        // 1, so nothing cancels), and v < 1 while cc t < 1 - v0.
        constexpr bool kLor = K == MRT_MOSAIC_LORENTZIAN || K == MRT_MOSAIC_PSEUDO_VOIGT;
        struct Lor {
            double l0, l1, l2, room;
        };
        auto lor_at = [&](double v0) {
            const double k = 1.0 - P.cau_g2, c0 = 1.0 - v0;
            return Lor{v0 * (2.0 - v0) + P.cau_g2 * c0 * c0, 2.0 * k * cc * c0, -k * (cc * cc), c0};
        };
        const double lor_scale = K == MRT_MOSAIC_PSEUDO_VOIGT ? P.m_eta * P.cau_norm : P.cau_norm;
        auto lor = [&](const Lor &L, double t, double b) {
            const double rq = dm::rsqrt(fma(fma(L.l2, t, L.l1), t, L.l0));
            return b < L.room ? (lor_scale * rq) * (rq * rq) : 0.0;
        };
        Lor lh{}, la{};
        if constexpr (kLor) {
            lh = lor_at(v0h);
            la = lor_at(v0a);
        }
        // the densities at v0h + cc t and v0a + cc t.  exp(-kappa b) is
        // exactly 0 from kappa b = 746 on (below half the smallest
        // subnormal), and b grows with the node: the exponential is a branch
        // of its own, which the wave skips once every lane is past that point
        // (about three quarters of the nodes for a 0.1 deg mosaic)
        auto node = [&](double t, double &gh, double &ga) {
            const double b = cc * t;
            if constexpr (kVmf) {
                double e = 0.0;
                if (P.vmf_kappa * b <= 746.0) e = dm::exp_nonpos(-P.vmf_kappa * b);
                gh = eh * e;
                ga = ea * e;
                if constexpr (K == MRT_MOSAIC_PSEUDO_VOIGT) {
                    gh += lor(lh, t, b);
                    ga += lor(la, t, b);
                }
            } else if constexpr (kLor) {
                gh = lor(lh, t, b);
                ga = lor(la, t, b);
            } else {
                gh = density<K>(P, v0h + b);
                ga = density<K>(P, v0a + b);
            }
        };
        // the node tables through the constant address space: their
        // indices are wave-uniform, so the reads are scalar loads
        const MRT_CONST_AS double *tab = (const MRT_CONST_AS double *)P.psi_tab;
        const MRT_CONST_AS double *tc2 = (const MRT_CONST_AS double *)P.psi_cos2;
        double gh, ga;
        node(0.0, gh, ga);
        double sum_h = tab[1] * gh, sum_a = tab[1] * ga, s2h = 0.0, s2a = 0.0;
        if constexpr (C2) {
            s2h = tc2[0] * gh;
            s2a = tc2[0] * ga;
        }
        for (int j = 1; j <= P.psi_nodes; ++j) {
            const double t = tab[2 * j], wj = tab[2 * j + 1];
            node(t, gh, ga);
            sum_h = fma(wj, gh, sum_h);
            sum_a = fma(wj, ga, sum_a);
            if constexpr (C2) {
                const double wc = tc2[j];
                s2h = fma(wc, gh, s2h);
                s2a = fma(wc, ga, s2a);
            }
        }
        ih = 2.0 * sum_h;
        ia = 2.0 * sum_a;
        i2h = s2h;
        i2a = s2a;
    }
    template <bool C2>
    static __device__ __forceinline__ void psi_integrals(const TraceParams &P, double alpha,
                                                         double beta, double &ih, double &ia,
                                                         double &i2h, double &i2a) {
        switch (P.mdf) {
        case MRT_MOSAIC_GAUSSIAN_VMF:
            psi_pair<MRT_MOSAIC_GAUSSIAN_VMF, C2>(P, alpha, beta, ih, ia, i2h, i2a);
            break;
        case MRT_MOSAIC_LORENTZIAN:
            psi_pair<MRT_MOSAIC_LORENTZIAN, C2>(P, alpha, beta, ih, ia, i2h, i2a);
            break;
        case MRT_MOSAIC_PSEUDO_VOIGT:
            psi_pair<MRT_MOSAIC_PSEUDO_VOIGT, C2>(P, alpha, beta, ih, ia, i2h, i2a);
            break;
        case MRT_MOSAIC_WRAPPED_LORENTZIAN:
            psi_pair<MRT_MOSAIC_WRAPPED_LORENTZIAN, C2>(P, alpha, beta, ih, ia, i2h, i2a);
            break;
        case MRT_MOSAIC_GAUSSIAN:
            psi_pair<MRT_MOSAIC_GAUSSIAN, C2>(P, alpha, beta, ih, ia, i2h, i2a);
            break;
        default:
            psi_pair<MRT_MOSAIC_SPHERICAL_WRAPPED_LORENTZIAN, C2>(P, alpha, beta, ih, ia, i2h, i2a);
            break;
        }
    }
    // The polarisation's direction about k in the frame of planes of normal
    // N at glancing angle alpha: (c, s) = (p.u, p.(k x u)) normalised, u =
    // (N + sin(alpha) k) / cos(alpha) the unit component of N normal to k (so
    // only p's component normal to k counts, as in the paper's angle phi);
    // the crystallite at azimuth psi has G = 1 - sin^2(2 b) (c cos(psi) +
    // s sin(psi))^2.
    static __device__ __forceinline__ void pol_frame(const V3<double> &p, const V3<double> &N,
                                                     const V3<double> &k, double sa, double ca,
                                                     double &c, double &s) {
        const V3<double> u{(N.x + sa * k.x) / ca, (N.y + sa * k.y) / ca, (N.z + sa * k.z) / ca};
        c = dot(p, u);
        s = dot(p, cross(k, u));
        const double r2 = c * c + s * s;
        if (r2 > 0.0) {
            const double inv = 1.0 / ::sqrt(r2);
            c *= inv;
            s *= inv;
        }
    }

    // ---- one event: free path, then exit, absorption or a pending
    // reflection.  Returns the end status, or -1 (`pend` set when the event
    // is a reflection off the planes of normal Ns at glancing angle alpha_s).
    static __device__ __forceinline__ int event(const TraceParams &P, RayT &ry, bool &pend,
                                                V3<double> &Ns, double &alpha_s, int &pset) {
        if (ry.nev == P.max_events) return MRT_TRUNCATED;
        const dm::Words w = dm::philox(P.key0, P.key1, ry.nev, (uint32_t)ry.id,
                                       (uint32_t)(ry.id >> 32), 1u);
        ++ry.nev;
        const int exit_status = ry.nrefl ? MRT_EXIT_REFLECTED : MRT_EXIT_TRANSMITTED;
        const double dist = B::exit_distance(P, ry.p, ry.k);
        const V3<double> N = B::normal_at(P, ry.p);
        double sn = -dot(ry.k, N);
        sn = sn > 1.0 ? 1.0 : (sn < -1.0 ? -1.0 : sn);
        const double alpha = ::asin(sn);
        if constexpr (PLANES) return event_planes(P, ry, pend, Ns, alpha_s, pset, w, exit_status,
                                                  dist, N, sn, alpha);
        double sig_h = 0.0, sig_a = 0.0;
        if (ry.sa < 1.0 && (int)ry.nrefl < P.max_refl) {
            const double beta = ::asin(ry.sa) + P.shift;
            double ih, ia, i2h, i2a;
            bool polar = false;
            if constexpr (POL) polar = P.user_p != nullptr;
            if (polar) {
                // Eq. SimpleReflXsectionPol; cos(2 phi') is the same seen
                // from the H and anti-H planes
                psi_integrals<true>(P, alpha, beta, ih, ia, i2h, i2a);
                double c = 0.0, s = 0.0;
                const double ca = ::sqrt(fma(-sn, sn, 1.0));
                if constexpr (POL) {
                    if (ca > 0.0) pol_frame(ry.pol, N, ry.k, sn, ca, c, s);
                }
                double s2, c2;
                sincos_(2.0 * beta, &s2, &c2);
                const double S = s2 * s2, cos2 = c * c - s * s;
                ih = (1.0 - S / 2.0) * ih - S * cos2 * i2h;
                ia = (1.0 - S / 2.0) * ia - S * cos2 * i2a;
            } else {
                psi_integrals<false>(P, alpha, beta, ih, ia, i2h, i2a);
            }
            const double qc = P.q * cos_(beta);
            sig_h = qc * ih;
            sig_a = qc * ia;
        }
        const double mu = P.mu0 + sig_h + sig_a;
        const double l = -dm::log_u01(w.w0) / mu;
        if (l >= dist) {
            ry.p = axpy(ry.p, dist, ry.k);
            return exit_status;
        }
        ry.p = axpy(ry.p, l, ry.k);
        if (dm::u01_f64(w.w1) <= P.mu0 / mu) return MRT_ABSORBED;
        // H planes (normal N) or anti-H planes (normal -N), by their share
        const bool anti = !(dm::u01_f64(w.w2) * (sig_h + sig_a) < sig_h);
        Ns = anti ? V3<double>{-N.x, -N.y, -N.z} : N;
        alpha_s = anti ? -alpha : alpha;
        pend = true;
        return -1;
    }

    // One event with plane sets: the H and anti-H terms of every set j (its
    // Bragg angle, shift, and curve of strength a_j and width scale s_j, so
    // q_j = a_j s_j q), the anti-H terms times hbar; the reflecting set and
    // side drawn by u2 against the running sum in the order H_0, anti-H_0,
    // H_1, ... (at most four sets; the loops unroll over them).
    static __device__ __forceinline__ double sigma_pair(const TraceParams &P, const RayT &ry,
                                                        const V3<double> &N, double sn,
                                                        double alpha, double beta, double &ia) {
        double ih, i2h, i2a;
        bool polar = false;
        if constexpr (POL) polar = P.user_p != nullptr;
        if (polar) {
            psi_integrals<true>(P, alpha, beta, ih, ia, i2h, i2a);
            double c = 0.0, s = 0.0;
            const double ca = ::sqrt(fma(-sn, sn, 1.0));
            if constexpr (POL) {
                if (ca > 0.0) pol_frame(ry.pol, N, ry.k, sn, ca, c, s);
            }
            double s2, c2;
            sincos_(2.0 * beta, &s2, &c2);
            const double S = s2 * s2, cos2 = c * c - s * s;
            ih = (1.0 - S / 2.0) * ih - S * cos2 * i2h;
            ia = (1.0 - S / 2.0) * ia - S * cos2 * i2a;
        } else {
            psi_integrals<false>(P, alpha, beta, ih, ia, i2h, i2a);
        }
        return ih;
    }
    static __device__ __forceinline__ int event_planes(const TraceParams &P, RayT &ry, bool &pend,
                                                       V3<double> &Ns, double &alpha_s, int &pset,
                                                       const dm::Words &w, int exit_status,
                                                       double dist, const V3<double> &N, double sn,
                                                       double alpha) {
        double sh[kSets], sa[kSets], sum = 0.0;
#pragma unroll
        for (int j = 0; j < kSets; ++j) {
            sh[j] = 0.0;
            sa[j] = 0.0;
            if (j < P.n_planes) {
                const double sj = j ? kHC / (P.plane_2d[j] * ry.E) : ry.sa;
                if (sj < 1.0 && (int)ry.nrefl < P.max_refl) {
                    double shift, scale;
                    set_curve(P, ry, j, shift, scale);
                    const double beta = ::asin(sj) + shift;
                    double ia;
                    const double ih = sigma_pair(P, ry, N, sn, alpha, beta, ia);
                    const double qc = P.q * (P.plane_a[j] * scale) * cos_(beta);
                    sh[j] = qc * ih;
                    sa[j] = P.hbar * qc * ia;
                }
                sum += sh[j];
                sum += sa[j];
            }
        }
        const double mu = P.mu0 + sum;
        const double l = -dm::log_u01(w.w0) / mu;
        if (l >= dist) {
            ry.p = axpy(ry.p, dist, ry.k);
            return exit_status;
        }
        ry.p = axpy(ry.p, l, ry.k);
        if (dm::u01_f64(w.w1) <= P.mu0 / mu) return MRT_ABSORBED;
        const double target = dm::u01_f64(w.w2) * sum;
        double acc = 0.0;
        int js = P.n_planes - 1;
        bool anti = true, chosen = false;
#pragma unroll
        for (int j = 0; j < kSets; ++j) {
            if (j < P.n_planes && !chosen) {
                acc += sh[j];
                if (target < acc) {
                    js = j;
                    anti = false;
                    chosen = true;
                } else {
                    acc += sa[j];
                    if (target < acc) {
                        js = j;
                        anti = true;
                        chosen = true;
                    }
                }
            }
        }
        Ns = anti ? V3<double>{-N.x, -N.y, -N.z} : N;
        alpha_s = anti ? -alpha : alpha;
        pset = js;
        pend = true;
        return -1;
    }
    static constexpr int kSets = 4;
    // Set j's curve shift and width scale; an energy-dependent curve
    // (sec. 2.2.1) gives the main set Delta_M(E) and s(E).
    static __device__ __forceinline__ void set_curve(const TraceParams &P, const RayT &ry, int j,
                                                     double &shift, double &scale) {
        if (j == 0 && P.dep_n > 0) {
            shift = B::interp(P.dep, P.dep + P.dep_n, P.dep_n, ry.E);
            scale = B::interp(P.dep, P.dep + 2 * P.dep_n, P.dep_n, ry.E);
        } else {
            shift = P.plane_shift[j];
            scale = P.plane_scale[j];
        }
    }

    // ---- the sampler's target: the integrand of Eq. ReflXsection --------
    // f(psi, Delta) = r(Delta - Delta_M) cos(b) W(v), b = alpha_B + Delta,
    // v = 2 sin^2((alpha - b)/2) + 2 cos(alpha) cos(b) sin^2(psi/2).  The
    // sampler keeps the factors of the current point: a psi move changes
    // only sin(psi/2), a Delta move only r, cos(b) and sin((alpha - b)/2), so
    // each factor is evaluated once per move, as the full formula would.
    // With polarisation the target is the integrand of Eq. ReflXsectionPol:
    // f G, G = 1 - sin^2(2 b) (c cos(psi) + s sin(psi))^2 (pol_frame); the
    // point then also keeps sin^2(2 b) and cos(psi/2).
    struct Point {
        double r, cb, sab, sp;   // r(Delta - Delta_M), cos(b), sin((alpha - b)/2), sin(psi/2)
        double s2b, cp;          // polarised: sin^2(2 b), cos(psi/2)
    };
    static __device__ __forceinline__ double value(const TraceParams &P, const Point &x,
                                                   double ca, bool polar, double pc, double ps) {
        if (!(x.r > 0.0)) return 0.0;
        const double v = 2.0 * x.sab * x.sab + 2.0 * ca * x.cb * x.sp * x.sp;
        const double f = x.r * x.cb * density_any(P, v);
        if (!polar) return f;
        // cos(psi) = 1 - 2 sin^2(psi/2), sin(psi) = 2 sin(psi/2) cos(psi/2)
        const double proj = pc * (1.0 - 2.0 * x.sp * x.sp) + ps * (2.0 * x.sp * x.cp);
        return f * (1.0 - x.s2b * proj * proj);
    }
    // (sa, ca: sin and cos of alpha.)  Without polarisation cos(b) comes
    // from the same sin/cos as sin((alpha - b) / 2): with d = (alpha - b) / 2,
    // cos(b) = cos(alpha) (1 - 2 sin^2 d) + sin(alpha) 2 sin(d) cos(d).  The
    // two terms cancel only as b nears 90 deg, where the relative error grows
    // as 1 / cos(b) (a few ulps at cos(b) = 0.05).
    static __device__ __forceinline__ void at_delta(const TraceParams &P, const double *lut,
                                                    double alpha, double sa, double ca, double ab,
                                                    double delta, double shift, double scale,
                                                    bool polar, Point &x) {
        const double b = ab + delta;
        // a further plane set reads the curve at (Delta - its shift) / its scale
        x.r = B::irc_ratio(P, lut, scale == 1.0 ? delta - shift : (delta - shift) / scale);
        if (polar) {
            double sb;
            sincos_(b, &sb, &x.cb);
            const double s2 = 2.0 * sb * x.cb;
            x.s2b = s2 * s2;
            x.sab = sin_((alpha - b) / 2.0);
        } else {
            double sd, cd;
            sincos_((alpha - b) / 2.0, &sd, &cd);
            x.sab = sd;
            x.cb = fma(ca, fma(-2.0 * sd, sd, 1.0), 2.0 * sa * sd * cd);
        }
    }

    // ---- Metropolis-within-Gibbs draw and the reflection -----------------
    // From (0, Delta_M): burn_in sweeps of a psi move and (unless the IRC is
    // disabled, which holds Delta at Delta_M) a Delta move,
    // symmetric uniform random walks, a move taken when u f(current) <
    // f(proposed) or from a point of zero density, Delta outside
    // [-alpha_B, pi/2 - alpha_B] rejected, psi wrapped on [-pi, pi).  Sweep s
    // of event e draws the Philox words of counter (s, ray, 2^31 + e).  Then
    // N is rotated by alpha - (alpha_B + Delta) about N x k and by psi about
    // k, and k is reflected (sec. 2.2.4).
    static __device__ __forceinline__ void reflect(const TraceParams &P, const double *lut, RayT &ry,
                                                   V3<double> Ns, double alpha, int pset) {
        // the reflecting set: its Bragg angle, shift and width scale
        double ab, shift = P.shift, scale = 1.0;
        if constexpr (PLANES) {
            ab = ::asin(pset ? kHC / (P.plane_2d[pset] * ry.E) : ry.sa);
            set_curve(P, ry, pset, shift, scale);
        } else {
            ab = ::asin(ry.sa);
        }
        const double w_delta = PLANES ? P.w_delta * scale : P.w_delta;
        const double lo = -ab, hi = kPiHalf - ab;
        double psi = 0.0, delta = shift;
        delta = delta < lo ? lo : (delta > hi ? hi : delta);
        double cbm = cos_(ab + shift);
        cbm = cbm > 0.05 ? cbm : 0.05;
        const double w_psi = P.fwhm / cbm;
        double sa, ca;
        sincos_(alpha, &sa, &ca);
        const uint32_t event = ry.nev - 1u;
        bool polar = false;
        double pc = 0.0, ps = 0.0;
        if constexpr (POL) {
            polar = P.user_p != nullptr;
            if (polar && ca > 0.0) pol_frame(ry.pol, Ns, ry.k, sa, ca, pc, ps);
        }
        Point x;
        at_delta(P, lut, alpha, sa, ca, ab, delta, shift, scale, polar, x);
        x.sp = 0.0;   // sin(0 / 2)
        x.cp = 1.0;
        double f = value(P, x, ca, polar, pc, ps);
        for (int s = 0; s < P.burn_in; ++s) {
            const dm::Words w = dm::philox(P.key0, P.key1, (uint32_t)s, (uint32_t)ry.id,
                                           (uint32_t)(ry.id >> 32), 0x80000000u | event);
            double pn = psi + w_psi * (2.0 * dm::u01_f64(w.w0) - 1.0);
            pn = pn >= kPi ? pn - 2.0 * kPi : (pn < -kPi ? pn + 2.0 * kPi : pn);
            Point y = x;
            if (polar) sincos_(pn / 2.0, &y.sp, &y.cp);
            else y.sp = sin_(pn / 2.0);
            double fn = value(P, y, ca, polar, pc, ps);
            if (dm::u01_f64(w.w1) * f < fn || f == 0.0) {
                psi = pn;
                x = y;
                f = fn;
            }
            const double dn = delta + w_delta * (2.0 * dm::u01_f64(w.w2) - 1.0);
            if (!P.irc_off && dn >= lo && dn <= hi) {   // the IRC disabled: Delta stays
                y = x;
                at_delta(P, lut, alpha, sa, ca, ab, dn, shift, scale, polar, y);
                fn = value(P, y, ca, polar, pc, ps);
                if (dm::u01_f64(w.w3) * f < fn || f == 0.0) {
                    delta = dn;
                    x = y;
                    f = fn;
                }
            }
        }
        // crystallite normal
        const double th = alpha - (ab + delta);
        const V3<double> k = ry.k;
        V3<double> n0 = Ns;
        if (ca > 0.0) {
            double st, ct;
            sincos_(th, &st, &ct);
            n0 = V3<double>{ct * Ns.x + st * (k.x + sa * Ns.x) / ca, ct * Ns.y + st * (k.y + sa * Ns.y) / ca,
                            ct * Ns.z + st * (k.z + sa * Ns.z) / ca};
        }
        const V3<double> kx = cross(k, n0);
        double sp, cp;
        sincos_(psi, &sp, &cp);
        const double kn0 = dot(k, n0);
        const V3<double> n{cp * n0.x + sp * kx.x + (1.0 - cp) * kn0 * k.x,
                           cp * n0.y + sp * kx.y + (1.0 - cp) * kn0 * k.y,
                           cp * n0.z + sp * kx.z + (1.0 - cp) * kn0 * k.z};
        const double two_kn = 2.0 * dot(k, n);
        const V3<double> ks{k.x - two_kn * n.x, k.y - two_kn * n.y, k.z - two_kn * n.z};
        const double nr = ::sqrt(dot(ks, ks));
        ry.k = V3<double>{ks.x / nr, ks.y / nr, ks.z / nr};
        if constexpr (POL) {
            if (polar) {
                // the polarisation after the reflection (sec. 2.2.4)
                const double pks = dot(ry.pol, ry.k), g = ::sqrt(1.0 - pks * pks);
                ry.pol = V3<double>{(ry.pol.x - pks * ry.k.x) / g, (ry.pol.y - pks * ry.k.y) / g,
                                    (ry.pol.z - pks * ry.k.z) / g};
            }
        }
        ++ry.nrefl;
    }

    static constexpr double kPi = 3.14159265358979323846;
    static constexpr double kInv2Pi = 0.15915494309189533577;
    static constexpr double kPiHalf = 1.57079632679489661923;
};

// ---------------------------------------------------------------------------
// The persistent loop of one wave for the paper's model.  Ray starts, the
// queue refill and the detector work are those of trace_loop (same queue,
// same claims, same counters); the event step differs, and lanes whose event
// is a reflection park until the wave runs the sampler for all of them.
// ---------------------------------------------------------------------------
template <class T, class Claim, class Q>
__device__ __forceinline__ void mwg_loop(const TraceParams &P, const double *lut, const double *cdf,
                                         Claim &claim, Q &q) {
    typename T::RayT ry;
    bool active = false;
    bool pend = false;            // the lane waits for the sampler
    V3<double> Ns{0.0, 0.0, 0.0};
    double alpha_s = 0.0;
    int pset = 0;                 // the reflecting plane set (PLANES)
    WaveCounts cnt{};
    uint64_t next = 0, end = 0;
    bool more = true;
    uint32_t head = 0, queued = 0;
    const uint32_t refill_at = P.refill_idle < 1u ? 1u : (P.refill_idle > 64u ? 64u : P.refill_idle);
    const uint32_t batch = P.mwg_batch < 1 ? 1u : (P.mwg_batch > 64 ? 64u : (uint32_t)P.mwg_batch);
    const uint32_t lane = __lane_id();

    for (;;) {
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
        }
        const uint64_t act0 = ballot(active);
        if (act0 == 0) {
            if (!more && queued == 0) break;
            continue;
        }

        const uint32_t keep = more || queued ? 65u - refill_at : 1u;
        for (;;) {
            int status = -1;
            const bool stepping = active && !pend;
            if (stepping) status = T::event(P, ry, pend, Ns, alpha_s, pset);
            const bool ended = status >= 0;
            bool det = false;
            if (ended) {
                det = T::finish(P, ry, status);
                active = false;
            }
            cnt.events += popc(ballot(stepping && status != MRT_TRUNCATED));
            const uint64_t endm = ballot(ended);
            if (endm) {
                cnt.absorbed += popc(ballot(ended && status == MRT_ABSORBED));
                cnt.exit_refl += popc(ballot(ended && status == MRT_EXIT_REFLECTED));
                cnt.exit_trans += popc(ballot(ended && status == MRT_EXIT_TRANSMITTED));
                cnt.truncated += popc(ballot(ended && status == MRT_TRUNCATED));
                cnt.detected += popc(ballot(det));
            }
            // The parked lanes run the sampler together once `batch` of them
            // wait.  While rays can still be taken in, at most `keep` wait
            // (then no lane steps and the wave would not break to refill);
            // while draining, they also run when no lane can step.
            const uint32_t npend = popc(ballot(pend));
            const bool refilling = more || queued;
            const uint32_t due = refilling && keep < batch ? keep : batch;
            if (npend && (npend >= due || (!refilling && popc(ballot(active && !pend)) == 0))) {
                if (pend) {
                    T::reflect(P, lut, ry, Ns, alpha_s, pset);
                    pend = false;
                }
                cnt.reflections += npend;
            }
            if (popc(ballot(active)) < keep) break;
        }
    }
    flush(P, cnt);
}

// At least 4 waves per SIMD for the instances without polarisation or plane
// sets: held to 128 VGPRs they spill about 27 to scratch outside the
// quadrature and sampler loops, and the extra wave per SIMD hides more of
// the loops' latency (von Hamos 2%, flat 5% faster).  The others keep the
// compiler's choice (they need 160-210 VGPRs).
template <bool POL, bool PLANES>
constexpr int kMwgMinWaves = POL || PLANES ? 1 : 4;
template <int GEOM, bool REC, bool POL, bool PLANES = false>
__global__ void __launch_bounds__(256, (kMwgMinWaves<POL, PLANES>)) mwg_kernel(const TraceParams P) {
    using T = MwgTracer<GEOM, REC, POL, PLANES>;
    const TraceParams &Q = *(const TraceParams *)__builtin_amdgcn_kernarg_segment_ptr();
    RangeClaim claim{Q.chunk_counter, Q.first, Q.n, Q.chunk};
    __shared__ typename T::Queue queues[4];   // one per wave
    typename T::Queue &q = queues[uniform(threadIdx.x >> 6)];
    mwg_loop<T>(Q, Q.lut, Q.bin_cdf, claim, q);
}

template <int GEOM, bool POL, bool PLANES> const void *mwg_kernel_of(bool records) {
    return records ? (const void *)mwg_kernel<GEOM, true, POL, PLANES>
                   : (const void *)mwg_kernel<GEOM, false, POL, PLANES>;
}
template <int GEOM> const void *mwg_kernel_geom(bool records, bool polarised, bool planes) {
    if (planes)
        return polarised ? mwg_kernel_of<GEOM, true, true>(records) : mwg_kernel_of<GEOM, false, true>(records);
    return polarised ? mwg_kernel_of<GEOM, true, false>(records) : mwg_kernel_of<GEOM, false, false>(records);
}

}  // namespace tk

const void *mwg_kernel_ptr(int geometry, bool records, bool polarised, bool planes) {
    if (geometry == MRT_GEOMETRY_FLAT)
        return tk::mwg_kernel_geom<MRT_GEOMETRY_FLAT>(records, polarised, planes);
    if (geometry == MRT_GEOMETRY_CYLINDER)
        return tk::mwg_kernel_geom<MRT_GEOMETRY_CYLINDER>(records, polarised, planes);
    return nullptr;
}

}  // namespace mrt
