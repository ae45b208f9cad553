/*
 * Oracle for the per-ray mosaic-crystal transport of HEART (arXiv 2503.16955).
 *
 * TEST INFRASTRUCTURE.  Plain scalar FP64 C with glibc libm and pthreads.
 * Loaded only by the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark.  It shares nothing with the GPU library but the written
 * model it follows; each function names the part of the paper it restates.
 *
 * Two event models.  The paper's own (sec. 2.2.3, 2.2.4; mwg_events): a free
 * path from exp(-(mu0 + gamma0 sigma) l) (Eq. AnyEvent) with gamma0 sigma from
 * Eq. SimpleReflXsection, absorption with probability mu0 / mu_eff, and
 * otherwise a reflecting crystallite sampled from the integrand of Eq.
 * ReflXsection by Metropolis-within-Gibbs.  The default realises the same
 * law without the approximation of Eq. SimpleReflXsection and without a
 * Markov chain, by null-collision (Woodcock) stepping: candidate
 * crystallite encounters arrive at a majorant rate lambda_c = R_max / h, each
 * draws a crystallite normal from the mosaic distribution on the unit sphere
 * (sec. 2.2.2) and reflects with probability r(Delta - Delta_M) / R_max,
 * where r is the intrinsic rocking curve (sec. 2.2.1).  Because the accepted
 * normals are distributed exactly as R(Delta) cos(alpha_B + Delta)
 * W(theta(psi)) d Delta d psi, this samples psi rather than theta, which is
 * the correct ("method II") orientation law of appendix A.
 *
 * Parity unpinned: the absolute reflectivity scale (only R_max / h is
 * identifiable), which is an input of the workloads, not of this code.
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORC_HC 12.398419843320026   /* h c in keV Angstrom (SI 2019 exact) */
#define ORC_TWO_PI 6.283185307179586476925286766559
#define ORC_PI 3.1415926535897932384626433832795

/* ------------------------------------------------------------------------ */
/* Philox4xW-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11). */
/* One round: two wide multiplies of words 0 and 2, their high halves xored  */
/* with the other two words and the round key, words permuted; the key is   */
/* bumped by the Weyl constants between rounds.                              */
/* ------------------------------------------------------------------------ */
static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

#define PHILOX_10(T, MULHILO, M0, M1, W0, W1, ctr, key, out)                 \
    do {                                                                      \
        T c_[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};                           \
        T k_[2] = {key[0], key[1]};                                           \
        for (int r_ = 0; r_ < 10; ++r_) {                                     \
            T hi0_, lo0_, hi1_, lo1_;                                         \
            MULHILO((T)(M0), c_[0], &hi0_, &lo0_);                            \
            MULHILO((T)(M1), c_[2], &hi1_, &lo1_);                            \
            T n0_ = hi1_ ^ c_[1] ^ k_[0];                                     \
            T n2_ = hi0_ ^ c_[3] ^ k_[1];                                     \
            c_[0] = n0_; c_[1] = lo1_; c_[2] = n2_; c_[3] = lo0_;             \
            k_[0] = (T)(k_[0] + (T)(W0));                                     \
            k_[1] = (T)(k_[1] + (T)(W1));                                     \
        }                                                                     \
        out[0] = c_[0]; out[1] = c_[1]; out[2] = c_[2]; out[3] = c_[3];       \
    } while (0)

void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    PHILOX_10(uint32_t, mulhilo32, 0xD2511F53u, 0xCD9E8D57u,
              0x9E3779B9u, 0xBB67AE85u, ctr, key, out);
}

void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    PHILOX_10(uint64_t, mulhilo64, 0xD2E7470EE14C6C93ull, 0xCA5A826395121157ull,
              0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull, ctr, key, out);
}

/* Random words of one ray: counter (index, ray_lo, ray_hi, domain), key =
   the 64-bit seed split into two halves.  Domain 0 feeds the source, domain
   1 the depth events (index = 0-based event number). */
static void ray_words(uint64_t seed, uint64_t ray, uint32_t domain, uint32_t index,
                      double u[4]) {
    uint32_t ctr[4] = {index, (uint32_t)ray, (uint32_t)(ray >> 32), domain};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32(ctr, key, w);
    for (int i = 0; i < 4; ++i) u[i] = ((double)w[i] + 0.5) * 0x1p-32; /* open (0,1) */
}

/* ------------------------------------------------------------------------ */
/* Small vector helpers.                                                     */
/* ------------------------------------------------------------------------ */
static double dot(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross(const double a[3], const double b[3], double r[3]) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static void sub(const double a[3], const double b[3], double r[3]) {
    r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static void axpy(const double p[3], double t, const double k[3], double r[3]) {
    r[0] = p[0] + t * k[0]; r[1] = p[1] + t * k[1]; r[2] = p[2] + t * k[2];
}
static void note(double *m, double v) {
    v = fabs(v);
    if (v < *m) *m = v;
}

/* ------------------------------------------------------------------------ */
/* Bragg's law (Eq. BraggLaw): hc / E = 2 d sin(alpha_B).                    */
/* ------------------------------------------------------------------------ */
double orc_bragg_angle(double energy_kev, double two_d) {
    double s = ORC_HC / (two_d * energy_kev);
    if (!(s < 1.0)) return -1.0;
    return asin(s);
}

/* Linear interpolation of a table of the photon energy (nodes x strictly
   increasing), the end values held outside it. */
static double interp_clamped(const double *x, const double *y, int n, double E) {
    if (n == 1 || !(E > x[0])) return y[0];
    if (!(E < x[n - 1])) return y[n - 1];
    int j = 0;   /* the last node at or below E */
    while (x[j + 1] <= E) ++j;
    double slope = (y[j + 1] - y[j]) / (x[j + 1] - x[j]);
    return y[j] + slope * (E - x[j]);
}

/* ------------------------------------------------------------------------ */
/* Intrinsic rocking curve (sec. 2.2.1).                                     */
/* ------------------------------------------------------------------------ */
void orc_pvoigt_params(double g, double l, double *fwhm, double *eta) {
    /* total width: fifth root of the weighted quintic in (Lambda_G, Lambda_L) */
    double f5 = pow(g, 5) + 2.69269 * pow(g, 4) * l + 2.42843 * pow(g, 3) * l * l
              + 4.47163 * g * g * pow(l, 3) + 0.07842 * g * pow(l, 4) + pow(l, 5);
    double f = pow(f5, 0.2);
    double q = l / f;
    *fwhm = f;
    *eta = 1.36603 * q - 0.47719 * q * q + 0.11116 * q * q * q;
}

static double gauss_unit(double x, double w) {   /* Eq. Gaussian, unit area */
    return sqrt(4.0 * log(2.0) / (ORC_PI * w * w)) * exp(-4.0 * log(2.0) * x * x / (w * w));
}
static double lorentz_unit(double x, double w) { /* Eq. Lorentz, unit area */
    return (w / (2.0 * ORC_PI)) / ((w / 2.0) * (w / 2.0) + x * x);
}

double orc_irc_value(const orc_irc *irc, double x) {
    switch (irc->kind) {
    case ORC_IRC_GAUSS:
        return irc->peak * exp(-4.0 * log(2.0) * x * x / (irc->fwhm * irc->fwhm));
    case ORC_IRC_PVOIGT: {
        double w, eta;
        orc_pvoigt_params(irc->fwhm_g, irc->fwhm_l, &w, &eta);
        double rx = eta * lorentz_unit(x, w) + (1.0 - eta) * gauss_unit(x, w);
        double r0 = eta * lorentz_unit(0.0, w) + (1.0 - eta) * gauss_unit(0.0, w);
        return irc->peak * rx / r0;
    }
    case ORC_IRC_TABLE: {
        int n = irc->n_table;
        if (x < irc->x_min || x > irc->x_max) return 0.0;
        if (x == irc->x_max) return irc->table[n - 1];
        double f = (x - irc->x_min) / (irc->x_max - irc->x_min) * (double)(n - 1);
        int j = (int)floor(f);
        if (j >= n - 1) return irc->table[n - 1];
        double t = f - (double)j;
        return (1.0 - t) * irc->table[j] + t * irc->table[j + 1];
    }
    case ORC_IRC_LORENTZ: {
        double h = irc->fwhm / 2.0;
        return irc->peak * h * h / (h * h + x * x);
    }
    case ORC_IRC_BOX:
        return fabs(x) <= irc->fwhm / 2.0 ? irc->peak : 0.0;
    }
    return 0.0;
}

static double irc_max(const orc_irc *irc) {
    if (irc->kind == ORC_IRC_TABLE) {
        double m = 0.0;
        for (int i = 0; i < irc->n_table; ++i)
            if (irc->table[i] > m) m = irc->table[i];
        return m;
    }
    return irc->peak;
}

/* ------------------------------------------------------------------------ */
/* Mosaic distribution on the unit sphere (sec. 2.2.2).  Each sampler maps  */
/* one uniform to v = 1 - cos(theta) by the inverse of the radial CDF; the  */
/* azimuth xi about N is uniform (the MDF is isotropic about N).             */
/* ------------------------------------------------------------------------ */
static double vmf_v(double gamma, double u) {
    /* Eq. MF: density in cos(theta) proportional to exp((cos theta - 1)/s^2),
       with Gamma = 2 s sqrt(2 ln 2). */
    double s = gamma / (2.0 * sqrt(2.0 * log(2.0)));
    double s2 = s * s;
    double floor_ = exp(-2.0 / s2);
    double v = -s2 * log(u + (1.0 - u) * floor_);
    return v < 2.0 ? v : 2.0;
}

static void lorentz_tilt(double gamma, double q, double *ct, double *st) {
    /* Isotropic tilt whose every one-dimensional marginal is the Lorentzian
       of Eq. Lorentz with FWHM Gamma: bivariate Cauchy in the tangent plane,
       radial CDF F(T) = 1 - g / sqrt(g^2 + T^2), g = Gamma / 2, mapped to
       the sphere by tan(theta) = T.  q = 1 - F. */
    double g = gamma / 2.0;
    double T = g * sqrt(1.0 - q * q) / q;
    double c = 1.0 / sqrt(1.0 + T * T);
    *ct = c;
    *st = T * c;
}

static void gauss_tilt(double gamma, double u, double *ct, double *st) {
    /* The regular Gaussian of Eq. Gaussian (Delta -> theta, Lambda ->
       Gamma) as an isotropic tilt: a bivariate normal in the tangent plane
       with standard deviation s = Gamma / (2 sqrt(2 ln 2)) on each axis, so
       that every one-dimensional marginal is Eq. Gaussian; its radius
       T = s sqrt(-2 ln u) (Rayleigh), mapped to the sphere by tan(theta) = T. */
    double s = gamma / (2.0 * sqrt(2.0 * log(2.0)));
    double T = s * sqrt(-2.0 * log(u));
    double c = 1.0 / sqrt(1.0 + T * T);
    *ct = c;
    *st = T * c;
}

void orc_mdf_sample(const orc_mosaic *m, double u2, double u3,
                    const double N[3], const double e1[3], const double e2[3],
                    double n_out[3]) {
    double ct = 1.0, st = 0.0;
    double gamma = m->fwhm;
    if (gamma > 0.0) {
        double v = -1.0;
        switch (m->kind) {
        case ORC_MDF_VMF:
            v = vmf_v(gamma, u2);
            break;
        case ORC_MDF_LORENTZ:
            lorentz_tilt(gamma, 1.0 - u2, &ct, &st);
            break;
        case ORC_MDF_PVOIGT:
            /* mixture: Lorentzian with probability eta, else von Mises-Fisher,
               both at the same FWHM */
            if (u2 < m->eta)
                lorentz_tilt(gamma, (m->eta - u2) / m->eta, &ct, &st);
            else
                v = vmf_v(gamma, (u2 - m->eta) / (1.0 - m->eta));
            break;
        case ORC_MDF_WRAPPED_LORENTZ: {
            /* Eq. WL: density in v proportional to 1 / (g^2 + 2 v) */
            double g = gamma / 2.0;
            double Z = log((g * g + 4.0) / (g * g));
            v = g * g * expm1(u2 * Z) / 2.0;
            if (v > 2.0) v = 2.0;
            break;
        }
        case ORC_MDF_SPHERICAL_WRAPPED_LORENTZ: {
            /* Eq. SWL: density in v proportional to 1 / (cosh(Gamma/2) - 1 + v)^2 */
            double a = gamma / 2.0;
            double sh = sinh(a / 2.0);
            v = 2.0 * sh * sh * 2.0 * u2 / (cosh(a) + 1.0 - 2.0 * u2);
            if (v > 2.0) v = 2.0;
            break;
        }
        case ORC_MDF_GAUSSIAN:
            gauss_tilt(gamma, u2, &ct, &st);
            break;
        }
        if (v >= 0.0) {
            ct = 1.0 - v;
            st = sqrt(v * (2.0 - v));
        }
    }
    double xi = ORC_TWO_PI * u3;
    double cx = cos(xi), sx = sin(xi);
    for (int i = 0; i < 3; ++i)
        n_out[i] = ct * N[i] + st * (cx * e1[i] + sx * e2[i]);
}

/* ------------------------------------------------------------------------ */
/* Photon source (sec. 2.1): origins at the source point or spread over    */
/* the source spot (sec. 4.2), directions uniform in solid angle inside a   */
/* cone, energies drawn from the spectrum used as a PDF; any of the three   */
/* may instead come from the user's arrays.                                  */
/* ------------------------------------------------------------------------ */
static void sample_point_source(const orc_source *s, const double *w, double o[3], double k[3],
                                double *energy);

void orc_source_sample(const orc_source *s, uint64_t seed, uint64_t ray_id,
                       double o[3], double k[3], double *energy) {
    double w[8];
    ray_words(seed, ray_id, 0, 0, w);
    ray_words(seed, ray_id, 0, 1, w + 4);
    uint64_t row = ray_id - s->user_first;
    sample_point_source(s, w, o, k, energy);

    /* spot: an offset (x, y) in the plane of spot_u, spot_v from the two
       uniforms w[5], w[6] -- a 2-D normal by the Box-Muller transform, or a
       point uniform over the disk (radius R sqrt(u) for a uniform area) */
    if (s->spot_kind != ORC_SPOT_POINT) {
        double phi = ORC_TWO_PI * w[6];
        double x, y;
        if (s->spot_kind == ORC_SPOT_GAUSSIAN) {
            double r = sqrt(-2.0 * log(w[5]));
            x = s->spot_sigma[0] * r * cos(phi);
            y = s->spot_sigma[1] * r * sin(phi);
        } else {
            double r = s->spot_sigma[0] * sqrt(w[5]);
            x = r * cos(phi);
            y = r * sin(phi);
        }
        for (int i = 0; i < 3; ++i) o[i] += x * s->spot_u[i] + y * s->spot_v[i];
    }
    if (s->user_o)
        for (int i = 0; i < 3; ++i) o[i] = s->user_o[3 * row + i];
    if (s->user_k)
        for (int i = 0; i < 3; ++i) k[i] = s->user_k[3 * row + i];
    if (s->user_e) *energy = s->user_e[row];
}

static void sample_point_source(const orc_source *s, const double *w, double o[3], double k[3],
                                double *energy) {

    /* direction: 1 - cos(theta) uniform on [0, 1 - cos(theta_max)] */
    double sh = sin(s->half_angle / 2.0);
    double v = w[0] * (2.0 * sh * sh);
    double ct = 1.0 - v;
    double st = sqrt(v * (2.0 - v));
    double phi = ORC_TWO_PI * w[1];
    double cp = cos(phi), sp = sin(phi);
    double b2[3];
    cross(s->axis, s->b1, b2);
    for (int i = 0; i < 3; ++i) {
        k[i] = ct * s->axis[i] + st * (cp * s->b1[i] + sp * b2[i]);
        o[i] = s->origin[i];
    }

    double E;
    if (s->spectrum == ORC_SPEC_UNIFORM) {
        E = s->e_min + w[2] * (s->e_max - s->e_min);
    } else if (s->spectrum == ORC_SPEC_LINES) {
        /* pick a component against the cumulative normalised weights: the
           lines in order, then the flat background */
        double total = 0.0;
        for (int j = 0; j < s->n_lines; ++j) total += s->line_w[j];
        total += s->background_w;
        double acc = 0.0;
        int pick = s->n_lines;
        for (int j = 0; j < s->n_lines; ++j) {
            acc += s->line_w[j];
            if (w[2] < acc / total) { pick = j; break; }
        }
        if (pick < s->n_lines)
            E = s->line_e[pick] + s->line_sigma[pick] * sqrt(-2.0 * log(w[3]))
                                  * cos(ORC_TWO_PI * w[4]);
        else
            E = s->e_min + w[3] * (s->e_max - s->e_min);
    } else {
        /* tabulated spectrum: bin b is the largest with C[b] <= u, C the
           normalised prefix sums; uniform inside the bin */
        int n = s->n_bins;
        double total = 0.0;
        for (int b = 0; b < n; ++b) total += s->bin_w[b];
        double acc = 0.0;
        int pick = 0;
        for (int b = 0; b < n; ++b) {
            if (acc / total <= w[2]) pick = b;
            acc += s->bin_w[b];
        }
        E = s->e_min + ((double)pick + w[3]) * (s->e_max - s->e_min) / (double)n;
    }
    *energy = E;
}

/* ------------------------------------------------------------------------ */
/* Crystal geometry (sec. 2.2: FlatCrystal and CylinderCrystal; separate    */
/* entry and inside/exit tests).                                             */
/* ------------------------------------------------------------------------ */
typedef struct cyl_edges {
    double b2[3];
    double o_plus[3], o_minus[3];   /* outward normals of the two azimuth edges */
} cyl_edges;

static void cyl_setup(const orc_crystal *c, cyl_edges *E) {
    cross(c->axis_dir, c->ref_dir, E->b2);
    double half = c->width / (2.0 * c->radius);
    double pp = c->phi_c + half, pm = c->phi_c - half;
    for (int i = 0; i < 3; ++i) {
        E->o_plus[i] = -sin(pp) * c->ref_dir[i] + cos(pp) * E->b2[i];
        E->o_minus[i] = sin(pm) * c->ref_dir[i] - cos(pm) * E->b2[i];
    }
}

/* radial vector from the axis and the axial coordinate of point p */
static void cyl_coords(const orc_crystal *c, const double p[3], double rho[3], double *z) {
    double d[3];
    sub(p, c->axis_pt, d);
    *z = dot(d, c->axis_dir);
    axpy(d, -*z, c->axis_dir, rho);
}

/* Front-face entry; returns 1 and the entry distance on a hit. */
static int crystal_entry(const orc_crystal *c, const cyl_edges *E, const double o[3],
                         const double k[3], double *t_out, double *margin) {
    if (c->geometry == ORC_GEOM_FLAT) {
        double d[3], e2[3], h[3];
        sub(o, c->centre, d);
        double zeta = dot(d, c->normal);
        double kn = dot(k, c->normal);
        if (!(kn < 0.0)) return 0;
        double t = -zeta / kn;
        if (!(t > 0.0)) return 0;
        axpy(o, t, k, h);
        sub(h, c->centre, d);
        cross(c->normal, c->e1, e2);
        double xi = dot(d, c->e1), eta = dot(d, e2);
        note(margin, c->length / 2.0 - fabs(xi));
        note(margin, c->width / 2.0 - fabs(eta));
        if (fabs(xi) <= c->length / 2.0 && fabs(eta) <= c->width / 2.0) {
            *t_out = t;
            return 1;
        }
        return 0;
    }
    /* cylinder: the source sits inside the bore; hit the front radius R */
    double rho[3], z, kp[3], h[3];
    cyl_coords(c, o, rho, &z);
    double ka = dot(k, c->axis_dir);
    axpy(k, -ka, c->axis_dir, kp);
    double a = dot(kp, kp), b = dot(rho, kp);
    double cc = dot(rho, rho) - c->radius * c->radius;
    if (!(cc < 0.0) || !(a > 0.0)) return 0;
    double disc = b * b - a * cc;
    double t = b >= 0.0 ? -cc / (b + sqrt(disc)) : (-b + sqrt(disc)) / a;
    axpy(o, t, k, h);
    cyl_coords(c, h, rho, &z);
    double dz = fabs(z - c->z_c);
    double sp = dot(rho, E->o_plus), sm = dot(rho, E->o_minus);
    note(margin, c->length / 2.0 - dz);
    note(margin, sp);
    note(margin, sm);
    if (dz <= c->length / 2.0 && sp <= 0.0 && sm <= 0.0) {
        *t_out = t;
        return 1;
    }
    return 0;
}

static double exit_distance(const orc_crystal *c, const cyl_edges *E,
                            const double p[3], const double k[3]) {
    double t = INFINITY;
    if (c->geometry == ORC_GEOM_FLAT) {
        double d[3], e2[3];
        sub(p, c->centre, d);
        cross(c->normal, c->e1, e2);
        double zeta = dot(d, c->normal), xi = dot(d, c->e1), eta = dot(d, e2);
        double kn = dot(k, c->normal), k1 = dot(k, c->e1), k2 = dot(k, e2);
        double hl = c->length / 2.0, hw = c->width / 2.0;
        if (kn > 0.0) t = fmin(t, -zeta / kn);
        if (kn < 0.0) t = fmin(t, (-c->thickness - zeta) / kn);
        if (k1 > 0.0) t = fmin(t, (hl - xi) / k1);
        if (k1 < 0.0) t = fmin(t, (-hl - xi) / k1);
        if (k2 > 0.0) t = fmin(t, (hw - eta) / k2);
        if (k2 < 0.0) t = fmin(t, (-hw - eta) / k2);
    } else {
        double rho[3], z, kp[3];
        cyl_coords(c, p, rho, &z);
        double ka = dot(k, c->axis_dir);
        axpy(k, -ka, c->axis_dir, kp);
        double a = dot(kp, kp), b = dot(rho, kp), r2 = dot(rho, rho);
        if (a > 0.0) {
            double ro = c->radius + c->thickness;
            double co = r2 - ro * ro;
            double disc = b * b - a * co;
            if (disc < 0.0) disc = 0.0;
            double to = b >= 0.0 ? -co / (b + sqrt(disc)) : (-b + sqrt(disc)) / a;
            t = fmin(t, to);
            if (b < 0.0) {
                double ci = r2 - c->radius * c->radius;
                double di = b * b - a * ci;
                if (di >= 0.0) t = fmin(t, ci / (-b + sqrt(di)));
            }
        }
        double hl = c->length / 2.0;
        if (ka > 0.0) t = fmin(t, (c->z_c + hl - z) / ka);
        if (ka < 0.0) t = fmin(t, (c->z_c - hl - z) / ka);
        double kop = dot(k, E->o_plus), kom = dot(k, E->o_minus);
        if (kop > 0.0) t = fmin(t, -dot(rho, E->o_plus) / kop);
        if (kom > 0.0) t = fmin(t, -dot(rho, E->o_minus) / kom);
    }
    return t > 0.0 ? t : 0.0;
}

double orc_exit_distance(const orc_crystal *c, const double p[3], const double k[3]) {
    cyl_edges E;
    if (c->geometry == ORC_GEOM_CYLINDER) cyl_setup(c, &E);
    return exit_distance(c, &E, p, k);
}

/* Local surface frame at p: N the surface normal facing the source side,
   e1 the length axis (flat) or the cylinder axis, e2 = N x e1. */
static void local_frame(const orc_crystal *c, const double p[3],
                        double N[3], double e1[3], double e2[3]) {
    if (c->geometry == ORC_GEOM_FLAT) {
        memcpy(N, c->normal, sizeof(double) * 3);
        memcpy(e1, c->e1, sizeof(double) * 3);
    } else {
        double rho[3], z;
        cyl_coords(c, p, rho, &z);
        double r = sqrt(dot(rho, rho));
        for (int i = 0; i < 3; ++i) N[i] = -rho[i] / r;
        memcpy(e1, c->axis_dir, sizeof(double) * 3);
    }
    cross(N, e1, e2);
}


/* ------------------------------------------------------------------------ */
/* The paper's own event model (sec. 2.2.3, 2.2.4): free paths at the rate  */
/* mu0 + gamma0 sigma(alpha) of Eq. AnyEvent with gamma0 sigma from Eq.     */
/* SimpleReflXsection, absorption with probability mu0 / mu_eff, otherwise  */
/* a reflection off a crystallite whose (psi, Delta) is drawn by a          */
/* Metropolis-within-Gibbs sampler from the integrand of Eq. ReflXsection.  */
/* The reflection strength is the one the stepping model uses: Q R(Delta) = */
/* r(Delta - Delta_M) / h, the per-encounter reflection probability over    */
/* the mean path between encounters, with the polarisation factor folded    */
/* into r's peak, so the two models agree up to the approximation of Eq.    */
/* SimpleReflXsection (an IRC much narrower than the mosaic).              */
/* ------------------------------------------------------------------------ */

/* Sphere densities of the mosaic distributions (sec. 2.2.2) per steradian,
   normalised over the sphere, as functions of v = 1 - cos(theta). */
static double vmf_density(double gamma, double v) {
    /* Eq. MF: proportional to exp(cos(theta) / s^2) */
    double s = gamma / (2.0 * sqrt(2.0 * log(2.0)));
    double kappa = 1.0 / (s * s);
    return kappa * exp(-kappa * v) / (ORC_TWO_PI * -expm1(-2.0 * kappa));
}

static double cauchy_density(double gamma, double v) {
    /* the bivariate Cauchy tilt of lorentz_tilt: planar density
       g / (2 pi (g^2 + T^2)^(3/2)) at T = tan(theta), times the gnomonic
       area ratio 1 / cos^3(theta); zero on the far hemisphere */
    double c = 1.0 - v;
    if (!(c > 0.0)) return 0.0;
    double g = gamma / 2.0;
    double q = v * (2.0 - v) + g * g * c * c;   /* sin^2 + g^2 cos^2 */
    return g / (ORC_TWO_PI * q * sqrt(q));
}

static double gauss_density(double gamma, double v) {
    /* the Gaussian tilt of gauss_tilt: planar density
       exp(-T^2 / (2 s^2)) / (2 pi s^2) at T = tan(theta), times the
       gnomonic area ratio 1 / cos^3(theta); zero on the far hemisphere */
    double c = 1.0 - v;
    if (!(c > 0.0)) return 0.0;
    double s = gamma / (2.0 * sqrt(2.0 * log(2.0)));
    double T2 = v * (2.0 - v) / (c * c);
    return exp(-T2 / (2.0 * s * s)) / (ORC_TWO_PI * s * s * c * c * c);
}

double orc_mdf_density(const orc_mosaic *m, double v) {
    double gamma = m->fwhm;
    switch (m->kind) {
    case ORC_MDF_VMF:
        return vmf_density(gamma, v);
    case ORC_MDF_LORENTZ:
        return cauchy_density(gamma, v);
    case ORC_MDF_PVOIGT:
        return m->eta * cauchy_density(gamma, v) + (1.0 - m->eta) * vmf_density(gamma, v);
    case ORC_MDF_WRAPPED_LORENTZ: {
        /* Eq. WL: proportional to 1 / (g^2 + 2 v), v in [0, 2] */
        double g = gamma / 2.0;
        double Z = log((g * g + 4.0) / (g * g));
        return 1.0 / (ORC_PI * Z * (g * g + 2.0 * v));
    }
    case ORC_MDF_SPHERICAL_WRAPPED_LORENTZ: {
        /* Eq. SWL: proportional to 1 / (cosh(Gamma/2) - 1 + v)^2, with
           cosh(Gamma/2) - 1 = 2 sinh^2(Gamma/4) free of cancellation */
        double sh = sinh(gamma / 4.0);
        double A = 2.0 * sh * sh;
        return A * (A + 2.0) / (2.0 * ORC_TWO_PI * (A + v) * (A + v));
    }
    case ORC_MDF_GAUSSIAN:
        return gauss_density(gamma, v);
    }
    return 0.0;
}

/* v = 1 - cos(theta(alpha, psi, beta)) of Eq. ThetaPsi, written without
   cancellation: 2 sin^2((alpha - beta)/2) + 2 cos(alpha) cos(beta) sin^2(psi/2). */
static double theta_v(double alpha, double beta, double psi) {
    double a = sin((alpha - beta) / 2.0), b = sin(psi / 2.0);
    return 2.0 * a * a + 2.0 * cos(alpha) * cos(beta) * b * b;
}

/* The psi integral of Eq. SimpleReflXsection, int W(theta(alpha, psi, beta))
   dpsi over [-pi, pi], by the trapezoid rule on the nodes
   psi_j = pi (j / M)^3, j = 0..M, dense near psi = 0 where the integrand
   peaks; the integrand is even in psi. */
double orc_psi_integral(const orc_mosaic *m, double alpha, double beta, int M) {
    double a = sin((alpha - beta) / 2.0);
    double v0 = 2.0 * a * a, cc = 2.0 * cos(alpha) * cos(beta);
    double prev_psi = 0.0, prev_f = orc_mdf_density(m, v0), sum = 0.0;
    for (int j = 1; j <= M; ++j) {
        double t = (double)j / (double)M;
        double psi = ORC_PI * t * t * t;
        double b = sin(psi / 2.0);
        double f = orc_mdf_density(m, v0 + cc * b * b);
        sum += (psi - prev_psi) * (prev_f + f) / 2.0;
        prev_psi = psi;
        prev_f = f;
    }
    return 2.0 * sum;
}

/* The polarisation angle phi of a ray about its direction (sec. 2.2.3):
   cos(phi) = p.(N x k) / cos(alpha) as the paper defines it, and
   sin(phi) = p.u with u the unit component of N normal to k,
   (N + sin(alpha) k) / cos(alpha), so that G(Delta, phi - psi) below equals
   1 - (p.k_s)^2 for the crystallite at azimuth psi (the paper's first form
   of G; pinned). */
double orc_polarisation_angle(const double p[3], const double N[3], const double k[3],
                              double alpha) {
    double ca = cos(alpha), sa = sin(alpha), nk[3], u[3];
    cross(N, k, nk);
    for (int i = 0; i < 3; ++i) u[i] = (N[i] + sa * k[i]) / ca;
    return atan2(dot(p, u), dot(p, nk) / ca);
}

/* G(Delta, phi - psi) = 1 - sin^2(2 b) sin^2(phi - psi), b = alpha_B + Delta:
   the polarisation factor of a crystallite at azimuth psi (Eq. G_pol). */
static double g_pol(double b, double phi, double psi) {
    double s2 = sin(2.0 * b), sp = sin(phi - psi);
    return 1.0 - s2 * s2 * sp * sp;
}

/* The psi integral of Eq. SimpleReflXsectionPol, int W(theta(alpha, psi,
   beta)) G(beta, phi - psi) dpsi over [-pi, pi], by the trapezoid rule on
   the nodes -psi_M .. -psi_1, 0, psi_1 .. psi_M (psi_j = pi (j / M)^3). */
double orc_psi_integral_pol(const orc_mosaic *m, double alpha, double beta, double phi, int M) {
    double sum = 0.0;
    for (int side = -1; side <= 1; side += 2) {
        double prev_psi = 0.0;
        double prev_f = orc_mdf_density(m, theta_v(alpha, beta, 0.0)) * g_pol(beta, phi, 0.0);
        for (int j = 1; j <= M; ++j) {
            double t = (double)j / (double)M;
            double psi = side * ORC_PI * t * t * t;
            double f = orc_mdf_density(m, theta_v(alpha, beta, psi)) * g_pol(beta, phi, psi);
            sum += fabs(psi - prev_psi) * (prev_f + f) / 2.0;
            prev_psi = psi;
            prev_f = f;
        }
    }
    return sum;
}

/* int r(x) dx over the whole curve (closed forms; the table by the
   trapezoid rule, exact for its linear interpolation). */
double orc_irc_integral(const orc_irc *irc) {
    switch (irc->kind) {
    case ORC_IRC_GAUSS:
        return irc->peak * irc->fwhm * sqrt(ORC_PI / (4.0 * log(2.0)));
    case ORC_IRC_PVOIGT: {
        double w, eta;
        orc_pvoigt_params(irc->fwhm_g, irc->fwhm_l, &w, &eta);
        return irc->peak / (eta * lorentz_unit(0.0, w) + (1.0 - eta) * gauss_unit(0.0, w));
    }
    case ORC_IRC_TABLE: {
        int n = irc->n_table;
        double sum = 0.0;
        for (int j = 0; j + 1 < n; ++j) sum += (irc->table[j] + irc->table[j + 1]) / 2.0;
        return sum * (irc->x_max - irc->x_min) / (double)(n - 1);
    }
    case ORC_IRC_LORENTZ:
        return irc->peak * ORC_PI * irc->fwhm / 2.0;
    case ORC_IRC_BOX:
        return irc->peak * irc->fwhm;
    }
    return 0.0;
}

/* Step width of the sampler's Delta proposals: the IRC's full width at half
   maximum (for the table, the span of its nodes at or above half its
   maximum). */
double orc_irc_width(const orc_irc *irc) {
    switch (irc->kind) {
    case ORC_IRC_PVOIGT: {
        double w, eta;
        orc_pvoigt_params(irc->fwhm_g, irc->fwhm_l, &w, &eta);
        return w;
    }
    case ORC_IRC_TABLE: {
        double mx = irc_max(irc);
        int cnt = 0;
        for (int j = 0; j < irc->n_table; ++j) cnt += irc->table[j] >= mx / 2.0;
        return (double)cnt * (irc->x_max - irc->x_min) / (double)(irc->n_table - 1);
    }
    default:
        return irc->fwhm;
    }
}

/* Integrand of Eq. ReflXsection in (psi, Delta) up to a constant: the
   target of the sampler.  ab = alpha_B; b = alpha_B + Delta is the angle of
   incidence on the crystallite. */
static double mwg_target(const orc_mosaic *m, const orc_irc *irc, double shift, double scale,
                         double alpha, double ab, double psi, double delta, const double *phi) {
    /* a further plane set reads the curve at (Delta - its shift) / its scale */
    double r = orc_irc_value(irc, scale == 1.0 ? delta - shift : (delta - shift) / scale);
    if (!(r > 0.0)) return 0.0;
    double b = ab + delta;
    double f = r * cos(b) * orc_mdf_density(m, theta_v(alpha, b, psi));
    /* polarised: the integrand of Eq. ReflXsectionPol */
    return phi ? f * g_pol(b, *phi, psi) : f;
}

/* Metropolis-within-Gibbs draw of (psi, Delta) (sec. 2.2.4): from
   (0, Delta_M), `burn_in` sweeps, each a psi move and then (moves_delta;
   with the IRC disabled, sec. 2.2.1, Delta stays at Delta_M) a Delta move,
   both symmetric uniform random walks (half-widths w_psi and w_delta); a
   move is taken when u f(current) < f(proposed), or from a point of zero
   density; Delta outside [-alpha_B, pi/2 - alpha_B] is rejected; psi wraps
   on [-pi, pi).  Sweep s of event e uses the Philox words of counter
   (s, ray, 2^31 + e). */
static void mwg_sample(const orc_mosaic *m, const orc_irc *irc, double shift, double scale,
                       double w_psi, double w_delta, uint64_t seed, uint64_t ray, uint32_t event,
                       int burn_in, int moves_delta, double alpha, double ab, const double *phi,
                       double *psi_out, double *delta_out, double *margin) {
    double lo = -ab, hi = ORC_PI / 2.0 - ab;
    double psi = 0.0, delta = shift;
    if (delta < lo) delta = lo;
    if (delta > hi) delta = hi;
    double f = mwg_target(m, irc, shift, scale, alpha, ab, psi, delta, phi);
    for (int s = 0; s < burn_in; ++s) {
        double u[4];
        ray_words(seed, ray, 0x80000000u | event, (uint32_t)s, u);
        double pn = psi + w_psi * (2.0 * u[0] - 1.0);
        if (pn >= ORC_PI) pn -= ORC_TWO_PI;
        else if (pn < -ORC_PI) pn += ORC_TWO_PI;
        double fn = mwg_target(m, irc, shift, scale, alpha, ab, pn, delta, phi);
        if (margin && f > 0.0 && fn > 0.0) note(margin, (fn - u[1] * f) / fmax(fn, u[1] * f));
        if (u[1] * f < fn || f == 0.0) {
            psi = pn;
            f = fn;
        }
        if (!moves_delta) continue;
        double dn = delta + w_delta * (2.0 * u[2] - 1.0);
        if (dn >= lo && dn <= hi) {
            fn = mwg_target(m, irc, shift, scale, alpha, ab, psi, dn, phi);
            if (margin && f > 0.0 && fn > 0.0) note(margin, (fn - u[3] * f) / fmax(fn, u[3] * f));
            if (u[3] * f < fn || f == 0.0) {
                delta = dn;
                f = fn;
            }
        }
    }
    *psi_out = psi;
    *delta_out = delta;
}

void orc_mwg_sample(const orc_mosaic *m, const orc_irc *irc, double w_psi, double w_delta,
                    uint64_t seed, uint64_t ray, uint32_t event, int burn_in,
                    double alpha, double ab, double *psi_out, double *delta_out,
                    double *margin) {
    mwg_sample(m, irc, irc->shift, 1.0, w_psi, w_delta, seed, ray, event, burn_in, 1, alpha, ab,
               NULL, psi_out, delta_out, margin);
}

void orc_mwg_sample_pol(const orc_mosaic *m, const orc_irc *irc, double w_psi, double w_delta,
                        uint64_t seed, uint64_t ray, uint32_t event, int burn_in,
                        double alpha, double ab, double phi, double *psi_out, double *delta_out,
                        double *margin) {
    mwg_sample(m, irc, irc->shift, 1.0, w_psi, w_delta, seed, ray, event, burn_in, 1, alpha, ab,
               &phi, psi_out, delta_out, margin);
}

void orc_mwg_sample_psi(const orc_mosaic *m, const orc_irc *irc, double w_psi,
                        uint64_t seed, uint64_t ray, uint32_t event, int burn_in,
                        double alpha, double ab, double *psi_out, double *delta_out,
                        double *margin) {
    mwg_sample(m, irc, irc->shift, 1.0, w_psi, 0.0, seed, ray, event, burn_in, 0, alpha, ab,
               NULL, psi_out, delta_out, margin);
}

/* Crystallite normal for glancing angle alpha on the planes of normal N
   (sin(alpha) = -k.N), angle of incidence b on the crystallite and
   rotation psi about the ray (sec. 2.2.2): N rotated by alpha - b about
   N x k, then by psi about k (Rodrigues' formula both times). */
void orc_crystallite(const double N[3], const double k[3], double alpha, double b,
                     double psi, double n[3]) {
    double th = alpha - b, ca = cos(alpha), sa = sin(alpha);
    double n0[3], kx[3];
    for (int i = 0; i < 3; ++i)   /* (k + sin(alpha) N) / cos(alpha) is the unit (N x k) x N */
        n0[i] = ca > 0.0 ? cos(th) * N[i] + sin(th) * (k[i] + sa * N[i]) / ca : N[i];
    cross(k, n0, kx);
    double kn0 = dot(k, n0), cp = cos(psi), sp = sin(psi);
    for (int i = 0; i < 3; ++i) n[i] = cp * n0[i] + sp * kx[i] + (1.0 - cp) * kn0 * k[i];
}

/* ------------------------------------------------------------------------ */
/* Detector (sec. 2.3): a rectangle of nx x ny square pixels.                */
/* ------------------------------------------------------------------------ */
static int detector_hit(const orc_detector *D, const double q[3], const double k[3],
                        double h[3], int *pi, int *pj, double *margin) {
    double kn = dot(k, D->normal);
    if (!(kn < 0.0)) return 0;
    double d[3];
    sub(D->centre, q, d);
    double t = dot(d, D->normal) / kn;
    if (!(t > 0.0)) return 0;
    axpy(q, t, k, h);
    sub(h, D->centre, d);
    double fu = dot(d, D->u) / D->pitch + (double)D->nx / 2.0;
    double fv = dot(d, D->v) / D->pitch + (double)D->ny / 2.0;
    note(margin, fu - nearbyint(fu));
    note(margin, fv - nearbyint(fv));
    double i = floor(fu), j = floor(fv);
    if (i < 0.0 || j < 0.0 || i >= (double)D->nx || j >= (double)D->ny) return 0;
    *pi = (int)i;
    *pj = (int)j;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* One ray, end to end.                                                      */
/* ------------------------------------------------------------------------ */
typedef struct trace_ctx {
    const orc_source *s;
    const orc_crystal *c;
    const orc_mosaic *m;
    const orc_irc *irc;
    const orc_detector *d;
    cyl_edges E;
    uint64_t seed;
    uint32_t max_events;
    double r_max, mu_tot, p_a;
    double plane_tot;        /* sum of the plane sets' peaks, both sides */
    /* the paper's event model */
    int mwg;                 /* 1: event model of sec. 2.2.3-2.2.4 */
    int burn_in, psi_nodes, irc_off;
    double q;                /* int r dx / h */
    double w_delta;          /* sampler step in Delta */
} trace_ctx;

static void ctx_init(trace_ctx *X, const orc_source *s, const orc_crystal *c,
                     const orc_mosaic *m, const orc_irc *irc, const orc_detector *d,
                     const orc_model *model, uint64_t seed, uint32_t max_events) {
    memset(X, 0, sizeof(*X));
    if (model && model->kind == ORC_MODEL_MWG) {
        X->mwg = 1;
        X->burn_in = model->burn_in;
        X->psi_nodes = model->psi_nodes;
        X->irc_off = model->irc_off;
        X->q = orc_irc_integral(irc) / c->mfp;
        X->w_delta = orc_irc_width(irc);
    }
    X->s = s; X->c = c; X->m = m; X->irc = irc; X->d = d;
    X->seed = seed;
    X->max_events = max_events ? max_events : (1u << 20);
    if (c->geometry == ORC_GEOM_CYLINDER) cyl_setup(c, &X->E);
    /* majorant encounter rate lambda_c = R_max / h; every encounter is a
       candidate reflection accepted with probability r / R_max */
    X->r_max = irc_max(irc);
    double lambda_c = X->r_max / c->mfp;
    /* with further planes each set and side is a candidate at its own
       peak: the majorant is the sum of the peaks */
    X->plane_tot = 1.0;
    if (c->planes) {
        double sum = 1.0;
        for (int j = 0; j < c->planes->n_extra; ++j) sum += c->planes->strength[j];
        X->plane_tot = sum * fmax(1.0, c->planes->hbar_ratio);
        lambda_c = X->r_max * X->plane_tot / c->mfp;
    }
    X->mu_tot = c->mu0 + lambda_c;
    X->p_a = X->mu_tot > 0.0 ? c->mu0 / X->mu_tot : 1.0;
}


/* Events of one ray in the paper's model (sec. 2.2.3, 2.2.4).  Event i draws
   (u0, u1, u2) = the Philox words of counter (i, ray, 1): the free path
   -ln(u0) / mu_eff with mu_eff = mu0 + gamma0 sigma_H(alpha) +
   gamma0 sigma_anti-H(-alpha) at the event's start point (sin(alpha) =
   -k.N there; the normal is held along the path, the paper's assumption),
   exit when the path reaches the boundary, absorption when
   u1 <= mu0 / mu_eff, otherwise a reflection off the H planes (normal N)
   when u2 sigma < sigma_H, else off the anti-H planes (normal -N). */
/* The psi integral of W (or of W G with a polarisation at angle phi). */
static double psi_int(const trace_ctx *X, double alpha, double beta, const double *phi) {
    return phi ? orc_psi_integral_pol(X->m, alpha, beta, *phi, X->psi_nodes)
               : orc_psi_integral(X->m, alpha, beta, X->psi_nodes);
}

/* With further plane sets (sec. 2.2.3, closing paragraphs) the attenuation
   sums the H and anti-H terms of every set j, each with its own Bragg angle
   alpha_B,j, shift Delta_M,j and curve r((x - Delta_M,j) / s_j) of peak
   strength a_j (so its integral is a_j s_j int r), the anti-H terms times
   hbar_ratio; the reflecting set and side are then drawn by their shares,
   in the order H_0, anti-H_0, H_1, ..., and the crystallite is sampled for
   that set. */
static void mwg_events_planes(const trace_ctx *X, uint64_t ray, double E, double p[3],
                              double k[3], double *pol, uint32_t *n_ev, uint32_t *n_rf,
                              int *status, double *m) {
    const orc_crystal *c = X->c;
    const orc_planes *pl = c->planes;
    const orc_irc *q = X->irc;
    int nset = 1 + (pl ? pl->n_extra : 0);
    double hbar = pl ? pl->hbar_ratio : 1.0;
    double ab[4], shift[4], scale[4], strength[4];
    for (int j = 0; j < nset; ++j) {
        ab[j] = orc_bragg_angle(E, j ? pl->two_d[j - 1] : c->two_d);
        shift[j] = j ? pl->shift[j - 1] : q->shift;
        scale[j] = j ? pl->width_scale[j - 1] : 1.0;
        strength[j] = j ? pl->strength[j - 1] : 1.0;
    }
    if (q->n_dep > 0) {
        /* the energy-dependent curve (sec. 2.2.1) is the main set's shift
           Delta_M(E) and width scale s(E) */
        shift[0] = interp_clamped(q->dep_kev, q->dep_shift, q->n_dep, E);
        scale[0] = interp_clamped(q->dep_kev, q->dep_scale, q->n_dep, E);
    }
    uint32_t n_events = 0, n_refl = 0;
    for (;;) {
        if (n_events == X->max_events) { *status = ORC_TRUNCATED; break; }
        double u[4];
        ray_words(X->seed, ray, 1, n_events, u);
        uint32_t event = n_events++;
        double dist = exit_distance(c, &X->E, p, k);
        double N[3], e1[3], e2[3];
        local_frame(c, p, N, e1, e2);
        double sn = -dot(k, N);
        if (sn > 1.0) sn = 1.0;
        if (sn < -1.0) sn = -1.0;
        double alpha = asin(sn);
        double minus_N[3] = {-N[0], -N[1], -N[2]};
        double phi_h = pol ? orc_polarisation_angle(pol, N, k, alpha) : 0.0;
        double phi_a = pol ? orc_polarisation_angle(pol, minus_N, k, -alpha) : 0.0;
        double sh[4], sa[4], sum = 0.0;
        for (int j = 0; j < nset; ++j) {
            sh[j] = sa[j] = 0.0;
            if (ab[j] >= 0.0 && (int)n_refl < c->max_refl) {
                double beta = ab[j] + shift[j];
                double qc = X->q * (strength[j] * scale[j]) * cos(beta);
                sh[j] = qc * psi_int(X, alpha, beta, pol ? &phi_h : NULL);
                sa[j] = hbar * qc * psi_int(X, -alpha, beta, pol ? &phi_a : NULL);
            }
            sum += sh[j];
            sum += sa[j];
        }
        double mu = c->mu0 + sum;
        double l = -log(u[0]) / mu;
        note(m, (l - dist) / fmax(l, dist));
        if (l >= dist) {
            axpy(p, dist, k, p);
            *status = n_refl ? ORC_EXIT_REFLECTED : ORC_EXIT_TRANSMITTED;
            break;
        }
        axpy(p, l, k, p);
        double pa = c->mu0 / mu;
        note(m, u[1] - pa);
        if (u[1] <= pa) { *status = ORC_ABSORBED; break; }
        double target = u[2] * sum, acc = 0.0;
        int js = nset - 1, anti = 1;
        for (int j = 0; j < nset; ++j) {
            acc += sh[j];
            note(m, (acc - target) / sum);
            if (target < acc) { js = j; anti = 0; break; }
            acc += sa[j];
            note(m, (acc - target) / sum);
            if (target < acc) { js = j; anti = 1; break; }
        }
        double Ns[3];
        for (int i = 0; i < 3; ++i) Ns[i] = anti ? -N[i] : N[i];
        double as = anti ? -alpha : alpha;
        double cb = cos(ab[js] + shift[js]);
        double w_psi = X->m->fwhm / (cb > 0.05 ? cb : 0.05);
        double psi, delta, n[3], ks[3];
        double phi_s = anti ? phi_a : phi_h;
        mwg_sample(X->m, X->irc, shift[js], scale[js], w_psi, X->w_delta * scale[js], X->seed, ray,
                   event, X->burn_in, !X->irc_off, as, ab[js], pol ? &phi_s : NULL, &psi, &delta, m);
        orc_crystallite(Ns, k, as, ab[js] + delta, psi, n);
        axpy(k, -2.0 * dot(k, n), n, ks);
        double nr = sqrt(dot(ks, ks));
        for (int i = 0; i < 3; ++i) k[i] = ks[i] / nr;
        if (pol) {
            double pks = dot(pol, k), g = sqrt(1.0 - pks * pks);
            for (int i = 0; i < 3; ++i) pol[i] = (pol[i] - pks * k[i]) / g;
        }
        ++n_refl;
    }
    *n_ev = n_events;
    *n_rf = n_refl;
}

static void mwg_events(const trace_ctx *X, uint64_t ray, double alpha_b, double p[3],
                       double k[3], double *pol, uint32_t *n_ev, uint32_t *n_rf, int *status,
                       double *m) {
    const orc_crystal *c = X->c;
    uint32_t n_events = 0, n_refl = 0;
    double beta = alpha_b + X->irc->shift, cos_beta = cos(beta);
    double cb = cos_beta > 0.05 ? cos_beta : 0.05;
    double w_psi = X->m->fwhm / cb;
    for (;;) {
        if (n_events == X->max_events) { *status = ORC_TRUNCATED; break; }
        double u[4];
        ray_words(X->seed, ray, 1, n_events, u);
        uint32_t event = n_events++;
        double dist = exit_distance(c, &X->E, p, k);
        double N[3], e1[3], e2[3];
        local_frame(c, p, N, e1, e2);
        double sn = -dot(k, N);
        if (sn > 1.0) sn = 1.0;
        if (sn < -1.0) sn = -1.0;
        double alpha = asin(sn);
        double sig_h = 0.0, sig_a = 0.0;
        /* with polarisation, the angle of p about k seen from either side */
        double minus_N[3] = {-N[0], -N[1], -N[2]};
        double phi_h = pol ? orc_polarisation_angle(pol, N, k, alpha) : 0.0;
        double phi_a = pol ? orc_polarisation_angle(pol, minus_N, k, -alpha) : 0.0;
        if (alpha_b >= 0.0 && (int)n_refl < c->max_refl) {
            if (pol) {
                sig_h = X->q * cos_beta * orc_psi_integral_pol(X->m, alpha, beta, phi_h, X->psi_nodes);
                sig_a = X->q * cos_beta * orc_psi_integral_pol(X->m, -alpha, beta, phi_a, X->psi_nodes);
            } else {
                sig_h = X->q * cos_beta * orc_psi_integral(X->m, alpha, beta, X->psi_nodes);
                sig_a = X->q * cos_beta * orc_psi_integral(X->m, -alpha, beta, X->psi_nodes);
            }
        }
        double mu = c->mu0 + sig_h + sig_a;
        double l = -log(u[0]) / mu;
        note(m, (l - dist) / fmax(l, dist));
        if (l >= dist) {
            axpy(p, dist, k, p);
            *status = n_refl ? ORC_EXIT_REFLECTED : ORC_EXIT_TRANSMITTED;
            break;
        }
        axpy(p, l, k, p);
        double pa = c->mu0 / mu;
        note(m, u[1] - pa);
        if (u[1] <= pa) { *status = ORC_ABSORBED; break; }
        double sig = sig_h + sig_a;
        note(m, (sig_h - u[2] * sig) / sig);
        int anti = !(u[2] * sig < sig_h);
        double Ns[3];
        for (int i = 0; i < 3; ++i) Ns[i] = anti ? -N[i] : N[i];
        double as = anti ? -alpha : alpha;
        double psi, delta, n[3], ks[3];
        double phi_s = anti ? phi_a : phi_h;
        mwg_sample(X->m, X->irc, X->irc->shift, 1.0, w_psi, X->w_delta, X->seed, ray, event,
                   X->burn_in, !X->irc_off, as, alpha_b, pol ? &phi_s : NULL, &psi, &delta, m);
        orc_crystallite(Ns, k, as, alpha_b + delta, psi, n);
        /* reflection equation of sec. 2.2.4 */
        axpy(k, -2.0 * dot(k, n), n, ks);
        double nr = sqrt(dot(ks, ks));
        for (int i = 0; i < 3; ++i) k[i] = ks[i] / nr;
        if (pol) {
            /* the polarisation after the reflection (sec. 2.2.4) */
            double pks = dot(pol, k), g = sqrt(1.0 - pks * pks);
            for (int i = 0; i < 3; ++i) pol[i] = (pol[i] - pks * k[i]) / g;
        }
        ++n_refl;
    }
    *n_ev = n_events;
    *n_rf = n_refl;
}

static void trace_one(const trace_ctx *X, uint64_t ray, orc_record *rec, double *margin) {
    const orc_crystal *c = X->c;
    double o[3], k[3], E, p[3], t_in;
    double m = INFINITY;
    memset(rec, 0, sizeof(*rec));
    rec->ray_id = ray;
    rec->pix_i = rec->pix_j = -1;

    orc_source_sample(X->s, X->seed, ray, o, k, &E);
    rec->energy = E;
    /* polarisation, when the user supplies it (sec. 2.1) */
    int polarised = X->s->user_p != NULL;
    double pol[3] = {0.0, 0.0, 0.0};
    if (polarised)
        for (int i = 0; i < 3; ++i) pol[i] = X->s->user_p[3 * (ray - X->s->user_first) + i];
    if (!crystal_entry(c, &X->E, o, k, &t_in, &m)) {
        rec->status = ORC_MISS;
        for (int i = 0; i < 3; ++i) {
            rec->entry[i] = NAN;
            rec->end[i] = NAN;
            rec->dir[i] = k[i];
        }
        *margin = m;
        return;
    }
    axpy(o, t_in, k, p);
    memcpy(rec->entry, p, sizeof(p));

    double alpha_b = orc_bragg_angle(E, c->two_d);
    int can_reflect = alpha_b >= 0.0;
    uint32_t n_events = 0, n_refl = 0;
    int status = ORC_TRUNCATED;

    if (X->mwg) {
        if (c->planes || X->irc->n_dep > 0)
            mwg_events_planes(X, ray, E, p, k, polarised ? pol : NULL, &n_events, &n_refl, &status, &m);
        else
            mwg_events(X, ray, alpha_b, p, k, polarised ? pol : NULL, &n_events, &n_refl, &status, &m);
        goto finish;
    }
    for (;;) {
        if (n_events == X->max_events) { status = ORC_TRUNCATED; break; }
        double u[4];
        ray_words(X->seed, ray, 1, n_events, u);
        ++n_events;
        double dist = exit_distance(c, &X->E, p, k);

        if ((int)n_refl >= c->max_refl) {
            /* reflection budget spent: only Beer-Lambert absorption remains */
            double l = -log(u[0]) / c->mu0;
            note(&m, (l - dist) / fmax(l, dist));
            if (l < dist) { axpy(p, l, k, p); status = ORC_ABSORBED; }
            else { axpy(p, dist, k, p); status = n_refl ? ORC_EXIT_REFLECTED : ORC_EXIT_TRANSMITTED; }
            break;
        }
        /* free path to the next event, Eq. AnyEvent with the majorant rate */
        double l = -log(u[0]) / X->mu_tot;
        note(&m, (l - dist) / fmax(l, dist));
        if (l >= dist) {
            axpy(p, dist, k, p);
            status = n_refl ? ORC_EXIT_REFLECTED : ORC_EXIT_TRANSMITTED;
            break;
        }
        axpy(p, l, k, p);
        /* absorb or reflect: absorbed when u < mu0 / mu_eff */
        note(&m, u[1] - X->p_a);
        if (u[1] < X->p_a) { status = ORC_ABSORBED; break; }
        if (!can_reflect) continue;
        double u_acc = (u[1] - X->p_a) / (1.0 - X->p_a);

        /* crystallite normal from the mosaic distribution about the local
           surface normal */
        double N[3], e1[3], e2[3], n[3];
        local_frame(c, p, N, e1, e2);
        orc_mdf_sample(X->m, u[2], u[3], N, e1, e2, n);

        /* deviation from the Bragg angle on this crystallite; |k.n| covers
           the H and anti-H planes alike */
        double kn = dot(k, n);
        double akn = fabs(kn);
        if (akn > 1.0) akn = 1.0;
        double delta = asin(akn) - alpha_b;
        double arg = delta - X->irc->shift;
        if (X->irc->n_dep > 0) {
            /* the curve of this energy (sec. 2.2.1): shifted to Delta_M(E),
               its width scaled by s(E) */
            const orc_irc *q = X->irc;
            double sh = interp_clamped(q->dep_kev, q->dep_shift, q->n_dep, E);
            double sc = interp_clamped(q->dep_kev, q->dep_scale, q->n_dep, E);
            arg = (delta - sh) / sc;
        }
        double ratio = orc_irc_value(X->irc, arg) / X->r_max;
        /* the reflected direction (reflection equation of sec. 2.2.4) and,
           with polarisations, the factor G = 1 - (p.k_s)^2 of sec. 2.2.3 */
        double ks[3];
        axpy(k, -2.0 * kn, n, ks);
        double nr = sqrt(dot(ks, ks));
        for (int i = 0; i < 3; ++i) ks[i] /= nr;
        double pks = 0.0, G = 1.0;
        if (polarised) {
            pks = dot(pol, ks);
            G = 1.0 - pks * pks;
        }
        int reflect;
        if (c->planes) {
            /* several plane sets and the two sides (sec. 2.2.3): the
               candidate reflects with the summed probability of every set
               j, sum_j a_j r_j(Delta_j), times hbar_ratio when the ray
               travels along n (it meets the antiparallel planes), over the
               majorant sum of the peaks.  The reflected direction is the
               same whichever set reflects, so none is chosen. */
            const orc_planes *pl = c->planes;
            double a = asin(akn);
            double sum = 0.0;
            for (int j = 0; j <= pl->n_extra; ++j) {
                double ab = j ? orc_bragg_angle(E, pl->two_d[j - 1]) : alpha_b;
                if (ab < 0.0) continue;
                double sh = j ? pl->shift[j - 1] : X->irc->shift;
                double sc = j ? pl->width_scale[j - 1] : 1.0;
                double st = j ? pl->strength[j - 1] : 1.0;
                sum += st * (orc_irc_value(X->irc, ((a - ab) - sh) / sc) / X->r_max);
            }
            double side = kn < 0.0 ? 1.0 : pl->hbar_ratio;
            double lhs = u_acc * X->plane_tot, rhs = G * (side * sum);
            note(&m, (lhs - rhs) / X->plane_tot);
            reflect = lhs < rhs;
        } else {
            note(&m, u_acc - G * ratio);
            reflect = u_acc < G * ratio;
        }
        if (reflect) {
            for (int i = 0; i < 3; ++i) k[i] = ks[i];
            if (polarised) {
                /* the polarisation after the reflection (sec. 2.2.4): its
                   component along k_s removed, renormalised */
                double g = sqrt(1.0 - pks * pks);
                for (int i = 0; i < 3; ++i) pol[i] = (pol[i] - pks * ks[i]) / g;
            }
            ++n_refl;
        }
    }

finish:
    rec->status = (uint8_t)status;
    rec->n_events = n_events;
    rec->n_refl = (uint16_t)n_refl;
    memcpy(rec->end, p, sizeof(p));
    memcpy(rec->dir, k, sizeof(k));
    if (status == ORC_EXIT_REFLECTED || status == ORC_EXIT_TRANSMITTED) {
        double h[3];
        int pi, pj;
        if (detector_hit(X->d, p, k, h, &pi, &pj, &m)) {
            rec->detected = 1;
            rec->pix_i = pi;
            rec->pix_j = pj;
            memcpy(rec->end, h, sizeof(h));
        }
    }
    *margin = m;
}

/* The polarisation factor and the polarisation after a reflection
   (sec. 2.2.3, 2.2.4) for a polarisation p and a reflected direction k_s,
   both unit: returns G = 1 - (p.k_s)^2 and writes the new polarisation. */
double orc_polarisation_reflect(const double p[3], const double ks[3], double out[3]) {
    double pks = dot(p, ks);
    double g = sqrt(1.0 - pks * pks);
    for (int i = 0; i < 3; ++i) out[i] = (p[i] - pks * ks[i]) / g;
    return 1.0 - pks * pks;
}

/* Energy a detected photon adds to the energy image (sec. 3): E, or E times
   the detector's quantum efficiency, the user's table interpolated linearly
   at E with the end values held outside it. */
static double detected_energy(const orc_detector *D, double E) {
    if (D->n_qe <= 0) return E;
    return E * interp_clamped(D->qe_kev, D->qe, D->n_qe, E);
}

/* ------------------------------------------------------------------------ */
/* Threaded driver: contiguous ray-id blocks, integer image accumulation.    */
/* ------------------------------------------------------------------------ */
typedef struct job {
    const trace_ctx *X;
    uint64_t first, lo, hi;
    const uint64_t *ids;
    uint32_t *counts;
    uint64_t *energy;
    orc_record *records;
    double *margins;
    orc_counters cnt;
} job;

static void *run_job(void *arg) {
    job *J = (job *)arg;
    const orc_detector *D = J->X->d;
    for (uint64_t i = J->lo; i < J->hi; ++i) {
        uint64_t ray = J->ids ? J->ids[i] : J->first + i;
        orc_record r;
        double mg;
        trace_one(J->X, ray, &r, &mg);
        J->cnt.emitted++;
        J->cnt.events += r.n_events;
        J->cnt.reflections += r.n_refl;
        switch (r.status) {
        case ORC_MISS: J->cnt.missed++; break;
        case ORC_ABSORBED: J->cnt.absorbed++; break;
        case ORC_EXIT_REFLECTED: J->cnt.exit_reflected++; break;
        case ORC_EXIT_TRANSMITTED: J->cnt.exit_transmitted++; break;
        default: J->cnt.truncated++; break;
        }
        if (r.detected) {
            J->cnt.detected++;
            size_t px = (size_t)r.pix_j * (size_t)D->nx + (size_t)r.pix_i;
            if (J->counts) __atomic_fetch_add(&J->counts[px], 1u, __ATOMIC_RELAXED);
            if (J->energy)
                __atomic_fetch_add(&J->energy[px], (uint64_t)nearbyint(detected_energy(D, r.energy) * 1e6),
                                   __ATOMIC_RELAXED);
        }
        if (J->records) J->records[i] = r;
        if (J->margins) J->margins[i] = mg;
    }
    return NULL;
}

static int validate(const orc_source *s, const orc_crystal *c, const orc_mosaic *m,
                    const orc_irc *irc, const orc_detector *d, const orc_model *model,
                    uint32_t max_events) {
    if (!s || !c || !m || !irc || !d) return -1;
    if (model && model->kind == ORC_MODEL_MWG) {
        if (!(m->fwhm > 0.0)) return -9;               /* W must be a density */
        if (model->burn_in < 0 || model->psi_nodes < 1) return -10;
        if (max_events > 0x7fffffffu) return -11;      /* sampler counter word */
    } else if (model && model->kind != ORC_MODEL_STEPPING) {
        return -12;
    }
    if (c->mfp <= 0.0 || c->mu0 < 0.0 || c->thickness <= 0.0 || c->two_d <= 0.0) return -2;
    if (c->geometry == ORC_GEOM_CYLINDER && !(c->width / (2.0 * c->radius) < ORC_PI / 2.0)) return -3;
    if (m->fwhm < 0.0 || m->eta < 0.0 || m->eta > 1.0) return -4;
    if (irc->kind == ORC_IRC_TABLE && (irc->n_table < 2 || !irc->table)) return -5;
    if (irc->n_dep < 0 || (irc->n_dep > 0 && (!irc->dep_kev || !irc->dep_shift || !irc->dep_scale)))
        return -14;
    for (int i = 0; i < irc->n_dep; ++i)
        if (!(irc->dep_scale[i] > 0.0) || (i && !(irc->dep_kev[i] > irc->dep_kev[i - 1]))) return -14;
    if (c->planes) {
        const orc_planes *pl = c->planes;
        if (!(pl->hbar_ratio >= 0.0) || pl->n_extra < 0 || pl->n_extra > 3) return -17;
        for (int j = 0; j < pl->n_extra; ++j)
            if (!(pl->two_d[j] > 0.0 && pl->two_d[j] <= c->two_d) || !(pl->strength[j] > 0.0) ||
                !(pl->width_scale[j] > 0.0))
                return -17;
        if (irc->n_dep > 0) return -17;
    }

    if (s->spectrum == ORC_SPEC_TABLE && (s->n_bins < 1 || !s->bin_w)) return -6;
    if (s->spot_kind < ORC_SPOT_POINT || s->spot_kind > ORC_SPOT_DISK) return -16;
    if (s->spot_kind != ORC_SPOT_POINT &&
        (!(s->spot_sigma[0] >= 0.0) || !(s->spot_sigma[1] >= 0.0))) return -16;
    if (s->spectrum == ORC_SPEC_LINES && (s->n_lines < 0 || s->n_lines > 8)) return -7;
    if (d->nx <= 0 || d->ny <= 0 || d->pitch <= 0.0) return -8;
    if (d->n_qe < 0 || (d->n_qe > 0 && (!d->qe_kev || !d->qe))) return -13;
    for (int i = 1; i < d->n_qe; ++i)
        if (!(d->qe_kev[i] > d->qe_kev[i - 1])) return -13;
    return 0;
}

static int run_threads(const trace_ctx *X, uint64_t first, uint64_t n, const uint64_t *ids,
                       uint32_t *counts, uint64_t *energy, orc_record *records,
                       orc_counters *counters, double *margins, int n_threads) {
    if (n_threads <= 0) n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads < 1) n_threads = 1;
    if ((uint64_t)n_threads > n) n_threads = n ? (int)n : 1;
    job *jobs = (job *)calloc((size_t)n_threads, sizeof(job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return -20; }
    for (int t = 0; t < n_threads; ++t) {
        jobs[t].X = X;
        jobs[t].first = first;
        jobs[t].lo = n * (uint64_t)t / (uint64_t)n_threads;
        jobs[t].hi = n * (uint64_t)(t + 1) / (uint64_t)n_threads;
        jobs[t].ids = ids;
        jobs[t].counts = counts;
        jobs[t].energy = energy;
        jobs[t].records = records;
        jobs[t].margins = margins;
    }
    for (int t = 1; t < n_threads; ++t) pthread_create(&th[t], NULL, run_job, &jobs[t]);
    run_job(&jobs[0]);
    for (int t = 1; t < n_threads; ++t) pthread_join(th[t], NULL);
    if (counters) {
        memset(counters, 0, sizeof(*counters));
        for (int t = 0; t < n_threads; ++t) {
            counters->emitted += jobs[t].cnt.emitted;
            counters->missed += jobs[t].cnt.missed;
            counters->absorbed += jobs[t].cnt.absorbed;
            counters->exit_reflected += jobs[t].cnt.exit_reflected;
            counters->exit_transmitted += jobs[t].cnt.exit_transmitted;
            counters->truncated += jobs[t].cnt.truncated;
            counters->detected += jobs[t].cnt.detected;
            counters->events += jobs[t].cnt.events;
            counters->reflections += jobs[t].cnt.reflections;
        }
    }
    free(jobs);
    free(th);
    return 0;
}

int orc_trace_model(const orc_source *s, const orc_crystal *c, const orc_mosaic *m,
                    const orc_irc *irc, const orc_detector *d, const orc_model *model,
                    uint64_t first, uint64_t n, uint64_t seed, uint32_t max_events,
                    uint32_t *counts, uint64_t *energy_mev,
                    orc_record *records, orc_counters *counters, double *margins,
                    int n_threads) {
    int e = validate(s, c, m, irc, d, model, max_events);
    if (e) return e;
    trace_ctx X;
    ctx_init(&X, s, c, m, irc, d, model, seed, max_events);
    return run_threads(&X, first, n, NULL, counts, energy_mev, records, counters, margins,
                       n_threads);
}

int orc_trace(const orc_source *s, const orc_crystal *c, const orc_mosaic *m,
              const orc_irc *irc, const orc_detector *d,
              uint64_t first, uint64_t n, uint64_t seed, uint32_t max_events,
              uint32_t *counts, uint64_t *energy_mev,
              orc_record *records, orc_counters *counters, double *margins,
              int n_threads) {
    return orc_trace_model(s, c, m, irc, d, NULL, first, n, seed, max_events, counts,
                           energy_mev, records, counters, margins, n_threads);
}

int orc_trace_ids_model(const orc_source *s, const orc_crystal *c, const orc_mosaic *m,
                        const orc_irc *irc, const orc_detector *d, const orc_model *model,
                        const uint64_t *ids, uint64_t n, uint64_t seed, uint32_t max_events,
                        orc_record *records, double *margins, int n_threads) {
    int e = validate(s, c, m, irc, d, model, max_events);
    if (e) return e;
    trace_ctx X;
    ctx_init(&X, s, c, m, irc, d, model, seed, max_events);
    return run_threads(&X, 0, n, ids, NULL, NULL, records, NULL, margins, n_threads);
}

int orc_trace_ids(const orc_source *s, const orc_crystal *c, const orc_mosaic *m,
                  const orc_irc *irc, const orc_detector *d,
                  const uint64_t *ids, uint64_t n, uint64_t seed, uint32_t max_events,
                  orc_record *records, double *margins, int n_threads) {
    return orc_trace_ids_model(s, c, m, irc, d, NULL, ids, n, seed, max_events, records,
                               margins, n_threads);
}

int orc_version(void) { return 1; }
