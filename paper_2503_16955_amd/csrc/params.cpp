// Validation of the public structs and construction of the kernels'
// parameter block, shared by mrt_trace and the request server.
#include "params.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

namespace mrt {

namespace {
constexpr double kPi = 3.1415926535897932384626433832795;
}  // namespace

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static bool unit(const double *v) { return std::fabs(std::sqrt(dot3(v, v)) - 1.0) <= 1e-12; }
static bool ortho(const double *a, const double *b) { return std::fabs(dot3(a, b)) <= 1e-12; }
static bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

mrt_status validate(const mrt_source *s, const mrt_crystal *c, const mrt_mosaic *m,
                    const mrt_rocking_curve *r, const mrt_detector *d, Failer fail) {
    if (!s || !c || !m || !r || !d) return fail(MRT_EINVAL, "null struct pointer");
    // source
    if (!finite3(s->origin) || !unit(s->axis) || !unit(s->b1) || !ortho(s->axis, s->b1))
        return fail(MRT_EINVAL, "source: axis and b1 must be orthonormal unit vectors");
    if (!(s->half_angle >= 0.0 && s->half_angle < kPi))
        return fail(MRT_EINVAL, "source: half_angle must lie in [0, pi)");
    if (s->spectrum < 0 || s->spectrum > 2) return fail(MRT_EINVAL, "source: unknown spectrum kind");
    if (!(s->e_min > 0.0) || !(s->e_max >= s->e_min))
        return fail(MRT_EINVAL, "source: need 0 < e_min <= e_max");
    if (s->spectrum == MRT_SPECTRUM_LINES) {
        if (s->n_lines < 0 || s->n_lines > 8) return fail(MRT_EINVAL, "source: n_lines must be 0..8");
        double tot = s->background_w;
        if (!(s->background_w >= 0.0)) return fail(MRT_EINVAL, "source: negative background weight");
        for (int j = 0; j < s->n_lines; ++j) {
            if (!(s->line_sigma[j] >= 0.0) || !(s->line_w[j] >= 0.0) || !(s->line_e[j] > 0.0))
                return fail(MRT_EINVAL, "source: line %d needs E > 0, sigma >= 0, weight >= 0", j);
            tot += s->line_w[j];
        }
        if (!(tot > 0.0)) return fail(MRT_EINVAL, "source: all spectrum weights are zero");
    }
    if (s->spectrum == MRT_SPECTRUM_TABLE) {
        if (s->n_bins < 1 || !s->bin_w) return fail(MRT_EINVAL, "source: table spectrum needs n_bins >= 1");
        double tot = 0.0;
        for (int b = 0; b < s->n_bins; ++b) {
            if (!(s->bin_w[b] >= 0.0)) return fail(MRT_EINVAL, "source: negative bin weight");
            tot += s->bin_w[b];
        }
        if (!(tot > 0.0)) return fail(MRT_EINVAL, "source: all bin weights are zero");
    }
    if (s->spot_kind < MRT_SPOT_POINT || s->spot_kind > MRT_SPOT_DISK)
        return fail(MRT_EINVAL, "source: unknown spot kind");
    if (s->spot_kind != MRT_SPOT_POINT) {
        if (!unit(s->spot_u) || !unit(s->spot_v) || !ortho(s->spot_u, s->spot_v))
            return fail(MRT_EINVAL, "source: spot_u and spot_v must be orthonormal unit vectors");
        const int ns = s->spot_kind == MRT_SPOT_GAUSSIAN ? 2 : 1;
        for (int i = 0; i < ns; ++i)
            if (!(s->spot_sigma[i] >= 0.0) || !std::isfinite(s->spot_sigma[i]))
                return fail(MRT_EINVAL, "source: spot_sigma must be finite and >= 0");
    }
    // crystal
    if (c->geometry == MRT_GEOMETRY_FLAT) {
        if (!finite3(c->centre) || !unit(c->normal) || !unit(c->e1) || !ortho(c->normal, c->e1))
            return fail(MRT_EINVAL, "crystal: normal and e1 must be orthonormal unit vectors");
    } else if (c->geometry == MRT_GEOMETRY_CYLINDER) {
        if (!finite3(c->axis_pt) || !unit(c->axis_dir) || !unit(c->ref_dir) ||
            !ortho(c->axis_dir, c->ref_dir))
            return fail(MRT_EINVAL, "crystal: axis_dir and ref_dir must be orthonormal unit vectors");
        if (!(c->radius > 0.0)) return fail(MRT_EINVAL, "crystal: radius must be > 0");
        if (!(c->width / c->radius < kPi)) return fail(MRT_EINVAL, "crystal: width / radius must be < pi");
        if (!std::isfinite(c->phi_c) || !std::isfinite(c->z_c)) return fail(MRT_EINVAL, "crystal: bad phi_c / z_c");
    } else {
        return fail(MRT_EINVAL, "crystal: unknown geometry");
    }
    if (!(c->length > 0.0) || !(c->width > 0.0) || !(c->thickness > 0.0))
        return fail(MRT_EINVAL, "crystal: length, width and thickness must be > 0");
    if (!(c->two_d > 0.0)) return fail(MRT_EINVAL, "crystal: two_d must be > 0");
    if (!(c->mu0 >= 0.0) || !std::isfinite(c->mu0)) return fail(MRT_EINVAL, "crystal: mu0 must be >= 0");
    if (!(c->mfp > 0.0) || !std::isfinite(c->mfp)) return fail(MRT_EINVAL, "crystal: mfp must be > 0");
    if (c->max_refl < 0) return fail(MRT_EINVAL, "crystal: max_refl must be >= 0");
    if (const mrt_planes *pl = c->planes) {
        if (!(pl->hbar_ratio >= 0.0) || !std::isfinite(pl->hbar_ratio))
            return fail(MRT_EINVAL, "planes: hbar_ratio must be finite and >= 0");
        if (pl->n_extra < 0 || pl->n_extra > 3) return fail(MRT_EINVAL, "planes: n_extra must be 0..3");
        for (int j = 0; j < pl->n_extra; ++j) {
            if (!(pl->two_d[j] > 0.0) || !(pl->two_d[j] <= c->two_d))
                return fail(MRT_EINVAL, "planes: two_d[%d] must lie in (0, crystal two_d]", j);
            if (!(pl->strength[j] > 0.0) || !std::isfinite(pl->strength[j]) ||
                !(pl->width_scale[j] > 0.0) || !std::isfinite(pl->width_scale[j]) ||
                !std::isfinite(pl->shift[j]))
                return fail(MRT_EINVAL, "planes: set %d needs finite strength > 0, width_scale > 0, shift", j);
        }
    }
    // mosaic
    if (m->kind < 0 || m->kind > 5) return fail(MRT_EINVAL, "mosaic: unknown kind");
    if (!(m->fwhm >= 0.0) || !std::isfinite(m->fwhm)) return fail(MRT_EINVAL, "mosaic: fwhm must be >= 0");
    if (!(m->eta >= 0.0 && m->eta <= 1.0)) return fail(MRT_EINVAL, "mosaic: eta must lie in [0, 1]");
    // rocking curve
    switch (r->kind) {
    case MRT_IRC_GAUSSIAN: case MRT_IRC_LORENTZIAN: case MRT_IRC_BOX:
        if (!(r->fwhm > 0.0)) return fail(MRT_EINVAL, "rocking curve: fwhm must be > 0");
        if (!(r->peak >= 0.0 && r->peak <= 1.0)) return fail(MRT_EINVAL, "rocking curve: peak must lie in [0, 1]");
        break;
    case MRT_IRC_PSEUDO_VOIGT:
        if (!(r->fwhm_g >= 0.0) || !(r->fwhm_l >= 0.0) || !(r->fwhm_g + r->fwhm_l > 0.0))
            return fail(MRT_EINVAL, "rocking curve: need fwhm_g, fwhm_l >= 0, not both 0");
        if (!(r->peak >= 0.0 && r->peak <= 1.0)) return fail(MRT_EINVAL, "rocking curve: peak must lie in [0, 1]");
        break;
    case MRT_IRC_TABLE:
        if (r->n_table < 2 || !r->table) return fail(MRT_EINVAL, "rocking curve: table needs n_table >= 2");
        if (!(r->x_max > r->x_min)) return fail(MRT_EINVAL, "rocking curve: need x_max > x_min");
        for (int i = 0; i < r->n_table; ++i)
            if (!(r->table[i] >= 0.0 && r->table[i] <= 1.0))
                return fail(MRT_EINVAL, "rocking curve: table values must lie in [0, 1]");
        break;
    default:
        return fail(MRT_EINVAL, "rocking curve: unknown kind");
    }
    if (!std::isfinite(r->shift)) return fail(MRT_EINVAL, "rocking curve: bad shift");
    if (r->n_dep < 0 || r->n_dep > kMaxQeNodes)
        return fail(MRT_EINVAL, "rocking curve: n_dep must lie in [0, %d]", kMaxQeNodes);
    if (r->n_dep > 0) {
        if (!r->dep_kev || !r->dep_shift || !r->dep_scale)
            return fail(MRT_EINVAL, "rocking curve: energy-dependence table pointers are NULL");
        for (int i = 0; i < r->n_dep; ++i) {
            if (!std::isfinite(r->dep_kev[i]) || !std::isfinite(r->dep_shift[i]) ||
                !(r->dep_scale[i] > 0.0 && std::isfinite(r->dep_scale[i])))
                return fail(MRT_EINVAL, "rocking curve: energy dependence needs finite shifts and scales > 0");
            if (i && !(r->dep_kev[i] > r->dep_kev[i - 1]))
                return fail(MRT_EINVAL, "rocking curve: energy-dependence energies must increase strictly");
        }
        if (c->planes)
            return fail(MRT_EINVAL, "an energy-dependent rocking curve takes no further reflecting planes");
    }
    {
        const size_t lut = r->kind == MRT_IRC_TABLE ? (size_t)r->n_table : 0;
        const size_t cdf = s->spectrum == MRT_SPECTRUM_TABLE ? (size_t)s->n_bins + 1 : 0;
        const size_t qe = d->n_qe > 0 ? 2 * (size_t)d->n_qe : 0;
        const size_t dep = r->n_dep > 0 ? 3 * (size_t)r->n_dep : 0;
        if ((lut + cdf + qe + dep) * sizeof(double) > (size_t)kMaxTableBytes)
            return fail(MRT_EINVAL, "rocking-curve table, spectrum bins and QE table exceed %d bytes",
                        kMaxTableBytes);
    }
    // detector
    if (!finite3(d->centre) || !unit(d->normal) || !unit(d->u) || !unit(d->v) ||
        !ortho(d->normal, d->u) || !ortho(d->normal, d->v) || !ortho(d->u, d->v))
        return fail(MRT_EINVAL, "detector: normal, u, v must be orthonormal unit vectors");
    if (d->nx < 1 || d->ny < 1 || (int64_t)d->nx * (int64_t)d->ny >= (int64_t(1) << 31))
        return fail(MRT_EINVAL, "detector: need nx, ny >= 1 and nx * ny < 2^31");
    if (!(d->pitch > 0.0)) return fail(MRT_EINVAL, "detector: pitch must be > 0");
    if (d->n_qe < 0 || d->n_qe > kMaxQeNodes)
        return fail(MRT_EINVAL, "detector: n_qe must lie in [0, %d]", kMaxQeNodes);
    if (d->n_qe > 0) {
        if (!d->qe_kev || !d->qe) return fail(MRT_EINVAL, "detector: QE table pointers are NULL");
        for (int i = 0; i < d->n_qe; ++i) {
            if (!std::isfinite(d->qe_kev[i]) || !(d->qe[i] >= 0.0 && d->qe[i] <= 1.0))
                return fail(MRT_EINVAL, "detector: QE values must lie in [0, 1] at finite energies");
            if (i && !(d->qe_kev[i] > d->qe_kev[i - 1]))
                return fail(MRT_EINVAL, "detector: QE energies must increase strictly");
        }
    }
    return MRT_OK;
}

static void pvoigt(double g, double l, double *fwhm, double *eta) {
    // total width and Lorentzian fraction of the pseudo-Voigt (sec. 2.2.1)
    const double f5 = std::pow(g, 5) + 2.69269 * std::pow(g, 4) * l + 2.42843 * std::pow(g, 3) * l * l +
                      4.47163 * g * g * std::pow(l, 3) + 0.07842 * g * std::pow(l, 4) + std::pow(l, 5);
    const double f = std::pow(f5, 0.2);
    const double q = l / f;
    *fwhm = f;
    *eta = 1.36603 * q - 0.47719 * q * q + 0.11116 * q * q * q;
}

// Fill the kernel parameters; `tables` receives the rocking-curve table
// followed by the spectrum CDF (uploaded by the caller).
// int r(x) dx of a rocking curve: closed forms, and the trapezoid rule for
// the table (exact for its linear interpolation).
static double irc_integral(const mrt_rocking_curve *r) {
    switch (r->kind) {
    case MRT_IRC_GAUSSIAN:
        return r->peak * r->fwhm * std::sqrt(kPi / (4.0 * std::log(2.0)));
    case MRT_IRC_PSEUDO_VOIGT: {
        // r = peak R(x) / R(0) with R of unit area (Eqs. Gaussian, Lorentz)
        double w, eta;
        pvoigt(r->fwhm_g, r->fwhm_l, &w, &eta);
        const double g0 = std::sqrt(4.0 * std::log(2.0) / (kPi * w * w)), l0 = 2.0 / (kPi * w);
        return r->peak / (eta * l0 + (1.0 - eta) * g0);
    }
    case MRT_IRC_LORENTZIAN:
        return r->peak * kPi * r->fwhm / 2.0;
    case MRT_IRC_BOX:
        return r->peak * r->fwhm;
    default: {
        double sum = 0.0;
        for (int j = 0; j + 1 < r->n_table; ++j) sum += (r->table[j] + r->table[j + 1]) / 2.0;
        return sum * (r->x_max - r->x_min) / (double)(r->n_table - 1);
    }
    }
}

// Step of the sampler's Delta proposals: the curve's full width at half
// maximum (for the table, the span of its nodes at or above half its maximum).
static double irc_width(const mrt_rocking_curve *r) {
    switch (r->kind) {
    case MRT_IRC_PSEUDO_VOIGT: {
        double w, eta;
        pvoigt(r->fwhm_g, r->fwhm_l, &w, &eta);
        return w;
    }
    case MRT_IRC_TABLE: {
        double mx = 0.0;
        for (int j = 0; j < r->n_table; ++j) mx = std::max(mx, r->table[j]);
        int cnt = 0;
        for (int j = 0; j < r->n_table; ++j) cnt += r->table[j] >= mx / 2.0;
        return (double)cnt * (r->x_max - r->x_min) / (double)(r->n_table - 1);
    }
    default:
        return r->fwhm;
    }
}

void build_mwg_params(const mrt_crystal *c, const mrt_mosaic *m, const mrt_rocking_curve *r,
                      int burn_in, int psi_nodes, int batch, bool irc_off, TraceParams &P,
                      std::vector<double> &psi) {
    P.burn_in = burn_in;
    P.irc_off = irc_off ? 1 : 0;
    P.psi_nodes = psi_nodes;
    P.mwg_batch = batch;
    P.q = irc_integral(r) / c->mfp;
    P.w_delta = irc_width(r);
    // sphere densities of the mosaic distributions per steradian (sec. 2.2.2)
    const double gamma = m->fwhm;
    const double sv = gamma / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    P.vmf_kappa = 1.0 / (sv * sv);
    P.vmf_norm = P.vmf_kappa / (2.0 * kPi * -std::expm1(-2.0 * P.vmf_kappa));
    const double g = gamma / 2.0;
    P.cau_g2 = g * g;
    P.cau_norm = g / (2.0 * kPi);
    P.wl_g2 = g * g;
    P.wl_norm = 1.0 / (kPi * std::log((g * g + 4.0) / (g * g)));
    const double sh = std::sinh(gamma / 4.0);
    P.swl_a = 2.0 * sh * sh;
    P.swl_norm = P.swl_a * (P.swl_a + 2.0) / (4.0 * kPi);
    P.gau_inv2s2 = 1.0 / (2.0 * sv * sv);
    P.gau_norm = 1.0 / (2.0 * kPi * sv * sv);
    // nodes psi_j = pi (j / M)^3, dense near psi = 0: (sin^2(psi_j / 2),
    // w_j) with the trapezoid weight w_j = (psi_{j+1} - psi_{j-1}) / 2 (the
    // missing neighbour of an end node taken as the node itself)
    auto node = [psi_nodes](int j) {
        const double t = (double)j / (double)psi_nodes;
        return kPi * t * t * t;
    };
    std::vector<double> w(psi_nodes + 1);
    for (int j = 0; j <= psi_nodes; ++j) {
        const double lo = j > 0 ? node(j) - node(j - 1) : 0.0;
        const double hi = j < psi_nodes ? node(j + 1) - node(j) : 0.0;
        w[j] = (lo + hi) / 2.0;
        const double b = std::sin(node(j) / 2.0);
        psi.push_back(b * b);
        psi.push_back(w[j]);
    }
    // then w_j cos(2 psi_j), j = 0..M, for the polarised cross-section
    for (int j = 0; j <= psi_nodes; ++j) psi.push_back(w[j] * std::cos(2.0 * node(j)));
}

bool uses_ext(const mrt_source *s, const mrt_crystal *c, const mrt_rocking_curve *r) {
    return r->n_dep > 0 || c->planes || s->polarisations;
}

void build_params(const mrt_source *s, const mrt_crystal *c, const mrt_mosaic *m,
                  const mrt_rocking_curve *r, const mrt_detector *d, TraceParams &P,
                  std::vector<double> &tables) {
    std::memset(&P, 0, sizeof P);
    // Crystal-local frame: origin O and rows of the rotation `rot` (the
    // local axes in global coordinates).  FLAT: x along e1, y along
    // e2 = normal x e1, z along the normal.  CYLINDER: z along the axis,
    // x along ref_dir (azimuth 0), y along axis x ref_dir.  In it the flat
    // crystal's frame and the cylinder's axis are the coordinate axes, which
    // the kernels use as constants.
    double O[3], X[3], Y[3], Z[3];
    if (c->geometry == MRT_GEOMETRY_FLAT) {
        for (int i = 0; i < 3; ++i) { O[i] = c->centre[i]; X[i] = c->e1[i]; Z[i] = c->normal[i]; }
        cross3(c->normal, c->e1, Y);
    } else {
        for (int i = 0; i < 3; ++i) {
            O[i] = c->axis_pt[i] + c->z_c * c->axis_dir[i];
            X[i] = c->ref_dir[i];
            Z[i] = c->axis_dir[i];
        }
        cross3(c->axis_dir, c->ref_dir, Y);
    }
    for (int i = 0; i < 3; ++i) {
        P.origin[i] = O[i];
        P.rot[0][i] = X[i];
        P.rot[1][i] = Y[i];
        P.rot[2][i] = Z[i];
    }
    // local coordinates of a global direction / position
    auto dir = [&](const double *g, double *l) {
        for (int r = 0; r < 3; ++r) l[r] = P.rot[r][0] * g[0] + P.rot[r][1] * g[1] + P.rot[r][2] * g[2];
    };
    auto pos = [&](const double *g, double *l) {
        const double d[3] = {g[0] - O[0], g[1] - O[1], g[2] - O[2]};
        dir(d, l);
    };

    // source
    pos(s->origin, P.so);
    dir(s->axis, P.sa);
    dir(s->b1, P.sb1);
    {
        double b2[3];
        cross3(s->axis, s->b1, b2);
        dir(b2, P.sb2);
    }
    P.spot_kind = s->spot_kind;
    if (s->spot_kind != MRT_SPOT_POINT) {
        dir(s->spot_u, P.spot_u);
        dir(s->spot_v, P.spot_v);
        P.spot_sigma[0] = s->spot_sigma[0];
        P.spot_sigma[1] = s->spot_kind == MRT_SPOT_GAUSSIAN ? s->spot_sigma[1] : 0.0;
    }
    P.user_o = s->origins;
    P.user_k = s->directions;
    P.user_e = s->energies;
    P.user_p = s->polarisations;
    const double sh = std::sin(s->half_angle / 2.0);
    P.vmax = 2.0 * sh * sh;
    P.spectrum = s->spectrum;
    P.e_min = s->e_min;
    P.e_span = s->e_max - s->e_min;
    if (s->spectrum == MRT_SPECTRUM_LINES) {
        P.n_lines = s->n_lines;
        double total = 0.0;
        for (int j = 0; j < s->n_lines; ++j) total += s->line_w[j];
        total += s->background_w;
        double acc = 0.0;
        for (int j = 0; j < s->n_lines; ++j) {
            acc += s->line_w[j];
            P.line_cum[j] = acc / total;
            P.line_e[j] = s->line_e[j];
            P.line_sig[j] = s->line_sigma[j];
        }
    }

    // crystal
    P.geometry = c->geometry;
    P.max_refl = c->max_refl;
    P.hl = c->length / 2.0;
    P.hw = c->width / 2.0;
    P.T = c->thickness;
    if (c->geometry != MRT_GEOMETRY_FLAT) {
        // outward normals of the two azimuth edges, in the local x-y plane
        const double half = c->width / (2.0 * c->radius);
        const double pp = c->phi_c + half, pm = c->phi_c - half;
        P.op[0] = -std::sin(pp);
        P.op[1] = std::cos(pp);
        P.om[0] = std::sin(pm);
        P.om[1] = -std::cos(pm);
        P.R = c->radius;
        P.R2 = c->radius * c->radius;
        const double ro = c->radius + c->thickness;
        P.Ro2 = ro * ro;
    }
    double rmax = r->peak;
    if (r->kind == MRT_IRC_TABLE) {
        rmax = 0.0;
        for (int i = 0; i < r->n_table; ++i) rmax = std::max(rmax, r->table[i]);
    }
    // reflecting planes: set 0 is the main set (the curve as given)
    P.n_planes = 1;
    P.plane_2d[0] = c->two_d;
    P.plane_a[0] = 1.0;
    P.plane_scale[0] = 1.0;
    P.plane_shift[0] = r->shift;
    P.hbar = 1.0;
    if (const mrt_planes *pl = c->planes) {
        P.has_planes = 1;
        P.hbar = pl->hbar_ratio;
        for (int j = 0; j < pl->n_extra; ++j) {
            P.plane_2d[1 + j] = pl->two_d[j];
            P.plane_a[1 + j] = pl->strength[j];
            P.plane_scale[1 + j] = pl->width_scale[j];
            P.plane_shift[1 + j] = pl->shift[j];
        }
        P.n_planes = 1 + pl->n_extra;
    }
    double sum_a = 0.0;
    for (int j = 0; j < P.n_planes; ++j) {
        sum_a += P.plane_a[j];
        P.plane_inv_scale[j] = 1.0 / P.plane_scale[j];
        P.plane_ratio[j] = c->two_d / P.plane_2d[j];
    }
    P.plane_tot = sum_a * std::max(1.0, P.hbar);
    // majorant crystallite-encounter rate: every set and side at its peak
    const double lambda_c = rmax * P.plane_tot / c->mfp;
    const double mu_tot = c->mu0 + lambda_c;
    P.mu0 = c->mu0;
    P.inv_mu0 = 1.0 / c->mu0;
    P.inv_mu_tot = 1.0 / mu_tot;
    P.p_a = mu_tot > 0.0 ? c->mu0 / mu_tot : 1.0;
    P.inv_1mpa = 1.0 / (1.0 - P.p_a);
    P.two_d = c->two_d;

    // mosaic
    P.mdf = m->kind;
    P.fwhm = m->fwhm;
    P.m_eta = m->eta;
    P.inv_eta = m->eta > 0.0 ? 1.0 / m->eta : 0.0;
    P.inv_1meta = m->eta < 1.0 ? 1.0 / (1.0 - m->eta) : 0.0;
    if (m->fwhm > 0.0) {
        const double sv = m->fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
        P.vmf_s2 = sv * sv;
        P.vmf_floor = std::exp(-2.0 / P.vmf_s2);
        P.gau_2s2 = 2.0 * sv * sv;   // tan^2(theta) = 2 s^2 (-ln u) for the Gaussian tilt
        const double g = m->fwhm / 2.0;
        P.lor_g = g;
        P.wl_half_g2 = g * g / 2.0;
        P.wl_z = std::log((g * g + 4.0) / (g * g));
        const double a = m->fwhm / 2.0;
        const double s2 = std::sinh(a / 2.0);
        P.swl_k = 2.0 * s2 * s2 * 2.0;
        P.swl_d = std::cosh(a) + 1.0;
    }

    // rocking curve
    P.irc = r->kind;
    P.shift = r->shift;
    const double ln2 = std::log(2.0);
    switch (r->kind) {
    case MRT_IRC_GAUSSIAN:
        P.g_k = 4.0 * ln2 / (r->fwhm * r->fwhm);
        break;
    case MRT_IRC_PSEUDO_VOIGT: {
        // r(x) / R(0) = A h^2 / (h^2 + x^2) + B exp(-g_k x^2), with
        // A = eta L(0) / R(0), B = (1 - eta) G(0) / R(0) (Eqs. Gaussian, Lorentz)
        double w, eta;
        pvoigt(r->fwhm_g, r->fwhm_l, &w, &eta);
        P.g_k = 4.0 * ln2 / (w * w);
        const double g0 = std::sqrt(4.0 * ln2 / (kPi * w * w));
        const double l0 = 2.0 / (kPi * w);
        const double r0 = eta * l0 + (1.0 - eta) * g0;
        P.pv_a = eta * l0 / r0;
        P.pv_b = (1.0 - eta) * g0 / r0;
        P.pv_h2 = (w / 2.0) * (w / 2.0);
        break;
    }
    case MRT_IRC_LORENTZIAN:
        P.lor_h2 = (r->fwhm / 2.0) * (r->fwhm / 2.0);
        break;
    case MRT_IRC_BOX:
        P.box_half = r->fwhm / 2.0;
        break;
    case MRT_IRC_TABLE:
        P.lut_n = r->n_table;
        P.lut_x0 = r->x_min;
        P.lut_x1 = r->x_max;
        P.lut_scale = (double)(r->n_table - 1) / (r->x_max - r->x_min);
        P.lut_inv_max = rmax > 0.0 ? 1.0 / rmax : 0.0;
        tables.insert(tables.end(), r->table, r->table + r->n_table);
        break;
    }
    P.g_k_log2e = P.g_k / ln2;
    if (s->spectrum == MRT_SPECTRUM_TABLE) {
        P.n_bins = s->n_bins;
        double total = 0.0;
        for (int b = 0; b < s->n_bins; ++b) total += s->bin_w[b];
        double acc = 0.0;
        for (int b = 0; b <= s->n_bins; ++b) {
            tables.push_back(b == s->n_bins ? 1.0 : acc / total);
            if (b < s->n_bins) acc += s->bin_w[b];
        }
    }

    // detector
    pos(d->centre, P.dP);
    dir(d->normal, P.dn);
    dir(d->u, P.du);
    dir(d->v, P.dv);
    P.nx = d->nx;
    P.ny = d->ny;
    P.pitch = d->pitch;
    P.half_nx = (double)d->nx / 2.0;
    P.half_ny = (double)d->ny / 2.0;
    P.dep_n = r->n_dep;
    P.dep_at = (int32_t)tables.size();
    if (r->n_dep > 0) {
        tables.insert(tables.end(), r->dep_kev, r->dep_kev + r->n_dep);
        tables.insert(tables.end(), r->dep_shift, r->dep_shift + r->n_dep);
        tables.insert(tables.end(), r->dep_scale, r->dep_scale + r->n_dep);
    }
    P.qe_n = d->n_qe;
    P.qe_at = (int32_t)tables.size();
    if (d->n_qe > 0) {
        tables.insert(tables.end(), d->qe_kev, d->qe_kev + d->n_qe);
        tables.insert(tables.end(), d->qe, d->qe + d->n_qe);
    }
    // The table curve's envelope for the FP32 acceptance filter: the minimum
    // and maximum node of each bucket of 2^env_shift nodes, as r / R_max
    // rounded down and up to float, packed as a float pair in one table
    // word.  The filter's interval of x (its 2e-6 rad band on either side,
    // widened by the smallest width scale of the curve) covers at most two
    // buckets when a bucket holds the interval's nodes plus two.
    P.env_at = (int32_t)tables.size();
    P.env_shift = 0;
    if (r->kind == MRT_IRC_TABLE) {
        double min_scale = 1.0;
        for (int i = 0; i < r->n_dep; ++i) min_scale = std::min(min_scale, r->dep_scale[i]);
        for (int j = 1; j < P.n_planes; ++j) min_scale = std::min(min_scale, P.plane_scale[j]);
        const double width = 2.0 * 2e-6 / min_scale * P.lut_scale + 2.0;
        int sh = 3;
        while (sh < 12 && (double)(1 << sh) < width) ++sh;
        P.env_shift = sh;
        const int bn = 1 << sh;
        for (int b = 0; b * bn < r->n_table; ++b) {
            double lo = r->table[b * bn], hi = lo;
            for (int i = b * bn; i < std::min(r->n_table, (b + 1) * bn); ++i) {
                lo = std::min(lo, r->table[i]);
                hi = std::max(hi, r->table[i]);
            }
            float fl = (float)(lo * P.lut_inv_max), fh = (float)(hi * P.lut_inv_max);
            if ((double)fl > lo * P.lut_inv_max) fl = std::nextafter(fl, -1.0f);
            if ((double)fh < hi * P.lut_inv_max) fh = std::nextafter(fh, 2.0f);
            const float pair[2] = {fl, fh};
            double word;
            std::memcpy(&word, pair, sizeof word);
            tables.push_back(word);
        }
    }

    // FP32 copies for the FP32-mixed kernels (round to nearest)
#define MRT_F32_S(n) P.f32.n = (float)P.n;
#define MRT_F32_V(n) \
    for (int i = 0; i < 3; ++i) P.f32.n[i] = (float)P.n[i];
    MRT_F32_SCALARS(MRT_F32_S)
    MRT_F32_VECTORS(MRT_F32_V)
#undef MRT_F32_S
#undef MRT_F32_V
}

}  // namespace mrt
