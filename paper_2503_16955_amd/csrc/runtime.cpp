// Host runtime of the C-ABI: validation, launch parameters, table staging,
// counters and timing.  Every step of the transport itself runs in the
// trace kernels (trace_impl.h, instantiated in trace_f64_*.hip and
// trace_f32_*.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mosaicrt.h"
#include "trace_params.h"

namespace {

thread_local std::string g_last_error;

constexpr double kHC = 12.398419843320026;   // h c in keV Angstrom (SI 2019 exact)
constexpr double kPi = 3.1415926535897932384626433832795;

mrt_status fail(mrt_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

mrt_status hip_fail(hipError_t e, const char *what) {
    return fail(MRT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
void cross3(const double *a, const double *b, double *r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
bool unit(const double *v) { return std::fabs(std::sqrt(dot3(v, v)) - 1.0) <= 1e-12; }
bool ortho(const double *a, const double *b) { return std::fabs(dot3(a, b)) <= 1e-12; }
bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

mrt_status validate(const mrt_source *s, const mrt_crystal *c, const mrt_mosaic *m,
                    const mrt_rocking_curve *r, const mrt_detector *d) {
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
    // mosaic
    if (m->kind < 0 || m->kind > 4) return fail(MRT_EINVAL, "mosaic: unknown kind");
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
    {
        const size_t lut = r->kind == MRT_IRC_TABLE ? (size_t)r->n_table : 0;
        const size_t cdf = s->spectrum == MRT_SPECTRUM_TABLE ? (size_t)s->n_bins + 1 : 0;
        if ((lut + cdf) * sizeof(double) > (size_t)mrt::kMaxTableBytes)
            return fail(MRT_EINVAL, "rocking-curve table plus spectrum bins exceed %d bytes of LDS",
                        mrt::kMaxTableBytes);
    }
    // detector
    if (!finite3(d->centre) || !unit(d->normal) || !unit(d->u) || !unit(d->v) ||
        !ortho(d->normal, d->u) || !ortho(d->normal, d->v) || !ortho(d->u, d->v))
        return fail(MRT_EINVAL, "detector: normal, u, v must be orthonormal unit vectors");
    if (d->nx < 1 || d->ny < 1 || (int64_t)d->nx * (int64_t)d->ny >= (int64_t(1) << 31))
        return fail(MRT_EINVAL, "detector: need nx, ny >= 1 and nx * ny < 2^31");
    if (!(d->pitch > 0.0)) return fail(MRT_EINVAL, "detector: pitch must be > 0");
    return MRT_OK;
}

void pvoigt(double g, double l, double *fwhm, double *eta) {
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
void build_params(const mrt_source *s, const mrt_crystal *c, const mrt_mosaic *m,
                  const mrt_rocking_curve *r, const mrt_detector *d, mrt::TraceParams &P,
                  std::vector<double> &tables) {
    std::memset(&P, 0, sizeof P);
    // local origin
    double O[3];
    if (c->geometry == MRT_GEOMETRY_FLAT) {
        for (int i = 0; i < 3; ++i) O[i] = c->centre[i];
    } else {
        for (int i = 0; i < 3; ++i) O[i] = c->axis_pt[i] + c->z_c * c->axis_dir[i];
    }
    for (int i = 0; i < 3; ++i) P.origin[i] = O[i];

    // source
    for (int i = 0; i < 3; ++i) {
        P.so[i] = s->origin[i] - O[i];
        P.sa[i] = s->axis[i];
        P.sb1[i] = s->b1[i];
    }
    cross3(s->axis, s->b1, P.sb2);
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
    if (c->geometry == MRT_GEOMETRY_FLAT) {
        for (int i = 0; i < 3; ++i) { P.N[i] = c->normal[i]; P.e1[i] = c->e1[i]; }
        cross3(c->normal, c->e1, P.e2);
    } else {
        double b2[3];
        cross3(c->axis_dir, c->ref_dir, b2);
        const double half = c->width / (2.0 * c->radius);
        const double pp = c->phi_c + half, pm = c->phi_c - half;
        for (int i = 0; i < 3; ++i) {
            P.ax[i] = c->axis_dir[i];
            P.op[i] = -std::sin(pp) * c->ref_dir[i] + std::cos(pp) * b2[i];
            P.om[i] = std::sin(pm) * c->ref_dir[i] - std::cos(pm) * b2[i];
        }
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
    const double lambda_c = rmax / c->mfp;   // majorant crystallite-encounter rate
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
    for (int i = 0; i < 3; ++i) {
        P.dP[i] = d->centre[i] - O[i];
        P.dn[i] = d->normal[i];
        P.du[i] = d->u[i];
        P.dv[i] = d->v[i];
    }
    P.nx = d->nx;
    P.ny = d->ny;
    P.pitch = d->pitch;
    P.half_nx = (double)d->nx / 2.0;
    P.half_ny = (double)d->ny / 2.0;
}

struct DeviceCache {
    int device = -1;
    int cus = 0;
};
thread_local DeviceCache g_dev;

mrt_status current_device(int *dev, int *cus) {
    int d = 0;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (g_dev.device != d) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, d);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        g_dev.device = d;
        g_dev.cus = prop.multiProcessorCount;
    }
    *dev = d;
    *cus = g_dev.cus;
    return MRT_OK;
}

}  // namespace

extern "C" {

const char *mrt_last_error(void) { return g_last_error.c_str(); }
int mrt_version(void) { return MRT_VERSION; }

mrt_status mrt_get_device_info(mrt_device_info *info) {
    if (!info) return fail(MRT_EINVAL, "null info");
    std::memset(info, 0, sizeof *info);
    int d = 0;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, d);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    info->device = d;
    info->compute_units = prop.multiProcessorCount;
    info->clock_khz = prop.clockRate;
    info->lds_bytes_per_block = (int32_t)prop.sharedMemPerBlock;
    std::snprintf(info->name, sizeof info->name, "%s", prop.name);
    std::snprintf(info->arch, sizeof info->arch, "%s", prop.gcnArchName);
    return MRT_OK;
}

mrt_status mrt_trace(const mrt_source *source, const mrt_crystal *crystal,
                     const mrt_mosaic *mosaic, const mrt_rocking_curve *rocking_curve,
                     const mrt_detector *detector, uint64_t first_ray_id, uint64_t n_rays,
                     uint64_t seed, const mrt_options *options, uint32_t *d_counts,
                     uint64_t *d_energy_mev, mrt_hit_record *d_records,
                     uint64_t records_capacity, mrt_counters *h_counters, void *hip_stream) {
    g_last_error.clear();
    mrt_status st = validate(source, crystal, mosaic, rocking_curve, detector);
    if (st != MRT_OK) return st;
    mrt_options opt{};
    if (options) opt = *options;
    if (opt.precision != MRT_FP64 && opt.precision != MRT_FP32_MIXED)
        return fail(MRT_EINVAL, "options: unknown precision");
    if (opt.records_mode < 0 || opt.records_mode > 2) return fail(MRT_EINVAL, "options: unknown records mode");
    if (n_rays == 0) return fail(MRT_EINVAL, "n_rays must be > 0");
    if (first_ray_id + n_rays < first_ray_id) return fail(MRT_EINVAL, "first_ray_id + n_rays overflows");
    if (!d_counts) return fail(MRT_EINVAL, "d_counts is required");
    if (opt.records_mode != MRT_RECORDS_NONE && !d_records)
        return fail(MRT_EINVAL, "records requested but d_records is NULL");
    if (opt.records_mode == MRT_RECORDS_ALL && records_capacity < n_rays)
        return fail(MRT_ECAPACITY, "records_capacity %llu < n_rays %llu",
                    (unsigned long long)records_capacity, (unsigned long long)n_rays);
    if (opt.block_threads < 0 || opt.block_threads > 256 || opt.block_threads % 64 != 0)
        return fail(MRT_EINVAL, "options: block_threads must be a multiple of 64 up to 256");
    if (opt.grid_blocks < 0) return fail(MRT_EINVAL, "options: grid_blocks must be >= 0");
    if (opt.refill_idle < 0 || opt.refill_idle > 64)
        return fail(MRT_EINVAL, "options: refill_idle must lie in [0, 64]");

    int dev = 0, cus = 0;
    if ((st = current_device(&dev, &cus)) != MRT_OK) return st;
    hipStream_t stream = (hipStream_t)hip_stream;

    mrt::TraceParams P;
    std::vector<double> tables;
    build_params(source, crystal, mosaic, rocking_curve, detector, P, tables);
    P.first = first_ray_id;
    P.n = n_rays;
    P.seed = seed;
    P.key0 = (uint32_t)seed;
    P.key1 = (uint32_t)(seed >> 32);
    P.max_events = opt.max_events ? opt.max_events : (1u << 20);
    P.records_mode = opt.records_mode;
    P.rec_cap = records_capacity;
    P.counts = d_counts;
    P.energy = (unsigned long long *)d_energy_mev;
    P.records = d_records;

    // library scratch: counters, chunk cursor, tables
    const size_t n_ctr = mrt::kNumCounters + 1;
    const size_t bytes = n_ctr * sizeof(unsigned long long) + tables.size() * sizeof(double);
    void *scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, bytes, stream);
    if (e != hipSuccess) return fail(MRT_ENOMEM, "hipMallocAsync(%zu): %s", bytes, hipGetErrorString(e));
    P.dev_counters = (unsigned long long *)scratch;
    P.chunk_counter = P.dev_counters + mrt::kNumCounters;
    double *dtab = (double *)(P.dev_counters + n_ctr);
    P.lut = rocking_curve->kind == MRT_IRC_TABLE ? dtab : nullptr;
    P.bin_cdf = source->spectrum == MRT_SPECTRUM_TABLE
                    ? dtab + (rocking_curve->kind == MRT_IRC_TABLE ? rocking_curve->n_table : 0)
                    : nullptr;

    auto release = [&](mrt_status s) {
        (void)hipFreeAsync(scratch, stream);
        return s;
    };
    if (!tables.empty()) {
        e = hipMemcpyAsync(dtab, tables.data(), tables.size() * sizeof(double), hipMemcpyHostToDevice,
                           stream);
        if (e != hipSuccess) return release(hip_fail(e, "hipMemcpyAsync(tables)"));
        // the host vector dies with this call: wait for the copy
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return release(hip_fail(e, "hipStreamSynchronize"));
    }
    if (mrt::launch_zero(P.dev_counters, 2 * n_ctr, stream) != 0)
        return release(fail(MRT_EDEVICE, "zero kernel launch failed"));
    if (!opt.accumulate) {
        const size_t px = (size_t)detector->nx * (size_t)detector->ny;
        if (mrt::launch_zero(d_counts, px, stream) != 0)
            return release(fail(MRT_EDEVICE, "zero kernel launch failed"));
        if (d_energy_mev && mrt::launch_zero(d_energy_mev, 2 * px, stream) != 0)
            return release(fail(MRT_EDEVICE, "zero kernel launch failed"));
    }

    const bool rec = opt.records_mode != MRT_RECORDS_NONE;
    const void *kernel = mrt::trace_kernel_ptr(opt.precision, crystal->geometry, mosaic->kind,
                                               rocking_curve->kind, rec);
    if (!kernel) return release(fail(MRT_EINVAL, "no kernel for this combination of kinds"));
    const int block = opt.block_threads ? opt.block_threads : 256;
    const size_t lds = tables.size() * sizeof(double);
    int grid = opt.grid_blocks;
    if (grid == 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        grid = cus * per_cu;
    }
    P.refill_idle = opt.refill_idle > 0 ? (uint32_t)opt.refill_idle : 16u;
    // chunk size: enough chunks for every wave to claim several
    const uint64_t waves = (uint64_t)grid * (uint64_t)(block / 64);
    uint64_t chunk = n_rays / (waves * 8);
    chunk = std::max<uint64_t>(64, std::min<uint64_t>(2048, chunk));
    P.chunk = (uint32_t)chunk;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (h_counters) {
        if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess ||
            hipEventRecord(ev0, stream) != hipSuccess)
            return release(hip_fail(hipGetLastError(), "hipEvent setup"));
    }
    void *args[] = {&P};
    if (hipLaunchKernel(kernel, dim3((unsigned)grid), dim3((unsigned)block), args, lds, stream) !=
        hipSuccess) {
        if (ev0) { (void)hipEventDestroy(ev0); (void)hipEventDestroy(ev1); }
        return release(fail(MRT_EDEVICE, "trace kernel launch failed: %s",
                            hipGetErrorString(hipGetLastError())));
    }
    mrt_status out = MRT_OK;
    if (h_counters) {
        (void)hipEventRecord(ev1, stream);
        unsigned long long host[mrt::kNumCounters];
        e = hipMemcpyAsync(host, P.dev_counters, sizeof host, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            (void)hipEventDestroy(ev0);
            (void)hipEventDestroy(ev1);
            return release(hip_fail(e, "counter readback"));
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, ev0, ev1);
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
        h_counters->emitted = n_rays;
        h_counters->missed = host[mrt::kCMissed];
        h_counters->absorbed = host[mrt::kCAbsorbed];
        h_counters->exit_reflected = host[mrt::kCExitReflected];
        h_counters->exit_transmitted = host[mrt::kCExitTransmitted];
        h_counters->truncated = host[mrt::kCTruncated];
        h_counters->detected = host[mrt::kCDetected];
        h_counters->events = host[mrt::kCEvents];
        h_counters->reflections = host[mrt::kCReflections];
        h_counters->refined = host[mrt::kCRefined];
        const unsigned long long nrec = host[mrt::kCRecords];
        h_counters->records = opt.records_mode == MRT_RECORDS_ALL ? n_rays
                              : std::min<unsigned long long>(nrec, records_capacity);
        h_counters->kernel_ms = ms;
        if (opt.records_mode == MRT_RECORDS_DETECTED && nrec > records_capacity)
            out = fail(MRT_ECAPACITY, "%llu detected records, capacity %llu", nrec,
                       (unsigned long long)records_capacity);
    }
    release(MRT_OK);
    return out;
}

}  // extern "C"
