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
#include "params.h"
#include "trace_params.h"

namespace mrt {

namespace {
thread_local std::string g_last_error;
}  // namespace

mrt_status fail(mrt_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

const char *last_error() { return g_last_error.c_str(); }
void clear_error() { g_last_error.clear(); }

}  // namespace mrt

namespace {

using mrt::fail;

mrt_status hip_fail(hipError_t e, const char *what) {
    return fail(MRT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
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

const char *mrt_last_error(void) { return mrt::last_error(); }
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

mrt_status mrt_calibration_map(const uint32_t *d_counts, const uint64_t *d_energy_mev,
                               uint64_t n_pixels, double *d_map_kev, void *hip_stream) {
    mrt::clear_error();
    if (!d_counts || !d_energy_mev || !d_map_kev)
        return fail(MRT_EINVAL, "calibration map: NULL image or map pointer");
    if (mrt::launch_calibration_map(d_counts, d_energy_mev, (size_t)n_pixels, d_map_kev, hip_stream) != 0)
        return fail(MRT_EDEVICE, "calibration map launch failed: %s", hipGetErrorString(hipGetLastError()));
    return MRT_OK;
}

mrt_status mrt_trace(const mrt_source *source, const mrt_crystal *crystal,
                     const mrt_mosaic *mosaic, const mrt_rocking_curve *rocking_curve,
                     const mrt_detector *detector, uint64_t first_ray_id, uint64_t n_rays,
                     uint64_t seed, const mrt_options *options, uint32_t *d_counts,
                     uint64_t *d_energy_mev, mrt_hit_record *d_records,
                     uint64_t records_capacity, mrt_counters *h_counters, void *hip_stream) {
    mrt::clear_error();
    mrt_status st = mrt::validate(source, crystal, mosaic, rocking_curve, detector, fail);
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
    if (opt.exact_decisions != 0 && opt.exact_decisions != 1)
        return fail(MRT_EINVAL, "options: exact_decisions must be 0 or 1");
    const bool mwg = opt.event_model == MRT_MODEL_MWG;
    if (opt.event_model != MRT_MODEL_STEPPING && !mwg) return fail(MRT_EINVAL, "options: unknown event model");
    if (!mwg && opt.mwg_irc_off != 0) return fail(MRT_EINVAL, "options: mwg_irc_off needs the MWG event model");
    if (mwg) {
        if (opt.precision != MRT_FP64) return fail(MRT_EINVAL, "options: the MWG event model runs in FP64");
        if (!(mosaic->fwhm > 0.0)) return fail(MRT_EINVAL, "the MWG event model needs a mosaic fwhm > 0");
        if (opt.mwg_burn_in < MRT_MWG_NO_BURN_IN) return fail(MRT_EINVAL, "options: mwg_burn_in must be >= -1");
        if (opt.psi_nodes < 0 || opt.psi_nodes > mrt::kMaxPsiNodes)
            return fail(MRT_EINVAL, "options: psi_nodes must lie in [0, %d]", mrt::kMaxPsiNodes);
        if (opt.mwg_batch < 0 || opt.mwg_batch > 64) return fail(MRT_EINVAL, "options: mwg_batch must lie in [0, 64]");
        if (opt.max_events > 0x7fffffffu) return fail(MRT_EINVAL, "options: the MWG event model needs max_events < 2^31");
        if (opt.mwg_irc_off != 0 && opt.mwg_irc_off != 1) return fail(MRT_EINVAL, "options: mwg_irc_off must be 0 or 1");
        if (opt.exact_decisions) return fail(MRT_EINVAL, "options: exact_decisions applies to the stepping model");
    }

    int dev = 0, cus = 0;
    if ((st = current_device(&dev, &cus)) != MRT_OK) return st;
    hipStream_t stream = (hipStream_t)hip_stream;

    mrt::TraceParams P;
    std::vector<double> tables;
    mrt::build_params(source, crystal, mosaic, rocking_curve, detector, P, tables);
    const size_t psi_at = tables.size();   // the psi table follows the other tables
    if (mwg) {
        const int burn = opt.mwg_burn_in == 0 ? 500 : (opt.mwg_burn_in < 0 ? 0 : opt.mwg_burn_in);
        mrt::build_mwg_params(crystal, mosaic, rocking_curve, burn, opt.psi_nodes ? opt.psi_nodes : 256,
                              opt.mwg_batch ? opt.mwg_batch : 32, opt.mwg_irc_off != 0, P, tables);
    }
    P.first = first_ray_id;
    P.n = n_rays;
    P.seed = seed;
    P.key0 = (uint32_t)seed;
    P.key1 = (uint32_t)(seed >> 32);
    P.max_events = opt.max_events ? opt.max_events : (1u << 20);
    P.records_mode = opt.records_mode;
    P.exact = opt.exact_decisions ? 1u : 0u;
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
    P.psi_tab = mwg ? dtab + psi_at : nullptr;
    P.psi_cos2 = mwg ? P.psi_tab + 2 * (P.psi_nodes + 1) : nullptr;
    P.qe = P.qe_n > 0 ? dtab + P.qe_at : nullptr;
    P.dep = P.dep_n > 0 ? dtab + P.dep_at : nullptr;

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
    const void *kernel = mwg ? mrt::mwg_kernel_ptr(crystal->geometry, rec, source->polarisations != nullptr,
                                                   crystal->planes != nullptr || rocking_curve->n_dep > 0)
                         : mrt::uses_ext(source, crystal, rocking_curve) || opt.exact_decisions
                             ? mrt::ext_kernel_ptr(opt.precision, rec)
                             : mrt::trace_kernel_ptr(opt.precision, crystal->geometry, mosaic->kind,
                                                     rocking_curve->kind, rec);
    if (!kernel) return release(fail(MRT_EINVAL, "no kernel for this combination of kinds"));
    const int block = opt.block_threads ? opt.block_threads : 256;
    const size_t lds = 0;   // the kernels read their tables from device memory
    int grid = opt.grid_blocks;
    if (grid == 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        grid = cus * per_cu;
    }
    P.refill_idle = opt.refill_idle > 0 ? (uint32_t)opt.refill_idle : 8u;
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
