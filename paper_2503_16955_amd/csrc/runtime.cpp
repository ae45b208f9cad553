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
#include <mutex>
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

// ---- a trace call, prepared on the host ---------------------------------
struct Launch {
    mrt::TraceParams P;
    std::vector<double> tables;   // rocking-curve table, spectrum CDF, QE, energy dependence, psi
    size_t psi_at = 0;            // the psi table's index in `tables`
    mrt_options opt{};
    bool mwg = false;
    const void *kernel = nullptr;
    int grid = 0, block = 0;
    int dev = 0;
    size_t pixels = 0;
    double *dtab = nullptr;       // device copy of `tables`
};

constexpr size_t kCounterWords = mrt::kNumCounters + 1;   // counters, then the chunk cursor

// Validation of every argument, the parameter block, the kernel and the
// launch shape.  Touches no device memory.
mrt_status prepare(const mrt_source *source, const mrt_crystal *crystal, const mrt_mosaic *mosaic,
                   const mrt_rocking_curve *rocking_curve, const mrt_detector *detector,
                   uint64_t first_ray_id, uint64_t n_rays, uint64_t seed,
                   const mrt_options *options, uint32_t *d_counts, uint64_t *d_energy_mev,
                   mrt_hit_record *d_records, uint64_t records_capacity, Launch &L) {
    mrt_status st = mrt::validate(source, crystal, mosaic, rocking_curve, detector, fail);
    if (st != MRT_OK) return st;
    mrt_options &opt = L.opt;
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
    const bool mwg = L.mwg = opt.event_model == MRT_MODEL_MWG;
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

    int cus = 0;
    if ((st = current_device(&L.dev, &cus)) != MRT_OK) return st;

    mrt::TraceParams &P = L.P;
    mrt::build_params(source, crystal, mosaic, rocking_curve, detector, P, L.tables);
    L.psi_at = L.tables.size();   // the psi table follows the other tables
    if (mwg) {
        const int burn = opt.mwg_burn_in == 0 ? 500 : (opt.mwg_burn_in < 0 ? 0 : opt.mwg_burn_in);
        mrt::build_mwg_params(crystal, mosaic, rocking_curve, burn, opt.psi_nodes ? opt.psi_nodes : 256,
                              opt.mwg_batch ? opt.mwg_batch : 32, opt.mwg_irc_off != 0, P, L.tables);
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
    L.pixels = (size_t)detector->nx * (size_t)detector->ny;

    const bool rec = opt.records_mode != MRT_RECORDS_NONE;
    const bool ext = !mwg && (mrt::uses_ext(source, crystal, rocking_curve) || opt.exact_decisions);
    L.kernel = mwg ? mrt::mwg_kernel_ptr(crystal->geometry, rec, source->polarisations != nullptr,
                                         crystal->planes != nullptr || rocking_curve->n_dep > 0)
               : ext ? mrt::ext_kernel_ptr(opt.precision, crystal->geometry, mosaic->kind,
                                         rocking_curve->kind, rec)
                   : mrt::trace_kernel_ptr(opt.precision, crystal->geometry, mosaic->kind,
                                           rocking_curve->kind, rec);
    if (!L.kernel) return fail(MRT_EINVAL, "no kernel for this combination of kinds");
    L.block = opt.block_threads ? opt.block_threads : 256;
    L.grid = opt.grid_blocks;
    if (L.grid == 0) {
        int per_cu = 0;
        // the kernels read their tables from device memory: no dynamic LDS
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, L.kernel, L.block, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        L.grid = cus * per_cu;
    }
    P.refill_idle = opt.refill_idle > 0 ? (uint32_t)opt.refill_idle
                                        : mrt::default_refill(mwg || ext, opt.precision == MRT_FP64);
    // chunk size: enough chunks for every wave to claim several
    const uint64_t waves = (uint64_t)L.grid * (uint64_t)(L.block / 64);
    uint64_t chunk = n_rays / (waves * 8);
    chunk = std::max<uint64_t>(64, std::min<uint64_t>(2048, chunk));
    P.chunk = (uint32_t)chunk;
    return MRT_OK;
}

// Device scratch of a call: counters and chunk cursor, then the tables.
size_t scratch_bytes(const Launch &L) {
    return kCounterWords * sizeof(unsigned long long) + L.tables.size() * sizeof(double);
}

// Point the parameter block at a scratch area of scratch_bytes(L) bytes.
void bind_scratch(Launch &L, void *scratch) {
    mrt::TraceParams &P = L.P;
    P.dev_counters = (unsigned long long *)scratch;
    P.chunk_counter = P.dev_counters + mrt::kNumCounters;
    double *dtab = L.dtab = (double *)(P.dev_counters + kCounterWords);
    P.lut = P.irc == MRT_IRC_TABLE ? dtab : nullptr;
    P.lut_env = P.irc == MRT_IRC_TABLE ? dtab + P.env_at : nullptr;
    P.bin_cdf = P.spectrum == MRT_SPECTRUM_TABLE ? dtab + (P.irc == MRT_IRC_TABLE ? P.lut_n : 0) : nullptr;
    P.psi_tab = L.mwg ? dtab + L.psi_at : nullptr;
    P.psi_cos2 = L.mwg ? P.psi_tab + 2 * (P.psi_nodes + 1) : nullptr;
    P.qe = P.qe_n > 0 ? dtab + P.qe_at : nullptr;
    P.dep = P.dep_n > 0 ? dtab + P.dep_at : nullptr;
}

// Clear the counters (and the images unless accumulating), launch the trace
// kernel and, with h_counters, wait for the stream and read the counters
// back (timed: also the kernel's duration between two HIP events).
mrt_status enqueue(Launch &L, hipStream_t stream, mrt_counters *h_counters, bool timed) {
    mrt::TraceParams &P = L.P;
    if (mrt::launch_zero(P.dev_counters, 2 * kCounterWords, stream) != 0)
        return fail(MRT_EDEVICE, "zero kernel launch failed");
    if (!L.opt.accumulate) {
        if (mrt::launch_zero(P.counts, L.pixels, stream) != 0)
            return fail(MRT_EDEVICE, "zero kernel launch failed");
        if (P.energy && mrt::launch_zero(P.energy, 2 * L.pixels, stream) != 0)
            return fail(MRT_EDEVICE, "zero kernel launch failed");
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    auto drop_events = [&] {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    };
    if (h_counters && timed) {
        if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess ||
            hipEventRecord(ev0, stream) != hipSuccess) {
            drop_events();
            return hip_fail(hipGetLastError(), "hipEvent setup");
        }
    }
    void *args[] = {&P};
    if (hipLaunchKernel(L.kernel, dim3((unsigned)L.grid), dim3((unsigned)L.block), args, 0, stream) !=
        hipSuccess) {
        drop_events();
        return fail(MRT_EDEVICE, "trace kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    }
    if (!h_counters) return MRT_OK;
    if (ev1) (void)hipEventRecord(ev1, stream);
    unsigned long long host[mrt::kNumCounters];
    hipError_t e = hipMemcpyAsync(host, P.dev_counters, sizeof host, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        drop_events();
        return hip_fail(e, "counter readback");
    }
    float ms = 0.0f;
    if (ev0) (void)hipEventElapsedTime(&ms, ev0, ev1);
    drop_events();
    h_counters->emitted = P.n;
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
    h_counters->records = L.opt.records_mode == MRT_RECORDS_ALL
                              ? P.n
                              : std::min<unsigned long long>(nrec, P.rec_cap);
    h_counters->kernel_ms = ms;
    if (L.opt.records_mode == MRT_RECORDS_DETECTED && nrec > P.rec_cap)
        return fail(MRT_ECAPACITY, "%llu detected records, capacity %llu", nrec,
                    (unsigned long long)P.rec_cap);
    return MRT_OK;
}

// ---- scratch of the entry point that allocates nothing --------------------
// Counters, chunk cursor and tables of mrt_trace_noalloc: one copy of this
// array per device, held until the process ends.  In host code the name
// `scratch` only identifies the symbol; its device address, which differs
// per device, comes from hipGetSymbolAddress (once per device, with that
// device current) and is the only way host code refers to its memory.
constexpr size_t kNoAllocScratchBytes = 128 * 1024;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices];

mrt_status noalloc_scratch(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(MRT_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(MRT_EDEVICE, "hipGetSymbolAddress(scratch) gave NULL");
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return MRT_OK;
}

// ---- pinned staging of host tables ---------------------------------------
// A call's tables go to the device by an asynchronous copy from pinned host
// memory owned by the library; an event recorded after the copy on the
// caller's stream marks when the buffer may be reused, so mrt_trace never
// waits for the stream to upload them.  Buffers are per device and kept
// until the process ends.
struct Stage {
    int dev;
    void *host;
    hipEvent_t done;
    bool busy;
};
std::mutex g_stage_mu;
std::vector<Stage *> g_stages;
constexpr size_t kStageBytes = (size_t)mrt::kMaxStagedTableBytes + 3 * ((size_t)mrt::kMaxPsiNodes + 1) * sizeof(double);

mrt_status stage_acquire(int dev, size_t bytes, Stage **out) {
    if (bytes > kStageBytes) return fail(MRT_EINVAL, "tables of %zu bytes exceed the staging size", bytes);
    std::lock_guard<std::mutex> lk(g_stage_mu);
    for (Stage *s : g_stages) {
        if (s->dev != dev || s->busy) continue;
        const hipError_t q = hipEventQuery(s->done);
        if (q == hipSuccess) {
            s->busy = true;
            *out = s;
            return MRT_OK;
        }
        if (q != hipErrorNotReady) return hip_fail(q, "hipEventQuery(staging)");
    }
    Stage *s = new Stage{dev, nullptr, nullptr, true};
    hipError_t e = hipHostMalloc(&s->host, kStageBytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (s->host) (void)hipHostFree(s->host);
        delete s;
        return fail(MRT_ENOMEM, "pinned table staging: %s", hipGetErrorString(e));
    }
    g_stages.push_back(s);
    *out = s;
    return MRT_OK;
}

// Return a buffer to the pool once its copy and the event after it are
// enqueued (or nothing reads it: the copy failed to enqueue).
void stage_release(Stage *s) {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    s->busy = false;
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
    Launch L;
    mrt_status st = prepare(source, crystal, mosaic, rocking_curve, detector, first_ray_id, n_rays,
                            seed, options, d_counts, d_energy_mev, d_records, records_capacity, L);
    if (st != MRT_OK) return st;
    hipStream_t stream = (hipStream_t)hip_stream;

    // library scratch in stream order: counters, chunk cursor, tables
    const size_t bytes = scratch_bytes(L);
    void *scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, bytes, stream);
    if (e != hipSuccess) return fail(MRT_ENOMEM, "hipMallocAsync(%zu): %s", bytes, hipGetErrorString(e));
    bind_scratch(L, scratch);
    auto release = [&](mrt_status s) {
        (void)hipFreeAsync(scratch, stream);
        return s;
    };
    if (!L.tables.empty()) {
        // through pinned staging that the stream releases after the copy,
        // so the call does not wait for the stream
        const size_t tb = L.tables.size() * sizeof(double);
        Stage *sg = nullptr;
        if ((st = stage_acquire(L.dev, tb, &sg)) != MRT_OK) return release(st);
        std::memcpy(sg->host, L.tables.data(), tb);
        e = hipMemcpyAsync(L.dtab, sg->host, tb, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) {
            stage_release(sg);
            return release(hip_fail(e, "table upload"));
        }
        e = hipEventRecord(sg->done, stream);
        if (e != hipSuccess) {
            // no event guards the buffer: wait until the stream has read it
            (void)hipStreamSynchronize(stream);
            stage_release(sg);
            return release(hip_fail(e, "hipEventRecord(staging)"));
        }
        stage_release(sg);
    }
    st = enqueue(L, stream, h_counters, true);
    release(MRT_OK);
    return st;
}

mrt_status mrt_trace_noalloc(const mrt_source *source, const mrt_crystal *crystal,
                             const mrt_mosaic *mosaic, const mrt_rocking_curve *rocking_curve,
                             const mrt_detector *detector, uint64_t first_ray_id, uint64_t n_rays,
                             uint64_t seed, const mrt_options *options, uint32_t *d_counts,
                             uint64_t *d_energy_mev, mrt_hit_record *d_records,
                             uint64_t records_capacity, mrt_counters *h_counters,
                             void *hip_stream) {
    mrt::clear_error();
    Launch L;
    mrt_status st = prepare(source, crystal, mosaic, rocking_curve, detector, first_ray_id, n_rays,
                            seed, options, d_counts, d_energy_mev, d_records, records_capacity, L);
    if (st != MRT_OK) return st;
    hipStream_t stream = (hipStream_t)hip_stream;
    const size_t bytes = scratch_bytes(L);
    if (bytes > kNoAllocScratchBytes)
        return fail(MRT_ECAPACITY, "counters and tables need %zu bytes, the static scratch holds %zu",
                    bytes, kNoAllocScratchBytes);
    void *ptr = nullptr;
    if ((st = noalloc_scratch(L.dev, &ptr)) != MRT_OK) return st;
    bind_scratch(L, ptr);
    if (!L.tables.empty()) {
        // from the (pageable) host vector, which dies with this call
        hipError_t e = hipMemcpyAsync(L.dtab, L.tables.data(), L.tables.size() * sizeof(double),
                                      hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "table upload");
    }
    return enqueue(L, stream, h_counters, false);
}

}  // extern "C"
