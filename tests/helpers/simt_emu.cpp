// CPU execution of the trace kernels' device code for tests.  A wave is 64
// coroutines (ucontext) stepped in lane order; each wave-level operation
// (ballot, readfirstlane) is a meeting point where every lane must arrive
// before any continues, which is exactly the lockstep the kernels assume at
// those points (they only occur in wave-uniform control flow).  A lane that
// reaches a different meeting point from its wave, or ends early, is an error.
// Waves of a grid run one after another (a valid interleaving for the
// kernels, which only communicate through atomics).
#include <hip/hip_runtime.h>
#include <ucontext.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

#include "mosaicrt.h"
#include "params.h"
#include "trace_impl.h"
#include "trace_mwg.h"   // the paper's event model (trace_mwg.hip)
#include "trace_params.h"

thread_local simt_dim3 threadIdx, blockIdx, blockDim, gridDim;

namespace {

constexpr int kLanes = 64;
constexpr size_t kStack = 512 * 1024;

enum Op { kNone = 0, kBallot = 1, kFirst = 2 };

struct Wave {
    ucontext_t sched;
    ucontext_t ctx[kLanes];
    std::vector<char> stacks;
    int lane = 0;
    bool finished[kLanes];
    int op[kLanes];
    uint64_t arg[kLanes];
    uint64_t result = 0;
    long long meetings = 0;
    int error = 0;
    std::function<void()> body;
};

thread_local Wave *g_wave = nullptr;

void lane_entry() {
    Wave *W = g_wave;
    W->body();
    W->finished[W->lane] = true;
    swapcontext(&W->ctx[W->lane], &W->sched);
}

uint64_t meet(int op, uint64_t v) {
    Wave *W = g_wave;
    W->op[W->lane] = op;
    W->arg[W->lane] = v;
    swapcontext(&W->ctx[W->lane], &W->sched);
    return W->result;
}

// Run `body` as one wave; returns 0, or -1 on a divergent meeting point.
int run_wave(const std::function<void()> &body, long long max_meetings) {
    Wave W;
    W.stacks.resize(kStack * kLanes);
    W.body = body;
    g_wave = &W;
    for (int l = 0; l < kLanes; ++l) {
        W.finished[l] = false;
        getcontext(&W.ctx[l]);
        W.ctx[l].uc_stack.ss_sp = W.stacks.data() + kStack * l;
        W.ctx[l].uc_stack.ss_size = kStack;
        W.ctx[l].uc_link = nullptr;
        makecontext(&W.ctx[l], lane_entry, 0);
    }
    for (;;) {
        for (int l = 0; l < kLanes; ++l) {
            W.lane = l;
            W.op[l] = kNone;
            threadIdx.x = (unsigned)l;
            swapcontext(&W.sched, &W.ctx[l]);
        }
        int n_done = 0;
        for (int l = 0; l < kLanes; ++l) n_done += W.finished[l];
        if (n_done == kLanes) break;
        if (n_done) { W.error = -1; break; }               // some lanes ended, others wait
        const int op = W.op[0];
        for (int l = 1; l < kLanes; ++l)
            if (W.op[l] != op) W.error = -1;               // lanes at different meeting points
        if (W.error) break;
        if (op == kBallot) {
            uint64_t m = 0;
            for (int l = 0; l < kLanes; ++l) m |= (W.arg[l] ? 1ull : 0ull) << l;
            W.result = m;
        } else {
            W.result = W.arg[0];
        }
        if (++W.meetings > max_meetings) { W.error = -2; break; }
    }
    g_wave = nullptr;
    return W.error;
}

}  // namespace

uint64_t simt_ballot(bool p) { return meet(kBallot, p ? 1 : 0); }
void simt_check_failed(const char *cond, const char *file, int line) {
    fprintf(stderr, "device-code check failed: %s (%s:%d)\n", cond, file, line);
    abort();
}
uint32_t simt_readfirstlane(uint32_t v) { return (uint32_t)meet(kFirst, v); }
int simt_lane() { return g_wave ? g_wave->lane : 0; }

namespace mrt {
// error reporting used by params.cpp
static thread_local char g_err[512];
mrt_status fail(mrt_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}
const char *last_error() { return g_err; }
void clear_error() { g_err[0] = 0; }
}  // namespace mrt

namespace {
using namespace mrt;
using namespace mrt::tk;

// `queue` is the wave's LDS ray queue: memory shared by the wave's lanes.
// kDefer: the serving loop with the one-call kernels' deferred detector work
// (the device's serving kernels run without it).
template <class R, bool kDefer = false>
void serve_body(const TraceParams *slots, const ServeItem *items, uint32_t n, uint64_t total,
                unsigned long long *cursors, uint32_t wave, uint32_t n_waves, void *queue) {
    // the serving kernel's body, with the wave index it would compute (the
    // device kernel runs each item in the loop specialised for its kinds,
    // the same template code; here the loop reads the kinds at run time)
    using T = Tracer<R, kAny, kAny, kAny, false>;
    serve_waves(slots, items, n, total, cursors, wave, n_waves,
                LoopRun<T, kDefer, RayQueue<R, false>>{*(RayQueue<R, false> *)queue});
}

// The extended serving kernel's body (spots, user arrays and polarisations,
// energy-dependent curves, further planes).
template <class R, bool kDefer = false>
void serve_body_ext(const TraceParams *slots, const ServeItem *items, uint32_t n, uint64_t total,
                    unsigned long long *cursors, uint32_t wave, uint32_t n_waves, void *queue) {
    using T = Tracer<R, kAny, kAny, kAny, false, true>;
    serve_waves(slots, items, n, total, cursors, wave, n_waves,
                LoopRun<T, kDefer, typename T::Queue>{*(typename T::Queue *)queue});
}

template <class R, bool REC, bool EXT = false>
void trace_body(const TraceParams &P, void *queue) {
    using T = Tracer<R, kAny, kAny, kAny, REC, EXT>;
    RangeClaim claim{P.chunk_counter, P.first, P.n, P.chunk};
    // as the kernels: the one-call kernels defer the ended rays' detector
    // work, the extended ones in FP32-mixed only
    constexpr bool kDefer = EXT ? !T::kF64 : true;
    trace_loop<T, kDefer>(P, P.lut, P.bin_cdf, claim, *(typename T::Queue *)queue);
}

template <bool REC, bool POL, bool PLANES = false>
void mwg_body(const TraceParams &P, void *queue) {
    using T = MwgTracer<kAny, REC, POL, PLANES>;
    RangeClaim claim{P.chunk_counter, P.first, P.n, P.chunk};
    mwg_loop<T>(P, P.lut, P.bin_cdf, claim, *(typename T::Queue *)queue);
}

// Room for any RayQueue, filled with a byte pattern so that a read of an
// entry no lane has written shows up as garbage.
struct QueueMem {
    alignas(64) unsigned char b[sizeof(RayQueue<double, true, true>)];
    QueueMem() { memset(b, 0xA5, sizeof b); }
};
}  // namespace

extern "C" {

// Fill a parameter block from the public structs (host pointers for the
// tables: the emulated kernels read them in place).
int emu_build_params(const mrt_source *s, const mrt_crystal *c, const mrt_mosaic *m,
                     const mrt_rocking_curve *r, const mrt_detector *d, TraceParams *P,
                     double *tables_out, int tables_cap, int *n_tables) {
    if (mrt::validate(s, c, m, r, d, mrt::fail) != MRT_OK) return -1;
    std::vector<double> t;
    mrt::build_params(s, c, m, r, d, *P, t);
    *n_tables = (int)t.size();
    if ((int)t.size() > tables_cap) return -2;
    for (size_t i = 0; i < t.size(); ++i) tables_out[i] = t[i];
    P->lut = P->irc == MRT_IRC_TABLE ? tables_out : nullptr;
    P->lut_env = P->irc == MRT_IRC_TABLE ? tables_out + P->env_at : nullptr;
    P->bin_cdf = P->spectrum == MRT_SPECTRUM_TABLE ? tables_out + (P->irc == MRT_IRC_TABLE ? P->lut_n : 0)
                                                   : nullptr;
    P->qe = P->qe_n > 0 ? tables_out + P->qe_at : nullptr;
    P->dep = P->dep_n > 0 ? tables_out + P->dep_at : nullptr;
    return 0;
}
int emu_params_size() { return (int)sizeof(TraceParams); }

// The FP32 acceptance filter as compiled here (Tracer::sin_delta_f32,
// asin_small_f32, x_bounds and filter), for case i: c = akn[i] = |k.n|,
// s = sa[i] = sin(alpha_B), u = u[i], and the curve read at
// (Delta - shift) / scale.  Outputs per case: the FP32 estimate of x before
// its error band (NaN when sin(Delta) > 1/4 or there is no bound), the
// reference x in long double, the bounds (lo, hi, slo, shi), whether there
// are bounds, the filter's decision (1, 0, -1) and the exact decisions of
// the FP32-mixed and FP64 paths (u < r(x) / R_max, x from FP64 asin), and
// the FP64 path's r(x) / R_max.  `bias` moves the hardware FP32 estimates by
// one ulp (simt_ulp_bias).
void emu_filter_cases(const TraceParams *P, const double *lut, int n, const double *akn,
                      const double *sa, const double *u, double shift, double scale, int bias,
                      float *x_est, double *x_ref, float *bounds, int *has, int *dec, int *dec32,
                      int *dec64, double *ratio) {
    using T32 = Tracer<float, kAny, kAny, kAny, false, true>;
    using T64 = Tracer<double, kAny, kAny, kAny, false, true>;
    simt_ulp_bias = bias;
    const bool ext = scale != 1.0 || shift != P->shift;
    const float shf = ext ? (float)shift : P->f32.shift;
    const float inv_sf = ext ? (float)(1.0 / scale) : 1.0f;
    for (int i = 0; i < n; ++i) {
        const double s = sa[i];
        const float saf = (float)s;
        const float caf = (float)std::sqrt(std::fma(-s, s, 1.0));
        float z = 0.0f;
        x_est[i] = T32::sin_delta_f32(akn[i], saf, caf, z) && std::fabs(z) <= 0.25f
                       ? T32::asin_small_f32(z) - shf
                       : NAN;
        const long double xr = ((asinl((long double)akn[i]) - asinl((long double)s)) -
                                (long double)shift) / (long double)scale;
        x_ref[i] = (double)xr;
        float *b = bounds + 4 * i;
        has[i] = T32::x_bounds(akn[i], saf, caf, shf, inv_sf, b[0], b[1], b[2], b[3]) ? 1 : 0;
        dec[i] = T32::filter(*P, akn[i], saf, caf, (float)u[i], shf, inv_sf);
        const double x = ((std::asin(akn[i]) - std::asin(s)) - shift) / scale;
        dec32[i] = u[i] < T32::irc_ratio(*P, lut, x) ? 1 : 0;
        ratio[i] = T64::irc_ratio(*P, lut, x);
        dec64[i] = u[i] < ratio[i] ? 1 : 0;
    }
    simt_ulp_bias = 0;
}

// The table curve's envelope as the filter reads it: the bucket shift, and
// for an x interval [slo, shi] the bounds table_bounds gives (returns its
// result), with the exact FP64 ratio at n_x points of the interval.
int emu_table_bounds(const TraceParams *P, float slo, float shi, float *r_lo, float *r_hi,
                     int n_x, double *x_out, double *ratio_out, int *env_shift) {
    using T = Tracer<double, kAny, kAny, kAny, false, true>;
    *env_shift = P->env_shift;
    const bool ok = T::table_bounds(*P, slo, shi, *r_lo, *r_hi);
    for (int i = 0; i < n_x; ++i) {
        const double x = (double)slo + ((double)shi - (double)slo) * (double)i / (double)(n_x - 1);
        x_out[i] = x;
        ratio_out[i] = T::irc_ratio(*P, P->lut, x);
    }
    return ok ? 1 : 0;
}

// The paper's event model: its parameters, with the psi table appended at
// tables_out[n_used...] (host memory the emulated kernel reads in place).
int emu_build_mwg(const mrt_crystal *c, const mrt_mosaic *m, const mrt_rocking_curve *r,
                  int burn_in, int psi_nodes, int batch, TraceParams *P, double *tables_out,
                  int tables_cap, int n_used) {
    std::vector<double> t;
    mrt::build_mwg_params(c, m, r, burn_in, psi_nodes, batch, false, *P, t);
    if (n_used + (int)t.size() > tables_cap) return -2;
    for (size_t i = 0; i < t.size(); ++i) tables_out[n_used + i] = t[i];
    P->psi_tab = tables_out + n_used;
    P->psi_cos2 = P->psi_tab + 2 * (psi_nodes + 1);
    return 0;
}

// Run the paper's event model's loop (FP64) with n_waves waves.
int emu_trace_mwg(TraceParams *P, int n_waves, long long max_meetings) {
    for (int w = 0; w < n_waves; ++w) {
        QueueMem q;
        int e = run_wave([&] {
            const bool rec = P->records_mode != MRT_RECORDS_NONE;
            if (P->has_planes || P->dep_n > 0) {
                if (P->user_p) { if (rec) mwg_body<true, true, true>(*P, q.b); else mwg_body<false, true, true>(*P, q.b); }
                else { if (rec) mwg_body<true, false, true>(*P, q.b); else mwg_body<false, false, true>(*P, q.b); }
            } else if (P->user_p) { if (rec) mwg_body<true, true>(*P, q.b); else mwg_body<false, true>(*P, q.b); }
            else { if (rec) mwg_body<true, false>(*P, q.b); else mwg_body<false, false>(*P, q.b); }
        }, max_meetings);
        if (e) return e;
    }
    return 0;
}

// The run fields of a parameter block (as the one-call path and the server
// set them).
void emu_set_run(TraceParams *P, uint64_t first, uint64_t n, uint64_t seed, uint32_t max_events,
                 uint32_t *counts, unsigned long long *energy, unsigned long long *counters,
                 uint32_t chunk, uint32_t refill_idle) {
    P->first = first;
    P->n = n;
    P->seed = seed;
    P->key0 = (uint32_t)seed;
    P->key1 = (uint32_t)(seed >> 32);
    P->max_events = max_events ? max_events : (1u << 20);
    P->records_mode = MRT_RECORDS_NONE;
    P->records = nullptr;
    P->counts = counts;
    P->energy = energy;
    P->dev_counters = counters;
    P->chunk_counter = counters + kNumCounters;
    P->chunk = chunk;
    P->refill_idle = refill_idle;
}

// Records of every ray (ALL mode) into host memory.
void emu_set_records(TraceParams *P, mrt_hit_record *records, uint64_t cap) {
    P->records_mode = MRT_RECORDS_ALL;
    P->records = records;
    P->rec_cap = cap;
}

int emu_serve_group(const TraceParams *slots, const ServeItem *items, uint32_t n, int n_waves,
                    int precision, long long max_meetings, bool ext, bool defer = false);

// The serving loops with deferred detector work (ext: the extended loop).
int emu_serve_defer(const TraceParams *slots, const ServeItem *items, uint32_t n, int n_waves,
                    int precision, long long max_meetings, int ext) {
    return emu_serve_group(slots, items, n, n_waves, precision, max_meetings, ext != 0, true);
}

// Run the serving kernel body with n_waves waves (one after another) over a
// round's items; 0 on success.
int emu_serve(const TraceParams *slots, const ServeItem *items, uint32_t n, int n_waves,
              int precision, long long max_meetings) {
    return emu_serve_group(slots, items, n, n_waves, precision, max_meetings, false);
}

// The same with the extended serving kernel's body.
int emu_serve_ext(const TraceParams *slots, const ServeItem *items, uint32_t n, int n_waves,
                  int precision, long long max_meetings) {
    return emu_serve_group(slots, items, n, n_waves, precision, max_meetings, true);
}

int emu_serve_group(const TraceParams *slots, const ServeItem *items, uint32_t n, int n_waves,
                    int precision, long long max_meetings, bool ext, bool defer) {
    uint64_t total = 0;
    for (uint32_t i = 0; i < n; ++i) total += items[i].count;
    std::vector<unsigned long long> cursors(n ? n : 1, 0ull);
    for (int w = 0; w < n_waves; ++w) {
        QueueMem q;
        int e = run_wave([&] {
            const uint32_t wv = (uint32_t)w, nw = (uint32_t)n_waves;
            const bool f64 = precision == MRT_FP64;
            if (defer) {
                if (ext && f64) serve_body_ext<double, true>(slots, items, n, total, cursors.data(), wv, nw, q.b);
                else if (ext) serve_body_ext<float, true>(slots, items, n, total, cursors.data(), wv, nw, q.b);
                else if (f64) serve_body<double, true>(slots, items, n, total, cursors.data(), wv, nw, q.b);
                else serve_body<float, true>(slots, items, n, total, cursors.data(), wv, nw, q.b);
            } else if (ext && precision == MRT_FP64)
                serve_body_ext<double>(slots, items, n, total, cursors.data(), wv, nw, q.b);
            else if (ext)
                serve_body_ext<float>(slots, items, n, total, cursors.data(), wv, nw, q.b);
            else if (precision == MRT_FP64)
                serve_body<double>(slots, items, n, total, cursors.data(), wv, nw, q.b);
            else
                serve_body<float>(slots, items, n, total, cursors.data(), wv, nw, q.b);
        }, max_meetings);
        if (e) return e;
    }
    return 0;
}

// Run the one-call trace loop (ray range P.first .. P.first + P.n) with
// n_waves waves; P's buffers and counters are host memory.
int emu_trace(TraceParams *P, int n_waves, int precision, long long max_meetings) {
    for (int w = 0; w < n_waves; ++w) {
        QueueMem q;
        int e = run_wave([&] {
            const bool rec = P->records_mode != MRT_RECORDS_NONE;
            // the extended-input kernel: energy-dependent rocking curve,
            // polarisations, further planes (the kernel the device takes)
            if (P->dep_n > 0 || P->user_p || P->has_planes) {
                if (precision == MRT_FP64) { if (rec) trace_body<double, true, true>(*P, q.b); else trace_body<double, false, true>(*P, q.b); }
                else { if (rec) trace_body<float, true, true>(*P, q.b); else trace_body<float, false, true>(*P, q.b); }
            } else if (precision == MRT_FP64) { if (rec) trace_body<double, true>(*P, q.b); else trace_body<double, false>(*P, q.b); }
            else { if (rec) trace_body<float, true>(*P, q.b); else trace_body<float, false>(*P, q.b); }
        }, max_meetings);
        if (e) return e;
    }
    return 0;
}

}  // extern "C"
