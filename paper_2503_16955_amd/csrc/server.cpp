// Request server (continuous batching): the host engine around the serving
// kernel.  The scheduling policy (admission, fair-share rounds, completion)
// lives in server_plan.h; this file owns the device memory, the background
// engine thread and the C-ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mosaicrt.h"
#include "params.h"
#include "server_plan.h"
#include "trace_params.h"

namespace {

using mrt::fail;

// Host record of one request.
struct Rec {
    mrt::TraceParams P;            // parameter block (device pointers set at admission)
    std::vector<double> tables;    // rocking-curve table, then spectrum CDF
    int32_t nx = 0, ny = 0;
    uint64_t n_rays = 0;
    uint32_t *d_counts = nullptr;
    unsigned long long *d_energy = nullptr;
    double *d_tables = nullptr;
    bool ext = false;              // uses the extended inputs
    mrt_counters counters{};
};

// Rounds in flight at once.  While one round's last waves finish, the next
// round's waves already fill the freed compute units (the rounds run on two
// streams), and the host prepares rounds while the device works.
constexpr int kDepth = 2;
static_assert(kDepth == 2, "the engine alternates between two round buffers");

// A launched round: its pieces (for completion) and its buffer.
struct Round {
    std::vector<mrt::serve::Item> items;
    int buf = 0;
};

}  // namespace

struct mrt_server {
    mrt_server_config cfg{};
    int device = 0;
    mrt::serve::Plan plan;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<uint64_t, Rec> recs;
    std::deque<uint64_t> finished;              // completion queue for wait_any
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread engine;
    hipStream_t setup = nullptr;                // admission uploads and frees
    hipEvent_t ev_setup = nullptr;              // end of the latest admission uploads
    bool setup_recorded = false;
    hipEvent_t ev_ref = nullptr;                // time origin of the busy figure
    // pinned staging per slot: parameter block and tables of the request in
    // the slot (rewritten only when the slot is reassigned, by which time the
    // previous request's rounds, which waited for its uploads, are done)
    mrt::TraceParams *h_params = nullptr;
    double *h_tables = nullptr;                 // max_slots x kMaxStagedTableBytes
    double busy_end = 0.0;                      // end of the last completed round (ms)
    mrt::TraceParams *d_slots = nullptr;
    unsigned long long *d_counters = nullptr;   // max_slots x kNumCounters
    // per round buffer (kDepth rounds in flight, each on its own stream)
    hipStream_t streams[kDepth] = {};
    hipEvent_t ev0[kDepth] = {}, ev1[kDepth] = {};
    // items of a round followed by their zeroed chunk cursors, one copy
    mrt::ServeItem *d_items[kDepth] = {};
    mrt::ServeItem *h_items[kDepth] = {};       // pinned staging
    unsigned long long *h_counters[kDepth] = {}; // pinned snapshot of all slots' counters
    std::deque<Round> inflight;
    const void *kernel = nullptr;
    int grid = 0;
    const void *kernel_ext = nullptr;   // for rounds holding extended-input requests
    int grid_ext = 0;
    std::chrono::steady_clock::time_point t0;
    mrt_server_stats stats{};

    mrt_server(const mrt_server_config &c, uint64_t round_rays, uint32_t chunk)
        : cfg(c), plan(c.hbm_budget_bytes, c.max_slots, round_rays, chunk),
          t0(std::chrono::steady_clock::now()) {}

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
            .count();
    }
};

namespace {

uint64_t request_bytes(const Rec &r) {
    return (uint64_t)r.nx * (uint64_t)r.ny * (sizeof(uint32_t) + sizeof(uint64_t)) +
           r.tables.size() * sizeof(double);
}

void free_rec(mrt_server *S, Rec &r) {
    if (r.d_counts) (void)hipFreeAsync(r.d_counts, S->setup);
    if (r.d_energy) (void)hipFreeAsync(r.d_energy, S->setup);
    if (r.d_tables) (void)hipFreeAsync(r.d_tables, S->setup);
    r.d_counts = nullptr;
    r.d_energy = nullptr;
    r.d_tables = nullptr;
}

// Device set-up of an admitted request (engine thread, lock held), enqueued
// on the set-up stream from pinned staging; the caller records the set-up
// event that every later round waits for.
bool admit_one(mrt_server *S, uint64_t ticket) {
    Rec &r = S->recs.at(ticket);
    const int32_t slot = S->plan.find(ticket)->slot;
    const size_t px = (size_t)r.nx * (size_t)r.ny;
    hipError_t e = hipMallocAsync((void **)&r.d_counts, px * sizeof(uint32_t), S->setup);
    if (e == hipSuccess)
        e = hipMallocAsync((void **)&r.d_energy, px * sizeof(uint64_t), S->setup);
    if (e == hipSuccess && !r.tables.empty())
        e = hipMallocAsync((void **)&r.d_tables, r.tables.size() * sizeof(double), S->setup);
    if (e != hipSuccess) {
        free_rec(S, r);
        return false;
    }
    mrt::TraceParams &P = r.P;
    P.counts = r.d_counts;
    P.energy = r.d_energy;
    const int nl = P.irc == MRT_IRC_TABLE ? P.lut_n : 0;
    P.lut = nl ? r.d_tables : nullptr;
    P.lut_env = nl ? r.d_tables + P.env_at : nullptr;
    P.bin_cdf = P.spectrum == MRT_SPECTRUM_TABLE ? r.d_tables + nl : nullptr;
    P.qe = P.qe_n > 0 ? r.d_tables + P.qe_at : nullptr;
    P.dep = P.dep_n > 0 ? r.d_tables + P.dep_at : nullptr;
    P.dev_counters = S->d_counters + (size_t)slot * mrt::kNumCounters;
    P.records_mode = MRT_RECORDS_NONE;
    P.refill_idle = S->cfg.refill_idle > 0 ? (uint32_t)S->cfg.refill_idle : mrt::default_refill(r.ext, S->cfg.precision == MRT_FP64);
    double *ht = S->h_tables + (size_t)slot * (mrt::kMaxStagedTableBytes / sizeof(double));
    if (!r.tables.empty()) {
        std::memcpy(ht, r.tables.data(), r.tables.size() * sizeof(double));
        e = hipMemcpyAsync(r.d_tables, ht, r.tables.size() * sizeof(double),
                           hipMemcpyHostToDevice, S->setup);
    }
    if (e == hipSuccess) e = (hipError_t)mrt::launch_zero(r.d_counts, px, S->setup);
    if (e == hipSuccess) e = (hipError_t)mrt::launch_zero(r.d_energy, 2 * px, S->setup);
    if (e == hipSuccess) e = (hipError_t)mrt::launch_zero(P.dev_counters, 2 * mrt::kNumCounters, S->setup);
    S->h_params[slot] = P;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&S->d_slots[slot], &S->h_params[slot], sizeof(P), hipMemcpyHostToDevice,
                           S->setup);
    if (e != hipSuccess) {
        free_rec(S, r);
        return false;
    }
    return true;
}

// A finished request's counters, from the snapshot taken after the round
// that finished it (which also waited for the round before it).
void read_counters(mrt_server *S, Rec &r, int32_t slot, int buf) {
    const unsigned long long *h = S->h_counters[buf] + (size_t)slot * mrt::kNumCounters;
    mrt_counters &c = r.counters;
    c.emitted = r.n_rays;
    c.missed = h[mrt::kCMissed];
    c.absorbed = h[mrt::kCAbsorbed];
    c.exit_reflected = h[mrt::kCExitReflected];
    c.exit_transmitted = h[mrt::kCExitTransmitted];
    c.truncated = h[mrt::kCTruncated];
    c.detected = h[mrt::kCDetected];
    c.events = h[mrt::kCEvents];
    c.reflections = h[mrt::kCReflections];
    c.refined = h[mrt::kCRefined];
    c.records = 0;
    c.kernel_ms = 0.0;
}

// Admit queued requests while slots and memory allow; their uploads are
// enqueued, and every round launched afterwards waits for them.
void admit_all(mrt_server *S) {
    std::vector<uint64_t> ok;
    for (uint64_t t : S->plan.admit(S->now_ms())) {
        if (admit_one(S, t)) {
            ok.push_back(t);
        } else {
            S->plan.fail(t, MRT_ENOMEM, S->now_ms());
            S->finished.push_back(t);
            S->cv_done.notify_all();
        }
    }
    if (!ok.empty()) {
        if (hipEventRecord(S->ev_setup, S->setup) == hipSuccess) {
            S->setup_recorded = true;
        } else {
            for (uint64_t t : ok) {
                S->plan.fail(t, MRT_EDEVICE, S->now_ms());
                S->finished.push_back(t);
            }
            S->cv_done.notify_all();
        }
    }
}

// Every running request of the given pieces fails (device error).
void fail_items(mrt_server *S, const std::vector<mrt::serve::Item> &items) {
    const double now = S->now_ms();
    for (const auto &it : items) {
        const mrt::serve::Request *q = S->plan.find(it.ticket);
        if (q && q->state == mrt::serve::kRunning) {
            S->plan.fail(it.ticket, MRT_EDEVICE, now);
            S->finished.push_back(it.ticket);
        }
    }
}

// Stage a round in buffer b (lock held): one item per request (the round's
// pieces of a request are contiguous), chunks of about a quarter of a wave's
// share of the round in whole waves of rays, as the one-call path sizes them.
// Stage a round's items in buffer b: the plain requests' items first, then
// those of requests using the extended inputs, each group with its own
// prefix sums and chunk size (the groups are traced by two launches, so that
// every request runs the kernel a separate mrt_trace call would use).
void stage_round(mrt_server *S, const std::vector<mrt::serve::Item> &items, int b, uint32_t *n_out,
                 uint64_t *total_out, uint32_t *n_ext_out, uint64_t *total_ext_out) {
    mrt::ServeItem *h = S->h_items[b];
    uint32_t n = 0;
    uint64_t tot[2] = {0, 0};
    uint32_t cnt[2] = {0, 0};
    for (int g = 0; g < 2; ++g) {
        const uint32_t start = n;
        for (const auto &it : items) {
            if ((int)S->recs.at(it.ticket).ext != g) continue;
            mrt::ServeItem *last = n > start ? &h[n - 1] : nullptr;
            if (last && last->slot == it.slot && last->first + last->count == it.first) {
                last->count += it.count;
            } else {
                h[n++] = mrt::ServeItem{it.first, it.count, tot[g], it.slot, 0u};
            }
            tot[g] += it.count;
        }
        cnt[g] = n - start;
        const uint64_t waves = (uint64_t)(g ? S->grid_ext : S->grid) * 4u;
        uint64_t chunk = (tot[g] / (waves * 4u) + 63u) / 64u * 64u;
        chunk = std::max<uint64_t>(64u, std::min<uint64_t>(2048u, chunk));
        for (uint32_t k = start; k < n; ++k) h[k].chunk = (uint32_t)chunk;
    }
    // the chunk cursors follow the items, zeroed by the same copy
    std::memset(h + n, 0, n * sizeof(unsigned long long));
    *n_out = cnt[0];
    *total_out = tot[0];
    *n_ext_out = cnt[1];
    *total_ext_out = tot[1];
}

// Enqueue a staged round on its stream (lock not held): wait for the latest
// admission uploads, copy the items and zeroed cursors, launch, then snapshot
// every slot's counters once the round before it (other) has ended too.
hipError_t launch_round(mrt_server *S, int b, uint32_t n, uint64_t total, uint32_t n_ext,
                        uint64_t total_ext, bool wait_setup, hipEvent_t other) {
    hipStream_t st = S->streams[b];
    const uint32_t n_all = n + n_ext;
    hipError_t e = wait_setup ? hipStreamWaitEvent(st, S->ev_setup, 0) : hipSuccess;
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->d_items[b], S->h_items[b],
                           n_all * (sizeof(mrt::ServeItem) + sizeof(unsigned long long)),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(S->ev0[b], st);
    unsigned long long *cursors = (unsigned long long *)(S->d_items[b] + n_all);
    if (e == hipSuccess && n) {
        void *args[] = {&S->d_slots, &S->d_items[b], &n, &total, &cursors};
        e = hipLaunchKernel(S->kernel, dim3((unsigned)S->grid), dim3(256), args, 0, st);
    }
    if (e == hipSuccess && n_ext) {
        mrt::ServeItem *items_ext = S->d_items[b] + n;
        unsigned long long *cursors_ext = cursors + n;
        void *args[] = {&S->d_slots, &items_ext, &n_ext, &total_ext, &cursors_ext};
        e = hipLaunchKernel(S->kernel_ext, dim3((unsigned)S->grid_ext), dim3(256), args, 0, st);
    }
    if (e == hipSuccess && other) e = hipStreamWaitEvent(st, other, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->h_counters[b], S->d_counters,
                           sizeof(unsigned long long) * mrt::kNumCounters * (size_t)S->cfg.max_slots,
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(S->ev1[b], st);
    return e;
}

// Wait for the oldest round in flight and account for it (lock held on
// entry and exit, released while waiting).  A device error fails the
// requests of every round in flight, after waiting for all of them.
void finish_oldest(mrt_server *S, std::unique_lock<std::mutex> &lk) {
    Round rd = std::move(S->inflight.front());
    S->inflight.pop_front();
    lk.unlock();
    hipError_t e = hipEventSynchronize(S->ev1[rd.buf]);
    float t0 = 0.0f, t1 = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t0, S->ev_ref, S->ev0[rd.buf]);
    if (e == hipSuccess) e = hipEventElapsedTime(&t1, S->ev_ref, S->ev1[rd.buf]);
    lk.lock();
    if (e != hipSuccess) {
        fail_items(S, rd.items);
        while (!S->inflight.empty()) {
            Round o = std::move(S->inflight.front());
            S->inflight.pop_front();
            lk.unlock();
            (void)hipEventSynchronize(S->ev1[o.buf]);
            lk.lock();
            fail_items(S, o.items);
        }
        S->cv_done.notify_all();
        return;
    }
    // busy time: the union of the rounds' kernel intervals
    S->stats.busy_ms += std::max(0.0, (double)t1 - std::max((double)t0, S->busy_end));
    S->busy_end = std::max(S->busy_end, (double)t1);
    S->stats.rounds += 1;
    for (const auto &it : rd.items) S->stats.rays_traced += it.count;
    for (uint64_t t : S->plan.complete_round(rd.items, S->now_ms())) {
        const mrt::serve::Request *q = S->plan.find(t);
        if (q && q->state == mrt::serve::kDone) read_counters(S, S->recs.at(t), q->slot, rd.buf);
        S->finished.push_back(t);
    }
    S->cv_done.notify_all();
}

void engine(mrt_server *S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        if (S->stop) break;
        admit_all(S);
        // keep kDepth rounds in flight
        while ((int)S->inflight.size() < kDepth && !S->stop) {
            std::vector<mrt::serve::Item> items = S->plan.plan_round();
            if (items.empty()) break;
            const int b = S->inflight.empty() ? 0 : 1 - S->inflight.back().buf;
            hipEvent_t other = S->inflight.empty() ? nullptr : S->ev1[S->inflight.back().buf];
            const bool wait_setup = S->setup_recorded;
            uint32_t n = 0, n_ext = 0;
            uint64_t total = 0, total_ext = 0;
            stage_round(S, items, b, &n, &total, &n_ext, &total_ext);
            lk.unlock();
            const hipError_t e = launch_round(S, b, n, total, n_ext, total_ext, wait_setup, other);
            lk.lock();
            if (e != hipSuccess) {
                fail_items(S, items);
                S->cv_done.notify_all();
                continue;
            }
            S->inflight.push_back(Round{std::move(items), b});
        }
        if (S->inflight.empty()) {
            S->cv_done.notify_all();
            if (!S->stop) S->cv_work.wait(lk);
            continue;
        }
        finish_oldest(S, lk);
    }
    while (!S->inflight.empty()) finish_oldest(S, lk);
    S->cv_done.notify_all();
}

void fill_result(const mrt_server *S, uint64_t ticket, mrt_request_result *out) {
    const mrt::serve::Request *q = S->plan.find(ticket);
    const Rec &r = S->recs.at(ticket);
    std::memset(out, 0, sizeof *out);
    out->state = q->state;
    out->status = q->status;
    out->d_counts = r.d_counts;
    out->d_energy_mev = (uint64_t *)r.d_energy;
    out->nx = r.nx;
    out->ny = r.ny;
    out->rays_done = q->completed;
    if (q->state == mrt::serve::kDone) out->counters = r.counters;
    out->submit_ms = q->t_submit;
    out->admit_ms = q->t_admit;
    out->done_ms = q->t_done;
}

bool terminal(int32_t s) {
    return s == mrt::serve::kDone || s == mrt::serve::kFailed || s == mrt::serve::kCanceled;
}

}  // namespace

extern "C" {

mrt_status mrt_server_create(const mrt_server_config *config, mrt_server **out) {
    if (!config || !out) return fail(MRT_EINVAL, "null argument");
    const mrt_server_config &c = *config;
    if (c.hbm_budget_bytes == 0) return fail(MRT_EINVAL, "hbm_budget_bytes must be > 0");
    if (c.max_slots < 1 || c.max_slots > 1024) return fail(MRT_EINVAL, "max_slots must be 1..1024");
    if (c.precision != MRT_FP64 && c.precision != MRT_FP32_MIXED)
        return fail(MRT_EINVAL, "unknown precision");
    if (c.chunk % 64 != 0) return fail(MRT_EINVAL, "chunk must be a multiple of 64");
    if (c.refill_idle < 0 || c.refill_idle > 64) return fail(MRT_EINVAL, "refill_idle must be 0..64");
    const uint64_t round_rays = c.round_rays ? c.round_rays : (1ull << 24);
    const uint32_t chunk = c.chunk ? c.chunk : 4096u;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MRT_EDEVICE, "no device");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(MRT_EDEVICE, "no device properties");
    mrt_server *S = new mrt_server(c, round_rays, chunk);
    S->cfg.round_rays = round_rays;
    S->cfg.chunk = chunk;
    S->device = dev;
    S->kernel = mrt::serve_kernel_ptr(c.precision, false);
    S->kernel_ext = mrt::serve_kernel_ptr(c.precision, true);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, S->kernel, 256, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    S->grid = per_cu * prop.multiProcessorCount;
    per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, S->kernel_ext, 256, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    S->grid_ext = per_cu * prop.multiProcessorCount;
    const size_t ms = (size_t)c.max_slots;
    bool ok = hipStreamCreateWithFlags(&S->setup, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreate(&S->ev_ref) == hipSuccess && hipEventCreate(&S->ev_setup) == hipSuccess &&
              hipHostMalloc((void **)&S->h_params, sizeof(mrt::TraceParams) * ms, 0) == hipSuccess &&
              hipHostMalloc((void **)&S->h_tables, (size_t)mrt::kMaxStagedTableBytes * ms, 0) == hipSuccess &&
              hipMalloc((void **)&S->d_slots, sizeof(mrt::TraceParams) * ms) == hipSuccess &&
              hipMalloc((void **)&S->d_counters, sizeof(unsigned long long) * mrt::kNumCounters * ms) ==
                  hipSuccess;
    for (int b = 0; ok && b < kDepth; ++b)
        ok = hipStreamCreateWithFlags(&S->streams[b], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreate(&S->ev0[b]) == hipSuccess && hipEventCreate(&S->ev1[b]) == hipSuccess &&
             hipMalloc((void **)&S->d_items[b], (sizeof(mrt::ServeItem) + sizeof(unsigned long long)) * ms) ==
                 hipSuccess &&
             hipHostMalloc((void **)&S->h_items[b], (sizeof(mrt::ServeItem) + sizeof(unsigned long long)) * ms,
                           0) == hipSuccess &&
             hipHostMalloc((void **)&S->h_counters[b], sizeof(unsigned long long) * mrt::kNumCounters * ms,
                           0) == hipSuccess;
    // the time origin of the busy figure
    ok = ok && hipEventRecord(S->ev_ref, S->setup) == hipSuccess &&
         hipStreamSynchronize(S->setup) == hipSuccess;
    if (!ok) {
        mrt_server_destroy(S);
        return fail(MRT_ENOMEM, "server set-up allocation failed");
    }
    S->engine = std::thread(engine, S);
    *out = S;
    return MRT_OK;
}

mrt_status mrt_server_submit(mrt_server *S, const mrt_request *q, uint64_t *ticket) {
    if (!S || !q || !ticket) return fail(MRT_EINVAL, "null argument");
    mrt_status st = mrt::validate(q->source, q->crystal, q->mosaic, q->rocking_curve, q->detector,
                                  fail);
    if (st != MRT_OK) return st;
    if (q->n_rays == 0) return fail(MRT_EINVAL, "n_rays must be > 0");
    Rec r;
    r.ext = mrt::uses_ext(q->source, q->crystal, q->rocking_curve);
    mrt::build_params(q->source, q->crystal, q->mosaic, q->rocking_curve, q->detector, r.P,
                      r.tables);
    // the slot's staging holds the validated tables plus the curve's envelope
    if (r.tables.size() * sizeof(double) > (size_t)mrt::kMaxStagedTableBytes)
        return fail(MRT_EINVAL, "tables of %zu bytes exceed the staging size",
                    r.tables.size() * sizeof(double));
    r.nx = q->detector->nx;
    r.ny = q->detector->ny;
    r.n_rays = q->n_rays;
    r.P.first = 0;
    r.P.n = q->n_rays;
    r.P.seed = q->seed;
    r.P.key0 = (uint32_t)q->seed;
    r.P.key1 = (uint32_t)(q->seed >> 32);
    r.P.max_events = q->max_events ? q->max_events : (1u << 20);
    const uint64_t bytes = request_bytes(r);
    std::lock_guard<std::mutex> lk(S->mu);
    const uint64_t t = S->next_ticket++;
    if (!S->plan.submit(t, q->n_rays, bytes, S->now_ms()))
        return fail(MRT_ENOMEM, "request needs %llu bytes, budget is %llu",
                     (unsigned long long)bytes, (unsigned long long)S->plan.budget());
    S->recs.emplace(t, std::move(r));
    S->stats.submitted += 1;
    *ticket = t;
    S->cv_work.notify_all();
    return MRT_OK;
}

mrt_status mrt_server_poll(mrt_server *S, uint64_t ticket, mrt_request_result *result) {
    if (!S || !result) return fail(MRT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->plan.find(ticket)) return fail(MRT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    fill_result(S, ticket, result);
    return MRT_OK;
}

mrt_status mrt_server_wait(mrt_server *S, uint64_t ticket, double timeout_ms,
                           mrt_request_result *result) {
    if (!S || !result) return fail(MRT_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    if (!S->plan.find(ticket)) return fail(MRT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    auto done = [&] { const auto *q = S->plan.find(ticket); return !q || terminal(q->state) || S->stop; };
    if (timeout_ms < 0) {
        S->cv_done.wait(lk, done);
    } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), done)) {
        fill_result(S, ticket, result);
        return fail(MRT_EAGAIN, "request %llu not finished", (unsigned long long)ticket);
    }
    if (!S->plan.find(ticket)) return fail(MRT_EINVAL, "ticket %llu released", (unsigned long long)ticket);
    fill_result(S, ticket, result);
    return MRT_OK;
}

mrt_status mrt_server_wait_any(mrt_server *S, double timeout_ms, uint64_t *ticket,
                               mrt_request_result *result) {
    if (!S || !ticket || !result) return fail(MRT_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                              std::chrono::duration<double, std::milli>(timeout_ms < 0 ? 0.0 : timeout_ms));
    for (;;) {
        // tickets released before they were reported are skipped
        while (!S->finished.empty() && !S->plan.find(S->finished.front())) S->finished.pop_front();
        if (!S->finished.empty()) break;
        if (S->stop) return fail(MRT_EINVAL, "server stopped");
        if (timeout_ms < 0) {
            S->cv_done.wait(lk);
        } else if (S->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
            while (!S->finished.empty() && !S->plan.find(S->finished.front())) S->finished.pop_front();
            if (S->finished.empty()) return fail(MRT_EAGAIN, "no request finished within the timeout");
            break;
        }
    }
    const uint64_t t = S->finished.front();
    S->finished.pop_front();
    *ticket = t;
    fill_result(S, t, result);
    return MRT_OK;
}

mrt_status mrt_server_cancel(mrt_server *S, uint64_t ticket) {
    if (!S) return fail(MRT_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->plan.cancel(ticket, S->now_ms()))
        return fail(MRT_EINVAL, "ticket %llu is unknown or finished", (unsigned long long)ticket);
    if (S->plan.find(ticket)->state == mrt::serve::kCanceled) S->finished.push_back(ticket);
    S->cv_work.notify_all();
    S->cv_done.notify_all();
    return MRT_OK;
}

mrt_status mrt_server_release(mrt_server *S, uint64_t ticket) {
    if (!S) return fail(MRT_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->recs.find(ticket);
    if (it == S->recs.end() || S->plan.release(ticket) < 0)
        return fail(MRT_EINVAL, "ticket %llu is unknown or not finished", (unsigned long long)ticket);
    free_rec(S, it->second);
    S->recs.erase(it);
    S->cv_work.notify_all();   // memory freed: queued requests may fit now
    return MRT_OK;
}

mrt_status mrt_server_get_stats(mrt_server *S, mrt_server_stats *out) {
    if (!S || !out) return fail(MRT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    out->queued = S->plan.queued();
    out->running = S->plan.running();
    uint64_t d = 0, f = 0, c = 0;
    for (const auto &kv : S->recs) {
        const auto *q = S->plan.find(kv.first);
        if (!q) continue;
        d += q->state == mrt::serve::kDone;
        f += q->state == mrt::serve::kFailed;
        c += q->state == mrt::serve::kCanceled;
    }
    out->done = d;
    out->failed = f;
    out->canceled = c;
    out->used_bytes = S->plan.used_bytes();
    out->budget_bytes = S->plan.budget();
    return MRT_OK;
}

void mrt_server_destroy(mrt_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
    if (S->engine.joinable()) S->engine.join();   // the engine waits for its rounds in flight
    if (S->setup) {
        for (auto &kv : S->recs) free_rec(S, kv.second);
        (void)hipStreamSynchronize(S->setup);
    }
    if (S->d_slots) (void)hipFree(S->d_slots);
    if (S->d_counters) (void)hipFree(S->d_counters);
    for (int b = 0; b < kDepth; ++b) {
        if (S->d_items[b]) (void)hipFree(S->d_items[b]);
        if (S->h_items[b]) (void)hipHostFree(S->h_items[b]);
        if (S->h_counters[b]) (void)hipHostFree(S->h_counters[b]);
        if (S->ev0[b]) (void)hipEventDestroy(S->ev0[b]);
        if (S->ev1[b]) (void)hipEventDestroy(S->ev1[b]);
        if (S->streams[b]) (void)hipStreamDestroy(S->streams[b]);
    }
    if (S->ev_ref) (void)hipEventDestroy(S->ev_ref);
    if (S->ev_setup) (void)hipEventDestroy(S->ev_setup);
    if (S->h_params) (void)hipHostFree(S->h_params);
    if (S->h_tables) (void)hipHostFree(S->h_tables);
    if (S->setup) (void)hipStreamDestroy(S->setup);
    delete S;
}

}  // extern "C"
