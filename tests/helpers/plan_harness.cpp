// C entry points over the request server's scheduling policy
// (paper_2503_16955_amd/csrc/server_plan.h) for the CPU tests.
#include <vector>

#include "server_plan.h"

using mrt::serve::Item;
using mrt::serve::Plan;

struct Harness {
    Plan plan;
    std::vector<Item> last;
    Harness(uint64_t b, int s, uint64_t r, uint32_t c) : plan(b, s, r, c) {}
};

extern "C" {
void *plan_new(uint64_t budget, int slots, uint64_t round_rays, uint32_t chunk) {
    return new Harness(budget, slots, round_rays, chunk);
}
void plan_free(void *h) { delete (Harness *)h; }
int plan_submit(void *h, uint64_t t, uint64_t n, uint64_t bytes, double now) {
    return ((Harness *)h)->plan.submit(t, n, bytes, now) ? 1 : 0;
}
int plan_admit(void *h, double now, uint64_t *out, int cap) {
    auto v = ((Harness *)h)->plan.admit(now);
    int n = 0;
    for (uint64_t t : v) if (n < cap) out[n++] = t;
    return (int)v.size();
}
int plan_round(void *h, uint64_t *tickets, int *slots, uint64_t *firsts, uint32_t *counts, int cap) {
    Harness *H = (Harness *)h;
    H->last = H->plan.plan_round();
    int n = 0;
    for (const Item &it : H->last) {
        if (n < cap) {
            tickets[n] = it.ticket;
            slots[n] = it.slot;
            firsts[n] = it.first;
            counts[n] = it.count;
        }
        ++n;
    }
    return n;
}
int plan_complete(void *h, double now, uint64_t *out, int cap) {
    Harness *H = (Harness *)h;
    auto v = H->plan.complete_round(H->last, now);
    H->last.clear();
    int n = 0;
    for (uint64_t t : v) if (n < cap) out[n++] = t;
    return (int)v.size();
}
void plan_fail(void *h, uint64_t t, int status, double now) { ((Harness *)h)->plan.fail(t, status, now); }
int plan_cancel(void *h, uint64_t t, double now) { return ((Harness *)h)->plan.cancel(t, now) ? 1 : 0; }
long long plan_release(void *h, uint64_t t) { return ((Harness *)h)->plan.release(t); }
// state, slot, scheduled, completed, t_admit, t_done of a request; 0 if unknown
int plan_query(void *h, uint64_t t, int *state, int *slot, uint64_t *scheduled, uint64_t *completed,
               double *t_admit, double *t_done) {
    const mrt::serve::Request *r = ((Harness *)h)->plan.find(t);
    if (!r) return 0;
    *state = r->state;
    *slot = r->slot;
    *scheduled = r->scheduled;
    *completed = r->completed;
    *t_admit = r->t_admit;
    *t_done = r->t_done;
    return 1;
}
uint64_t plan_used(void *h) { return ((Harness *)h)->plan.used_bytes(); }
int plan_free_slots(void *h) { return (int)((Harness *)h)->plan.free_slots(); }
int plan_queued(void *h) { return (int)((Harness *)h)->plan.queued(); }
int plan_running(void *h) { return (int)((Harness *)h)->plan.running(); }
}
