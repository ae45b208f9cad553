// Scheduling policy of the request server: admission by slots and device
// memory, fair-share rounds, completion, cancellation and release.  Pure
// host logic with no device calls (the server drives it and performs the
// allocations and launches), so it is testable on its own.
//
// A request holds a slot (its parameter block on the device) from admission
// until it is done, failed or cancelled, and its device memory (its images)
// from admission until it is released.  Admission is strict FIFO: the oldest
// queued request is admitted as soon as a slot is free and its bytes fit in
// the budget; nothing overtakes it.  Each round gives every running request
// the same share of rays (at least one chunk), so a small request that
// arrives while large ones run finishes after a few rounds.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <map>
#include <vector>

namespace mrt {
namespace serve {

enum State : int32_t {
    kQueued = 0,
    kRunning = 1,
    kDone = 2,
    kFailed = 3,
    kCanceled = 4,
    kReleased = 5
};

struct Request {
    uint64_t ticket = 0;
    uint64_t n_rays = 0;
    uint64_t bytes = 0;          // device memory held from admission to release
    uint64_t scheduled = 0;      // rays handed to rounds so far
    uint64_t completed = 0;      // rays of finished rounds
    int32_t state = kQueued;
    int32_t slot = -1;
    int32_t status = 0;          // failure status
    bool cancel = false;         // cancellation requested while running
    bool holds_bytes = false;
    double t_submit = 0, t_admit = -1, t_done = -1;
};

// One contiguous piece of a round: rays [first, first + count) of the request
// in `slot` (count <= chunk).
struct Item {
    uint64_t ticket;
    int32_t slot;
    uint64_t first;
    uint32_t count;
};

class Plan {
public:
    Plan(uint64_t budget_bytes, int32_t max_slots, uint64_t round_rays, uint32_t chunk)
        : budget_(budget_bytes), round_rays_(round_rays), chunk_(chunk ? chunk : 1) {
        for (int32_t s = max_slots - 1; s >= 0; --s) free_slots_.push_back(s);
    }

    // Queue a request.  Returns false when it could never fit in the budget.
    bool submit(uint64_t ticket, uint64_t n_rays, uint64_t bytes, double now) {
        if (bytes > budget_ || n_rays == 0) return false;
        Request r;
        r.ticket = ticket;
        r.n_rays = n_rays;
        r.bytes = bytes;
        r.t_submit = now;
        reqs_[ticket] = r;
        queue_.push_back(ticket);
        return true;
    }

    // Admit queued requests in FIFO order while slots and memory allow.
    std::vector<uint64_t> admit(double now) {
        std::vector<uint64_t> out;
        while (!queue_.empty()) {
            Request &r = reqs_.at(queue_.front());
            if (free_slots_.empty() || used_ + r.bytes > budget_) break;
            r.slot = free_slots_.back();
            free_slots_.pop_back();
            used_ += r.bytes;
            r.holds_bytes = true;
            r.state = kRunning;
            r.t_admit = now;
            running_.push_back(r.ticket);
            out.push_back(r.ticket);
            queue_.pop_front();
        }
        return out;
    }

    // The next round: each running request (not cancelled, rays left) gets
    // the same share of round_rays, rounded up to whole chunks.
    std::vector<Item> plan_round() {
        std::vector<Item> items;
        std::vector<Request *> live;
        for (uint64_t t : running_) {
            Request &r = reqs_.at(t);
            if (!r.cancel && r.scheduled < r.n_rays) live.push_back(&r);
        }
        if (live.empty()) return items;
        uint64_t share = round_rays_ / live.size();
        share = std::max<uint64_t>(chunk_, (share + chunk_ - 1) / chunk_ * chunk_);
        for (Request *r : live) {
            const uint64_t take = std::min<uint64_t>(share, r->n_rays - r->scheduled);
            for (uint64_t off = 0; off < take; off += chunk_) {
                const uint32_t c = (uint32_t)std::min<uint64_t>(chunk_, take - off);
                items.push_back(Item{r->ticket, r->slot, r->scheduled + off, c});
            }
            r->scheduled += take;
        }
        return items;
    }

    // A round finished: credit its rays; requests whose rays are all done
    // become done, cancelled ones become cancelled; their slots are freed.
    // Returns the tickets that finished (done or cancelled).
    std::vector<uint64_t> complete_round(const std::vector<Item> &items, double now) {
        for (const Item &it : items) {
            auto f = reqs_.find(it.ticket);
            if (f != reqs_.end()) f->second.completed += it.count;
        }
        std::vector<uint64_t> out;
        for (size_t i = 0; i < running_.size();) {
            Request &r = reqs_.at(running_[i]);
            const bool finished = r.completed == r.n_rays;
            const bool cancelled = r.cancel && r.completed == r.scheduled;
            if (finished || cancelled) {
                r.state = finished && !r.cancel ? kDone : kCanceled;
                r.t_done = now;
                free_slots_.push_back(r.slot);
                out.push_back(r.ticket);
                running_.erase(running_.begin() + (long)i);
            } else {
                ++i;
            }
        }
        return out;
    }

    // A running or queued request failed (e.g. its memory could not be
    // allocated); its slot and memory are returned at once.
    void fail(uint64_t ticket, int32_t status, double now) {
        auto f = reqs_.find(ticket);
        if (f == reqs_.end()) return;
        Request &r = f->second;
        if (r.state == kRunning) {
            free_slots_.push_back(r.slot);
            running_.erase(std::find(running_.begin(), running_.end(), ticket));
        } else if (r.state == kQueued) {
            queue_.erase(std::find(queue_.begin(), queue_.end(), ticket));
        } else {
            return;
        }
        if (r.holds_bytes) {
            used_ -= r.bytes;
            r.holds_bytes = false;
        }
        r.state = kFailed;
        r.status = status;
        r.t_done = now;
    }

    // Cancel: a queued request is cancelled at once; a running one stops
    // receiving rays and is cancelled when its rays in flight are done.
    // Returns false for an unknown or already finished request.
    bool cancel(uint64_t ticket, double now) {
        auto f = reqs_.find(ticket);
        if (f == reqs_.end()) return false;
        Request &r = f->second;
        if (r.state == kQueued) {
            queue_.erase(std::find(queue_.begin(), queue_.end(), ticket));
            r.state = kCanceled;
            r.t_done = now;
            return true;
        }
        if (r.state == kRunning) {
            r.cancel = true;
            return true;
        }
        return false;
    }

    // Release a finished request's memory and forget it.  Returns the bytes
    // freed, or -1 for an unknown or unfinished request.
    int64_t release(uint64_t ticket) {
        auto f = reqs_.find(ticket);
        if (f == reqs_.end()) return -1;
        Request &r = f->second;
        if (r.state != kDone && r.state != kFailed && r.state != kCanceled) return -1;
        const int64_t b = r.holds_bytes ? (int64_t)r.bytes : 0;
        if (r.holds_bytes) used_ -= r.bytes;
        reqs_.erase(f);
        return b;
    }

    const Request *find(uint64_t ticket) const {
        auto f = reqs_.find(ticket);
        return f == reqs_.end() ? nullptr : &f->second;
    }
    uint64_t used_bytes() const { return used_; }
    uint64_t budget() const { return budget_; }
    size_t queued() const { return queue_.size(); }
    size_t running() const { return running_.size(); }
    size_t free_slots() const { return free_slots_.size(); }

private:
    uint64_t budget_, used_ = 0, round_rays_;
    uint32_t chunk_;
    std::vector<int32_t> free_slots_;
    std::deque<uint64_t> queue_;
    std::vector<uint64_t> running_;
    std::map<uint64_t, Request> reqs_;
};

}  // namespace serve
}  // namespace mrt
