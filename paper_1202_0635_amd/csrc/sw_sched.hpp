// Host-side scheduling of the request server: the device-memory pool, the
// slot table and the admission / step / retirement policy of continuous
// batching.  Nothing here touches a GPU: the device work is delegated to an
// executor (the HIP one in sw_server.cpp; a recording fake in the tests), so
// the policy can be checked on a CPU, under sanitizers.
#pragma once

#include <stdint.h>

#include <deque>
#include <iterator>
#include <map>
#include <vector>

#include "sw.h"

namespace swmc {
namespace sched {

constexpr uint64_t kPoolAlign = 256;

// First-fit allocator over [0, size) with coalescing of freed neighbours.
// Blocks are multiples of kPoolAlign, so every offset is kPoolAlign-aligned.
class PoolAllocator {
public:
    explicit PoolAllocator(uint64_t size) : size_(size / kPoolAlign * kPoolAlign) {
        if (size_) free_[0] = size_;
    }
    static uint64_t rounded(uint64_t n) { return (n + kPoolAlign - 1) / kPoolAlign * kPoolAlign; }
    bool alloc(uint64_t n, uint64_t* off) {
        n = rounded(n);
        if (n == 0) n = kPoolAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n;
                const uint64_t at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        n = rounded(n);
        if (n == 0) n = kPoolAlign;
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t used() const { return used_; }
    uint64_t size() const { return size_; }
    // Number of free extents (1 when nothing is allocated: everything coalesced).
    size_t extents() const { return free_.size(); }
    uint64_t largest_free() const {
        uint64_t m = 0;
        for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }

private:
    uint64_t size_ = 0;
    uint64_t used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

// One admitted lattice.
struct Slot {
    bool used = false;
    sw_request req{};
    uint64_t bytes = 0;  // its state's device bytes
    uint64_t off = 0;    // offset in the pool
    int64_t done = 0;    // sweeps completed (steps are deterministic, so the host knows)
    double t_admit = 0.0;
};

// The policy.  Exec must provide:
//   uint64_t bytes_of(const sw_request&)        device bytes of a request's state
//   double now()                                the server clock
//   int admit(int slot, const Slot&)            make the state at slot.off (random start)
//   int run(int sweeps)                         that many sweeps over the used slots
//                                                 (a lattice stops at its sweep count)
//   int retire(int slot, const Slot&)           final results; the memory is free after it
//   void reject(const sw_request&)              a request that can never fit
//   int end_step()                              the step's device work is enqueued
//   int drain()                                 nothing is active: finish outstanding work
// and may read slots() / active list through the core.  All int returns are
// sw_status codes; the first error is passed through.
template <class Exec>
class ServerCore {
public:
    ServerCore(uint64_t budget, int max_slots, int sweeps_per_step, Exec* ex)
        : pool_(budget), slots_(static_cast<size_t>(max_slots)), k_(sweeps_per_step), ex_(ex) {}

    // Queue a request; one larger than the whole pool is rejected at once.
    void submit(const sw_request& r) {
        stats_.submitted += 1;
        if (ex_->bytes_of(r) > pool_.size()) {
            stats_.rejected += 1;
            ex_->reject(r);
            return;
        }
        waiting_.push_back(r);
        stats_.waiting += 1;
    }

    // Admit, run one step of k sweeps, retire the lattices that reached their
    // sweep count.  *active = lattices that ran.
    int step(int32_t* active) {
        int st = admit();
        if (st) return st;
        int32_t n = 0;
        for (const Slot& sl : slots_) n += sl.used ? 1 : 0;
        if (active) *active = n;
        if (n == 0) return ex_->drain();
        st = ex_->run(k_);
        if (st) return st;
        stats_.steps += 1;
        for (size_t i = 0; i < slots_.size(); ++i) {
            Slot& sl = slots_[i];
            if (!sl.used) continue;
            sl.done += k_;
            if (sl.done < sl.req.sweeps) continue;
            st = ex_->retire(static_cast<int>(i), sl);
            if (st) return st;
            pool_.release(sl.off, sl.bytes);
            stats_.active -= 1;
            stats_.completed += 1;
            stats_.spin_updates += static_cast<int64_t>(sl.req.lattice.L) * sl.req.lattice.L * sl.req.sweeps;
            sl.used = false;
            changed_ = true;
        }
        return ex_->end_step();
    }

    const std::vector<Slot>& slots() const { return slots_; }
    // The active set changed since the last call (admissions or retirements).
    bool take_changed() {
        const bool c = changed_;
        changed_ = false;
        return c;
    }
    sw_server_stats stats() const {
        sw_server_stats s = stats_;
        s.budget_bytes = pool_.size();
        s.used_bytes = pool_.used();
        return s;
    }
    const PoolAllocator& pool() const { return pool_; }
    size_t waiting() const { return waiting_.size(); }

private:
    // Arrival order: the head waits while it does not fit (memory or slot),
    // and nothing behind it overtakes it.
    int admit() {
        while (!waiting_.empty()) {
            int free_slot = -1;
            for (size_t i = 0; i < slots_.size(); ++i)
                if (!slots_[i].used) {
                    free_slot = static_cast<int>(i);
                    break;
                }
            if (free_slot < 0) return SW_OK;
            const sw_request& req = waiting_.front();
            const uint64_t bytes = ex_->bytes_of(req);
            uint64_t off = 0;
            if (!pool_.alloc(bytes, &off)) return SW_OK;
            Slot& sl = slots_[static_cast<size_t>(free_slot)];
            sl.used = true;
            sl.req = req;
            sl.bytes = bytes;
            sl.off = off;
            sl.done = 0;
            sl.t_admit = ex_->now();
            waiting_.pop_front();
            stats_.waiting -= 1;
            stats_.active += 1;
            changed_ = true;
            const int st = ex_->admit(free_slot, sl);
            if (st) return st;
        }
        return SW_OK;
    }

    PoolAllocator pool_;
    std::vector<Slot> slots_;
    std::deque<sw_request> waiting_;
    int k_;
    Exec* ex_;
    bool changed_ = true;
    sw_server_stats stats_{};
};

}  // namespace sched
}  // namespace swmc
