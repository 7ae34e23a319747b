// Serving runtime of libswmc: continuous batching of simulation requests.
//
// Lattice states live in one device pool of a fixed budget, carved by a
// first-fit allocator.  Every step admits waiting requests in arrival order
// while they fit (memory and slots), sweeps all active lattices together with
// the batched kernels (one launch per phase), and retires the lattices that
// reached their sweep count.  A lattice's chain does not depend on what else
// is in the batch: every draw is keyed by its own seed, site and sweep index.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "sw.h"
#include "sw_host.hpp"
#include "sw_internal.hpp"

using namespace swmc;
using namespace swmc::host;

namespace {

constexpr int kSweepLists[] = {kLBondPotts, kLBondClock, kLBlockMerge, kLBorderMerge, kLFlatten, kLFlip};
constexpr BatchKernel kKernelOf[kNumLists] = {kBKBondPotts, kBKBondClock, kBKBlockMerge, kBKBorderMerge,
                                              kBKFlatten,   kBKFlip,      kBKCounts,     kBKCountSum};

// First-fit allocator over [0, size) with coalescing of freed neighbours.
class PoolAllocator {
public:
    explicit PoolAllocator(uint64_t size) { free_[0] = size; }
    bool alloc(uint64_t n, uint64_t* off) {
        n = (n + kAlign - 1) / kAlign * kAlign;
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
        n = (n + kAlign - 1) / kAlign * kAlign;
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

private:
    uint64_t used_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

struct Pending {
    sw_request req;
};

struct Slot {
    bool used = false;
    sw_request req{};
    Layout lay{};
    uint64_t off = 0;
    SweepArgs args{};
    std::vector<uint32_t> table;
    int64_t done = 0;  // sweeps completed (the host knows: steps are deterministic)
    double t_admit = 0.0;
};

uint64_t mix64(uint64_t z) {
    // SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014).
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

struct sw_server {
    hipStream_t stream = nullptr;
    char* pool = nullptr;
    uint64_t budget = 0;
    PoolAllocator* alloc = nullptr;
    int max_slots = 0;
    int k = 1;
    int merge_tiles = kMergeTiles;
    bool sticky = false;
    std::chrono::steady_clock::time_point t0;
    std::deque<Pending> waiting;
    std::vector<Slot> slots;
    std::vector<sw_result> results;
    // launch lists of the active set
    char* meta = nullptr;
    uint64_t meta_entries = 0;  // capacity in 4-byte entries for all maps together
    SweepArgs* d_reps = nullptr;
    uint32_t* d_map[kNumLists] = {};
    uint32_t* d_begin[kNumLists] = {};
    uint32_t blocks[kNumLists] = {};
    std::vector<SweepArgs> h_reps;
    std::vector<uint32_t> h_map[kNumLists], h_begin[kNumLists];
    bool dirty = true;
    std::vector<int8_t> spins_host;
    sw_server_stats stats{};
};

namespace {

int sfail(sw_server* s, hipError_t e, const char* what) {
    if (s) s->sticky = true;
    return fail(SW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define SWS_HIP(s, call)                                        \
    do {                                                        \
        const hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return sfail(s, e_, #call);       \
    } while (0)

double now_s(const sw_server* s) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

int check_server(sw_server* s) {
    if (!s) return fail(SW_EINVAL, "null server");
    if (s->sticky) return fail(SW_ESTATE, "server had a device error earlier");
    return SW_OK;
}

int admit(sw_server* s) {
    while (!s->waiting.empty()) {
        int free_slot = -1;
        for (int i = 0; i < s->max_slots; ++i)
            if (!s->slots[static_cast<size_t>(i)].used) {
                free_slot = i;
                break;
            }
        if (free_slot < 0) return SW_OK;
        const sw_request& req = s->waiting.front().req;
        const Layout lay = layout_of(req.lattice);
        uint64_t off = 0;
        if (!s->alloc->alloc(lay.total, &off)) return SW_OK;  // the head waits for memory
        Slot& sl = s->slots[static_cast<size_t>(free_slot)];
        sl.used = true;
        sl.req = req;
        sl.lay = lay;
        sl.off = off;
        sl.done = 0;
        sl.t_admit = now_s(s);
        char* base = s->pool + off;
        sl.args = make_args(req.lattice, base, lay);
        sl.args.merge_tiles = s->merge_tiles;
        sl.table.resize(table_entries(req.lattice));
        build_table(req.lattice, sl.table.data());
        Control ctl = kFreshControl;
        ctl.target = static_cast<uint64_t>(req.sweeps);
        SWS_HIP(s, hipMemcpy(base + lay.ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice));
        SWS_HIP(s, hipMemcpyAsync(base + lay.table, sl.table.data(), sl.table.size() * 4, hipMemcpyHostToDevice,
                                  s->stream));
        SWS_HIP(s, launch_init(sl.args, s->stream));
        s->waiting.pop_front();
        s->stats.waiting -= 1;
        s->stats.active += 1;
        s->dirty = true;
    }
    return SW_OK;
}

// Rebuild the launch lists for the active lattices and upload them.
int rebuild(sw_server* s) {
    s->h_reps.clear();
    for (auto& sl : s->slots)
        if (sl.used) s->h_reps.push_back(sl.args);
    const size_t n = s->h_reps.size();
    uint64_t total = 0;
    for (int l = 0; l < kNumLists; ++l) {
        s->h_map[l].clear();
        s->h_begin[l].assign(n, 0u);
        if (l == kLCounts || l == kLCountSum) {  // retiring lattices are counted by the single-lattice launch
            s->blocks[l] = 0;
            total += n;
            continue;
        }
        for (size_t r = 0; r < n; ++r) {
            s->h_begin[l][r] = static_cast<uint32_t>(s->h_map[l].size());
            s->h_map[l].insert(s->h_map[l].end(), blocks_for(l, s->h_reps[r]), static_cast<uint32_t>(r));
        }
        s->blocks[l] = static_cast<uint32_t>(s->h_map[l].size());
        total += s->h_map[l].size() + n;
    }
    if (total > s->meta_entries) return fail(SW_ENOMEM, "launch lists need %llu entries, have %llu",
                                             static_cast<unsigned long long>(total),
                                             static_cast<unsigned long long>(s->meta_entries));
    char* m = s->meta;
    s->d_reps = reinterpret_cast<SweepArgs*>(m);
    m += up(static_cast<size_t>(s->max_slots) * sizeof(SweepArgs));
    if (n) SWS_HIP(s, hipMemcpyAsync(s->d_reps, s->h_reps.data(), n * sizeof(SweepArgs), hipMemcpyHostToDevice, s->stream));
    for (int l = 0; l < kNumLists; ++l) {
        s->d_map[l] = reinterpret_cast<uint32_t*>(m);
        m += s->h_map[l].size() * 4;
        s->d_begin[l] = reinterpret_cast<uint32_t*>(m);
        m += n * 4;
        if (!s->h_map[l].empty())
            SWS_HIP(s, hipMemcpyAsync(s->d_map[l], s->h_map[l].data(), s->h_map[l].size() * 4, hipMemcpyHostToDevice,
                                      s->stream));
        if (n) SWS_HIP(s, hipMemcpyAsync(s->d_begin[l], s->h_begin[l].data(), n * 4, hipMemcpyHostToDevice, s->stream));
    }
    s->dirty = false;
    return SW_OK;
}

int retire(sw_server* s, Slot& sl) {
    char* base = s->pool + sl.off;
    SweepArgs a = sl.args;
    a.count_row = reinterpret_cast<int64_t*>(base + sl.lay.scratch_row);
    SWS_HIP(s, launch_counts(a, s->stream));
    int64_t row[kRowWords];
    Control ctl;
    const size_t N = static_cast<size_t>(sl.req.lattice.L) * sl.req.lattice.L;
    s->spins_host.resize(N);
    SWS_HIP(s, hipStreamSynchronize(s->stream));
    SWS_HIP(s, hipMemcpy(row, a.count_row, sizeof row, hipMemcpyDeviceToHost));
    SWS_HIP(s, hipMemcpy(&ctl, base + sl.lay.ctl, sizeof ctl, hipMemcpyDeviceToHost));
    SWS_HIP(s, hipMemcpy(s->spins_host.data(), base + sl.lay.spins, N, hipMemcpyDeviceToHost));
    sw_result res{};
    res.tag = sl.req.tag;
    res.status = SW_OK;
    fill_obs(sl.req.lattice, row, ctl.t, Sums{}, &res.obs);
    uint64_t h = 0;
    for (size_t i = 0; i < N; ++i) h += mix64((static_cast<uint64_t>(i) << 8) | static_cast<uint8_t>(s->spins_host[i]));
    res.spin_hash = h;
    res.t_arrival = sl.req.t_arrival;
    res.t_admit = sl.t_admit;
    res.t_done = now_s(s);
    s->results.push_back(res);
    s->alloc->release(sl.off, sl.lay.total);
    s->stats.active -= 1;
    s->stats.completed += 1;
    s->stats.spin_updates += static_cast<int64_t>(N) * sl.req.sweeps;
    sl.used = false;
    s->dirty = true;
    return SW_OK;
}

}  // namespace

extern "C" {

int sw_server_create(uint64_t budget_bytes, int32_t max_slots, int32_t sweeps_per_step, void* stream,
                     sw_server** out) {
    if (!out) return fail(SW_EINVAL, "null output pointer");
    *out = nullptr;
    if (budget_bytes < (1u << 20)) return fail(SW_EINVAL, "budget must be at least 1 MiB");
    if (max_slots < 1 || max_slots > 65535) return fail(SW_EINVAL, "max_slots must be in [1, 65535]");
    if (sweeps_per_step < 1) return fail(SW_EINVAL, "sweeps_per_step must be >= 1");
    sw_server* s = new sw_server();
    s->stream = static_cast<hipStream_t>(stream);
    s->budget = budget_bytes;
    s->max_slots = max_slots;
    s->k = sweeps_per_step;
    s->t0 = std::chrono::steady_clock::now();
    s->slots.resize(static_cast<size_t>(max_slots));
    // Launch-list capacity: per lattice the sweep lists need at most about
    // N/600 + L/12 + 8 workgroup entries plus one begin entry per list
    // (N = L^2 sites, each holding at least 9 bytes of state).
    s->meta_entries = budget_bytes / 2048 + static_cast<uint64_t>(max_slots) * (46340 / 8 + 64);
    const uint64_t meta_bytes = up(static_cast<size_t>(max_slots) * sizeof(SweepArgs)) + s->meta_entries * 4;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, budget_bytes);
    if (e != hipSuccess) {
        delete s;
        return fail(SW_ENOMEM, "hipMalloc(%llu): %s", static_cast<unsigned long long>(budget_bytes),
                    hipGetErrorString(e));
    }
    s->pool = static_cast<char*>(p);
    e = hipMalloc(&p, meta_bytes);
    if (e != hipSuccess) {
        (void)hipFree(s->pool);
        delete s;
        return fail(SW_ENOMEM, "hipMalloc(%llu): %s", static_cast<unsigned long long>(meta_bytes), hipGetErrorString(e));
    }
    s->meta = static_cast<char*>(p);
    s->alloc = new PoolAllocator(budget_bytes);
    s->stats.budget_bytes = budget_bytes;
    *out = s;
    return SW_OK;
}

double sw_server_now(sw_server* s) { return s ? now_s(s) : 0.0; }

int sw_server_submit(sw_server* s, const sw_request* req) {
    int st = check_server(s);
    if (st) return st;
    if (!req) return fail(SW_EINVAL, "null request");
    std::string why;
    if (!lattice_ok(&req->lattice, &why)) return fail(SW_EINVAL, "%s", why.c_str());
    if (req->sweeps < 1) return fail(SW_EINVAL, "sweeps must be >= 1");
    s->stats.submitted += 1;
    const Layout lay = layout_of(req->lattice);
    if (lay.total > s->budget) {
        sw_result res{};
        res.tag = req->tag;
        res.status = SW_EBUDGET;
        res.t_arrival = req->t_arrival;
        res.t_admit = res.t_done = now_s(s);
        s->results.push_back(res);
        s->stats.rejected += 1;
        return SW_OK;
    }
    s->waiting.push_back(Pending{*req});
    s->stats.waiting += 1;
    return SW_OK;
}

int sw_server_step(sw_server* s, int32_t* active) {
    int st = check_server(s);
    if (st) return st;
    st = admit(s);
    if (st) return st;
    int32_t n_active = 0;
    for (auto& sl : s->slots) n_active += sl.used ? 1 : 0;
    if (active) *active = n_active;
    if (n_active == 0) return SW_OK;
    if (s->dirty) {
        st = rebuild(s);
        if (st) return st;
    }
    for (int sweep = 0; sweep < s->k; ++sweep)
        for (int l : kSweepLists) {
            if (s->blocks[l] == 0) continue;
            const BatchLaunch bl{s->d_reps, s->d_map[l], s->d_begin[l], s->blocks[l]};
            SWS_HIP(s, launch_batch(kKernelOf[l], bl, s->stream, 0));
        }
    SWS_HIP(s, hipStreamSynchronize(s->stream));
    s->stats.steps += 1;
    for (auto& sl : s->slots) {
        if (!sl.used) continue;
        sl.done += s->k;
        if (sl.done >= sl.req.sweeps) {
            st = retire(s, sl);
            if (st) return st;
        }
    }
    return SW_OK;
}

int sw_server_poll(sw_server* s, sw_result* out, int32_t cap, int32_t* n) {
    if (!s || !n || cap < 0 || (cap > 0 && !out)) return fail(SW_EINVAL, "bad arguments");
    const size_t k = s->results.size() < static_cast<size_t>(cap) ? s->results.size() : static_cast<size_t>(cap);
    for (size_t i = 0; i < k; ++i) out[i] = s->results[i];
    s->results.erase(s->results.begin(), s->results.begin() + static_cast<std::ptrdiff_t>(k));
    *n = static_cast<int32_t>(k);
    return SW_OK;
}

int sw_server_stats_read(sw_server* s, sw_server_stats* out) {
    if (!s || !out) return fail(SW_EINVAL, "bad arguments");
    *out = s->stats;
    out->used_bytes = s->alloc->used();
    return SW_OK;
}

void sw_server_destroy(sw_server* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    (void)hipFree(s->pool);
    (void)hipFree(s->meta);
    delete s->alloc;
    delete s;
}

}  // extern "C"
