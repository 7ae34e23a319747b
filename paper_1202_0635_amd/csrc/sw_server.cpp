// Serving runtime of libswmc: continuous batching of simulation requests.
//
// Lattice states live in one device pool of a fixed budget, carved by a
// first-fit allocator.  Every step admits waiting requests in arrival order
// while they fit (memory and slots), sweeps all active lattices together with
// the batched kernels (one launch per phase), and retires the lattices that
// reached their sweep count.  A lattice's chain does not depend on what else
// is in the batch: every draw is keyed by its own seed, site and sweep index.
//
// The policy (pool, slots, admission order, retirement) is the host-only
// ServerCore of sw_sched.hpp; this file is its HIP executor.  The device never
// waits for the host: a step's launches are enqueued, then the host waits for
// the previous step only (two steps in flight), and a retiring lattice's
// results (count row, device-computed state hash, control block) come back by
// small asynchronous copies into pinned memory, read once that step's event
// has completed.  Host-to-device staging (control blocks, cutoff tables,
// launch lists) is double-buffered by step parity, so no buffer is rewritten
// while a copy from it may still be pending.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "sw.h"
#include "sw_host.hpp"
#include "sw_internal.hpp"
#include "sw_sched.hpp"

using namespace swmc;
using namespace swmc::host;

namespace {

constexpr int kSweepLists[] = {kLBondPotts, kLBondClock, kLBlockMerge, kLBorderMerge, kLFlatten, kLFlip};
// The server keeps no canonical labels: the flatten leaves root copies.
constexpr BatchKernel kKernelOf[kNumLists] = {kBKBondPotts, kBKBondClock, kBKBlockMerge, kBKBorderMerge,
                                              kBKFlattenCopies, kBKFlip, kBKCounts, kBKCountSum,
                                              kBKHash, kBKHashSum};

// Results of one retiring lattice, copied back from the device.
struct Staging {
    int64_t row[kRowWords];
    uint64_t hash[2];
    Control ctl;
};

struct Retiring {
    int staging;
    sw_request req;
    double t_admit;
};

struct HipExec;

}  // namespace

struct sw_server {
    hipStream_t stream = nullptr;
    char* pool = nullptr;
    char* meta = nullptr;
    uint64_t meta_entries = 0;  // capacity in 4-byte entries for all maps together
    int max_slots = 0;
    int merge_tiles = kMergeTiles;
    bool sticky = false;
    std::chrono::steady_clock::time_point t0;
    std::vector<sw_result> results;
    HipExec* ex = nullptr;
    sched::ServerCore<HipExec>* core = nullptr;
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

struct HipExec {
    sw_server* s = nullptr;
    int parity = 0;  // step parity: which half of the host-to-device staging this step writes
    // per slot: kernel arguments; per (parity, slot): control block and cutoff table staging
    std::vector<SweepArgs> args;
    std::vector<Control> ctl_stage[2];
    std::vector<std::vector<uint32_t>> table_stage[2];
    // launch lists of the active set, host side per parity
    std::vector<SweepArgs> h_reps[2];
    std::vector<uint32_t> h_map[2][kNumLists], h_begin[2][kNumLists];
    SweepArgs* d_reps = nullptr;
    uint32_t* d_map[kNumLists] = {};
    uint32_t* d_begin[kNumLists] = {};
    uint32_t blocks[kNumLists] = {};
    // device-to-host results: pinned staging entries and the retirements of
    // the step in flight (cur) and of the step before it (prev)
    Staging* stage = nullptr;
    std::vector<int> free_stage;
    std::vector<Retiring> cur, prev;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool prev_pending = false;

    uint64_t bytes_of(const sw_request& r) const { return layout_of(r.lattice).total; }
    double now() const { return now_s(s); }

    int admit(int slot, const sched::Slot& sl) {
        const size_t i = static_cast<size_t>(slot);
        char* base = s->pool + sl.off;
        const Layout lay = layout_of(sl.req.lattice);
        SweepArgs a = make_args(sl.req.lattice, base, lay);
        a.merge_tiles = s->merge_tiles;
        a.count_row = reinterpret_cast<int64_t*>(base + lay.scratch_row);
        args[i] = a;
        std::vector<uint32_t>& tab = table_stage[parity][i];
        tab.resize(table_entries(sl.req.lattice));
        build_table(sl.req.lattice, tab.data());
        Control& ctl = ctl_stage[parity][i];
        ctl = kFreshControl;
        ctl.target = static_cast<uint64_t>(sl.req.sweeps);
        SWS_HIP(s, hipMemcpyAsync(base + lay.ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, s->stream));
        SWS_HIP(s, hipMemcpyAsync(base + lay.table, tab.data(), tab.size() * 4, hipMemcpyHostToDevice, s->stream));
        SWS_HIP(s, launch_init(a, s->stream));
        return SW_OK;
    }

    // Launch lists for the used slots (written to this step's parity half).
    int rebuild() {
        const auto& slots = s->core->slots();
        std::vector<SweepArgs>& reps = h_reps[parity];
        reps.clear();
        for (size_t i = 0; i < slots.size(); ++i)
            if (slots[i].used) reps.push_back(args[i]);
        const size_t n = reps.size();
        uint64_t total = 0;
        for (int l = 0; l < kNumLists; ++l) {
            auto& map = h_map[parity][l];
            auto& begin = h_begin[parity][l];
            map.clear();
            begin.assign(n, 0u);
            const bool sweep_list = l != kLCounts && l != kLCountSum && l != kLHash && l != kLHashSum;
            for (size_t r = 0; r < n && sweep_list; ++r) {
                begin[r] = static_cast<uint32_t>(map.size());
                map.insert(map.end(), blocks_for(l, reps[r]), static_cast<uint32_t>(r));
            }
            blocks[l] = static_cast<uint32_t>(map.size());
            total += map.size() + n;
        }
        if (total > s->meta_entries)
            return fail(SW_ENOMEM, "launch lists need %llu entries, have %llu", static_cast<unsigned long long>(total),
                        static_cast<unsigned long long>(s->meta_entries));
        char* m = s->meta;
        d_reps = reinterpret_cast<SweepArgs*>(m);
        m += up(static_cast<size_t>(s->max_slots) * sizeof(SweepArgs));
        if (n) SWS_HIP(s, hipMemcpyAsync(d_reps, reps.data(), n * sizeof(SweepArgs), hipMemcpyHostToDevice, s->stream));
        for (int l = 0; l < kNumLists; ++l) {
            auto& map = h_map[parity][l];
            auto& begin = h_begin[parity][l];
            d_map[l] = reinterpret_cast<uint32_t*>(m);
            m += map.size() * 4;
            d_begin[l] = reinterpret_cast<uint32_t*>(m);
            m += n * 4;
            if (!map.empty())
                SWS_HIP(s, hipMemcpyAsync(d_map[l], map.data(), map.size() * 4, hipMemcpyHostToDevice, s->stream));
            if (n) SWS_HIP(s, hipMemcpyAsync(d_begin[l], begin.data(), n * 4, hipMemcpyHostToDevice, s->stream));
        }
        return SW_OK;
    }

    int run(int sweeps) {
        if (s->core->take_changed()) {
            const int st = rebuild();
            if (st) return st;
        }
        for (int sweep = 0; sweep < sweeps; ++sweep)
            for (int l : kSweepLists) {
                if (blocks[l] == 0) continue;
                const BatchLaunch bl{d_reps, d_map[l], d_begin[l], blocks[l], kWaves};
                SWS_HIP(s, launch_batch(kKernelOf[l], bl, s->stream, 0));
            }
        return SW_OK;
    }

    // Final counts and the spin hash of the state, computed on the device and
    // copied into a pinned staging entry with the control block.
    int retire(int slot, const sched::Slot& sl) {
        const SweepArgs& a = args[static_cast<size_t>(slot)];
        if (free_stage.empty()) return fail(SW_ESTATE, "no free result staging entry");
        const int k = free_stage.back();
        free_stage.pop_back();
        Staging* st = stage + k;
        const uint32_t N = static_cast<uint32_t>(a.L) * static_cast<uint32_t>(a.L);
        SWS_HIP(s, launch_counts(a, s->stream));
        SWS_HIP(s, launch_hash_state(a.spins, nullptr, N, a.hash_partial, s->stream));
        SWS_HIP(s, hipMemcpyAsync(st->row, a.count_row, sizeof st->row, hipMemcpyDeviceToHost, s->stream));
        SWS_HIP(s, hipMemcpyAsync(st->hash, a.hash_partial + 2 * static_cast<size_t>(hash_state_blocks(N)), sizeof st->hash,
                                  hipMemcpyDeviceToHost, s->stream));
        SWS_HIP(s, hipMemcpyAsync(&st->ctl, a.ctl, sizeof st->ctl, hipMemcpyDeviceToHost, s->stream));
        cur.push_back({k, sl.req, sl.t_admit});
        return SW_OK;
    }

    void reject(const sw_request& r) {
        sw_result res{};
        res.tag = r.tag;
        res.status = SW_EBUDGET;
        res.t_arrival = r.t_arrival;
        res.t_admit = res.t_done = now();
        s->results.push_back(res);
    }

    // Results of a completed step.
    int finalize(std::vector<Retiring>& done) {
        for (const Retiring& r : done) {
            const Staging* st = stage + r.staging;
            const int fs = fault_status(st->ctl.fault);
            if (fs) {
                s->sticky = true;
                return fs;
            }
            sw_result res{};
            res.tag = r.req.tag;
            res.status = SW_OK;
            fill_obs(r.req.lattice, st->row, st->ctl.t, Sums{}, &res.obs);
            res.obs.hash_spins = st->hash[0];
            res.spin_hash = st->hash[0];
            res.t_arrival = r.req.t_arrival;
            res.t_admit = r.t_admit;
            res.t_done = now();
            s->results.push_back(res);
            free_stage.push_back(r.staging);
        }
        done.clear();
        return SW_OK;
    }

    // The step is enqueued: mark it, then wait for the step before it.
    int end_step() {
        SWS_HIP(s, hipEventRecord(ev[parity], s->stream));
        if (prev_pending) {
            SWS_HIP(s, hipEventSynchronize(ev[parity ^ 1]));
            const int st = finalize(prev);
            if (st) return st;
        }
        prev.swap(cur);
        prev_pending = true;
        parity ^= 1;
        return SW_OK;
    }

    int drain() {
        if (!prev_pending) return SW_OK;
        SWS_HIP(s, hipEventSynchronize(ev[parity ^ 1]));
        prev_pending = false;
        return finalize(prev);
    }
};

int check_server(sw_server* s) {
    if (!s) return fail(SW_EINVAL, "null server");
    if (s->sticky) return fail(SW_ESTATE, "server had a device error earlier");
    return SW_OK;
}

void destroy(sw_server* s) {
    if (s->stream || s->pool) (void)hipStreamSynchronize(s->stream);
    if (s->ex) {
        for (hipEvent_t e : s->ex->ev)
            if (e) (void)hipEventDestroy(e);
        if (s->ex->stage) (void)hipHostFree(s->ex->stage);
    }
    if (s->pool) (void)hipFree(s->pool);
    if (s->meta) (void)hipFree(s->meta);
    delete s->core;
    delete s->ex;
    delete s;
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
    s->max_slots = max_slots;
    s->t0 = std::chrono::steady_clock::now();
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
        destroy(s);
        return fail(SW_ENOMEM, "hipMalloc(%llu): %s", static_cast<unsigned long long>(meta_bytes), hipGetErrorString(e));
    }
    s->meta = static_cast<char*>(p);
    HipExec* ex = new HipExec();
    s->ex = ex;
    ex->s = s;
    ex->args.resize(static_cast<size_t>(max_slots));
    for (int par = 0; par < 2; ++par) {
        ex->ctl_stage[par].resize(static_cast<size_t>(max_slots));
        ex->table_stage[par].resize(static_cast<size_t>(max_slots));
    }
    // result staging: at most max_slots retirements in each of two steps in flight
    const size_t nstage = 2 * static_cast<size_t>(max_slots);
    e = hipHostMalloc(reinterpret_cast<void**>(&ex->stage), nstage * sizeof(Staging), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ex->ev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ex->ev[1], hipEventDisableTiming);
    if (e != hipSuccess) {
        destroy(s);
        return fail(SW_EDEVICE, "sw_server_create: %s", hipGetErrorString(e));
    }
    for (size_t k = nstage; k-- > 0;) ex->free_stage.push_back(static_cast<int>(k));
    s->core = new sched::ServerCore<HipExec>(budget_bytes, max_slots, sweeps_per_step, ex);
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
    s->core->submit(*req);
    return SW_OK;
}

int sw_server_step(sw_server* s, int32_t* active) {
    const int st = check_server(s);
    if (st) return st;
    return s->core->step(active);
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
    *out = s->core->stats();
    return SW_OK;
}

void sw_server_destroy(sw_server* s) {
    if (!s) return;
    destroy(s);
}

}  // extern "C"
