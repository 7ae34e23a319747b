// Batched runtime of libswmc: many independent lattices (replicas of uneven
// L, q, model and T) swept together.  Each phase of a sweep is one launch over
// the workgroups of every replica (a per-launch map sends workgroup b to its
// replica), and a sweep's launches are captured once in a hipGraph that is
// replayed for every further sweep.  Results per replica are identical to the
// single-lattice path: every draw is keyed by the replica's own seed, site and
// sweep index.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "sw.h"
#include "sw_host.hpp"
#include "sw_internal.hpp"

using namespace swmc;
using namespace swmc::host;

namespace {

constexpr int kSchedules[] = {1, 2, 4};  // first-level merge block sizes the tuner tries
constexpr int kTileWavesChoices[] = {kWaves, kWavesSmall};
// A call of n sweeps replays one graph that holds min(n, kMaxGraphSweeps)
// sweeps (and one for the remainder); the last kGraphCache sizes are kept.
constexpr int32_t kMaxGraphSweeps = 512;
constexpr size_t kGraphCache = 4;

constexpr BatchKernel kListKernel[kNumLists] = {kBKBondPotts, kBKBondClock, kBKBlockMerge, kBKBorderMerge,
                                                kBKFlatten,   kBKFlip,      kBKCounts,     kBKCountSum,
                                                kBKHash,      kBKHashSum};

struct Replica {
    sw_lattice p{};
    Layout lay{};
    size_t offset = 0;
    SweepArgs args{};
    std::vector<uint32_t> table;
    Sums sums;  // running sums over measured sweeps
    bool have_canon = false;
    std::vector<HashRecord> hashes;  // per-sweep hashes (SW_HASH) not yet read
};

}  // namespace

struct sw_batch {
    std::vector<Replica> reps;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    bool owns = false;
    bool sticky = false;
    int merge_tiles = kMergeTiles;
    int tile_waves = kWaves;  // waves per tile of the batched bond kernels
    std::string arch;         // gcnArchName of the device, for the autotuner cache
    size_t meta_off = 0;
    SweepArgs* d_reps = nullptr;
    uint32_t* d_map[kNumLists] = {};
    uint32_t* d_begin[kNumLists] = {};
    uint32_t blocks[kNumLists] = {};
    std::vector<SweepArgs> h_reps;
    std::vector<uint32_t> h_map[kNumLists], h_begin[kNumLists];
    // captured runs of k sweeps (k -> instantiated graph), at most kGraphCache of them
    std::vector<std::pair<int32_t, hipGraphExec_t>> execs;
    hipStream_t cap_stream = nullptr;  // private stream the sweeps are captured on
    std::vector<int64_t> ring_host;
    // per-launch timing (SW_PROFILE): event pairs per list
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> free_events;
    int64_t prof_launches[kNumLists] = {};
    double prof_ms[kNumLists] = {};
};

namespace {

const char* const kListNames[kNumLists] = {"kb_bond_local<potts>", "kb_bond_local<clock>", "kb_block_merge",
                                           "kb_border_merge",      "kb_flatten",           "kb_flip",
                                           "kb_counts",            "kb_count_sum",         "kb_hash",
                                           "kb_hash_sum"};

int bfail(sw_batch* b, hipError_t e, const char* what) {
    if (b) b->sticky = true;
    return fail(SW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define SWB_HIP(b, call)                                        \
    do {                                                        \
        const hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return bfail(b, e_, #call);       \
    } while (0)

// Metadata bytes for the largest lists any schedule can need.
size_t meta_bytes(const std::vector<sw_lattice>& ps) {
    const size_t n = ps.size();
    size_t total = up(n * sizeof(SweepArgs));
    for (int l = 0; l < kNumLists; ++l) {
        uint64_t worst = 0;
        for (int mt : kSchedules) {
            uint64_t s = 0;
            for (const sw_lattice& p : ps) {
                SweepArgs a = make_args(p, nullptr, Layout{});
                a.merge_tiles = mt;
                s += blocks_for(l, a);
            }
            if (s > worst) worst = s;
        }
        total += up(worst * 4) + up(n * 4);
    }
    return total;
}

bool batch_params_ok(const sw_lattice* ps, int32_t n, std::string* why) {
    if (!ps || n <= 0) return *why = "need at least one lattice", false;
    if (n > 65535) return *why = "at most 65535 replicas", false;
    for (int32_t r = 0; r < n; ++r)
        if (!lattice_ok(&ps[r], why)) {
            *why = "replica " + std::to_string(r) + ": " + *why;
            return false;
        }
    return true;
}

size_t arena_bytes(const sw_lattice* ps, int32_t n, size_t* meta_off) {
    size_t o = 0;
    for (int32_t r = 0; r < n; ++r) o += layout_of(ps[r]).total;
    if (meta_off) *meta_off = o;
    std::vector<sw_lattice> v(ps, ps + n);
    return o + meta_bytes(v);
}

void drop_graphs(sw_batch* b) {
    for (auto& g : b->execs) (void)hipGraphExecDestroy(g.second);
    b->execs.clear();
}

// (Re)build the per-launch maps for the current schedule and upload them.
int upload_lists(sw_batch* b) {
    const size_t n = b->reps.size();
    b->h_reps.resize(n);
    for (size_t r = 0; r < n; ++r) {
        b->reps[r].args.merge_tiles = b->merge_tiles;
        b->h_reps[r] = b->reps[r].args;
    }
    char* m = b->base + b->meta_off;
    b->d_reps = reinterpret_cast<SweepArgs*>(m);
    m += up(n * sizeof(SweepArgs));
    std::vector<sw_lattice> ps;
    for (auto& rp : b->reps) ps.push_back(rp.p);
    for (int l = 0; l < kNumLists; ++l) {
        auto& map = b->h_map[l];
        auto& begin = b->h_begin[l];
        map.clear();
        begin.assign(n, 0u);
        for (size_t r = 0; r < n; ++r) {
            begin[r] = static_cast<uint32_t>(map.size());
            const uint32_t nb = blocks_for(l, b->h_reps[r]);
            map.insert(map.end(), nb, static_cast<uint32_t>(r));
        }
        b->blocks[l] = static_cast<uint32_t>(map.size());
        uint64_t worst = 0;
        for (int mt : kSchedules) {
            uint64_t s = 0;
            for (const sw_lattice& p : ps) {
                SweepArgs a = make_args(p, nullptr, Layout{});
                a.merge_tiles = mt;
                s += blocks_for(l, a);
            }
            if (s > worst) worst = s;
        }
        b->d_map[l] = reinterpret_cast<uint32_t*>(m);
        m += up(worst * 4);
        b->d_begin[l] = reinterpret_cast<uint32_t*>(m);
        m += up(n * 4);
        if (!map.empty())
            SWB_HIP(b, hipMemcpyAsync(b->d_map[l], map.data(), map.size() * 4, hipMemcpyHostToDevice, b->stream));
        SWB_HIP(b, hipMemcpyAsync(b->d_begin[l], begin.data(), n * 4, hipMemcpyHostToDevice, b->stream));
    }
    SWB_HIP(b, hipMemcpyAsync(b->d_reps, b->h_reps.data(), n * sizeof(SweepArgs), hipMemcpyHostToDevice, b->stream));
    SWB_HIP(b, hipStreamSynchronize(b->stream));  // host vectors may change after return
    drop_graphs(b);
    return SW_OK;
}

hipEvent_t take_event(sw_batch* b) {
    if (!b->free_events.empty()) {
        hipEvent_t e = b->free_events.back();
        b->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int launch_list(sw_batch* b, int l, bool profile, uint32_t row = 0, bool verify = false) {
    if (b->blocks[l] == 0) return SW_OK;
    BatchKernel k = kListKernel[l];
    if (l == kLFlip && verify) k = kBKFlipVerify;
    // only the flip reads the labels of a sweep without canonical labels
    if (l == kLFlatten && !verify) k = kBKFlattenCopies;
    const BatchLaunch bl{b->d_reps, b->d_map[l], b->d_begin[l], b->blocks[l], b->tile_waves};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (profile) {
        e0 = take_event(b);
        e1 = take_event(b);
        if (!e0 || !e1) return bfail(b, hipErrorOutOfMemory, "hipEventCreate");
        SWB_HIP(b, hipEventRecord(e0, b->stream));
    }
    SWB_HIP(b, launch_batch(k, bl, b->stream, row));
    if (profile) {
        SWB_HIP(b, hipEventRecord(e1, b->stream));
        b->pending.push_back({l, {e0, e1}});
    }
    return SW_OK;
}

// One sweep of every replica; hash_row >= 0 adds the state hashes of the
// sweep (after the border merge, before the flatten) into that ring row.
int enqueue_sweep(sw_batch* b, bool profile, bool verify, int hash_row = -1) {
    for (int l : {kLBondPotts, kLBondClock, kLBlockMerge, kLBorderMerge, kLFlatten, kLFlip}) {
        if (l == kLFlatten && hash_row >= 0) {
            int st = launch_list(b, kLHash, profile);
            if (!st) st = launch_list(b, kLHashSum, profile, static_cast<uint32_t>(hash_row));
            if (st) return st;
        }
        const int st = launch_list(b, l, profile, 0, verify);
        if (st) return st;
    }
    return SW_OK;
}

// Move hash ring rows [0, rows) of every replica to the host.
int flush_hashes(sw_batch* b, int rows) {
    if (rows <= 0) return SW_OK;
    SWB_HIP(b, hipStreamSynchronize(b->stream));
    std::vector<uint64_t> buf(2 * static_cast<size_t>(rows));
    for (auto& rp : b->reps) {
        Control ctl;
        SWB_HIP(b, hipMemcpy(&ctl, b->base + rp.offset + rp.lay.ctl, sizeof ctl, hipMemcpyDeviceToHost));
        const int st = fault_status(ctl.fault);
        if (st) {
            b->sticky = true;
            return st;
        }
        SWB_HIP(b, hipMemcpy(buf.data(), b->base + rp.offset + rp.lay.hash_ring, buf.size() * 8, hipMemcpyDeviceToHost));
        for (int r = 0; r < rows; ++r)
            rp.hashes.push_back({ctl.t - static_cast<uint64_t>(rows - 1 - r), buf[2 * r], buf[2 * r + 1]});
    }
    return SW_OK;
}

// The instantiated graph of k sweeps' launches, captured on first use (on a
// private stream: the caller's may be the null stream, which cannot be
// captured) and replayed on the caller's stream.  The sweep index lives in
// each replica's control block, so every captured sweep advances the chains.
int graph_of(sw_batch* b, int32_t k, hipGraphExec_t* out) {
    for (auto& g : b->execs)
        if (g.first == k) {
            *out = g.second;
            return SW_OK;
        }
    if (!b->cap_stream) SWB_HIP(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    hipStream_t user = b->stream;
    b->stream = b->cap_stream;
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    int st = SW_OK;
    for (int32_t s = 0; e == hipSuccess && s < k && !st; ++s) st = enqueue_sweep(b, false, false);
    hipGraph_t g = nullptr;
    const hipError_t e2 = (e == hipSuccess) ? hipStreamEndCapture(b->cap_stream, &g) : hipSuccess;
    b->stream = user;
    if (e != hipSuccess) return bfail(b, e, "hipStreamBeginCapture");
    if (st || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st ? st : bfail(b, e2, "hipStreamEndCapture");
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) return bfail(b, e3, "hipGraphInstantiate");
    if (b->execs.size() >= kGraphCache) {
        (void)hipGraphExecDestroy(b->execs.front().second);
        b->execs.erase(b->execs.begin());
    }
    b->execs.push_back({k, exec});
    *out = exec;
    return SW_OK;
}

int flush_rings(sw_batch* b, int rows) {
    if (rows <= 0) return SW_OK;
    SWB_HIP(b, hipStreamSynchronize(b->stream));
    b->ring_host.resize(static_cast<size_t>(rows) * kRowWords);
    for (auto& rp : b->reps) {
        SWB_HIP(b, hipMemcpy(b->ring_host.data(), b->base + rp.offset + rp.lay.ring, b->ring_host.size() * 8,
                             hipMemcpyDeviceToHost));
        for (int r = 0; r < rows; ++r) {
            rp.sums.add(observables_of(rp.p, b->ring_host.data() + static_cast<size_t>(r) * kRowWords));
        }
    }
    return SW_OK;
}

int check_batch(sw_batch* b) {
    if (!b) return fail(SW_EINVAL, "null batch");
    if (b->sticky) return fail(SW_ESTATE, "batch had a device error earlier");
    return SW_OK;
}

int check_replica(sw_batch* b, int32_t r) {
    const int st = check_batch(b);
    if (st) return st;
    if (r < 0 || static_cast<size_t>(r) >= b->reps.size()) return fail(SW_EINVAL, "replica %d out of range", r);
    return SW_OK;
}

}  // namespace

extern "C" {

size_t sw_batch_bytes(const sw_lattice* ps, int32_t n) {
    std::string why;
    if (!batch_params_ok(ps, n, &why)) {
        fail(SW_EINVAL, "%s", why.c_str());
        return 0;
    }
    return arena_bytes(ps, n, nullptr);
}

int sw_batch_init(const sw_lattice* ps, int32_t n, void* dev_mem, size_t bytes, void* stream, sw_batch** out) {
    if (!out) return fail(SW_EINVAL, "null output pointer");
    *out = nullptr;
    std::string why;
    if (!batch_params_ok(ps, n, &why)) return fail(SW_EINVAL, "%s", why.c_str());
    size_t meta_off = 0;
    const size_t total = arena_bytes(ps, n, &meta_off);
    if (dev_mem) {
        if (reinterpret_cast<uintptr_t>(dev_mem) % kAlign != 0) return fail(SW_EINVAL, "dev_mem must be 256-byte aligned");
        if (bytes < total) return fail(SW_ENOMEM, "dev_mem has %zu bytes, need %zu", bytes, total);
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SW_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fail(SW_EDEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SW_EDEVICE, "libswmc is built for gfx950; device %d is %s", dev, prop.gcnArchName);

    sw_batch* b = new sw_batch();
    b->stream = static_cast<hipStream_t>(stream);
    b->arch = std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':'));
    b->meta_off = meta_off;
    if (dev_mem) {
        b->base = static_cast<char*>(dev_mem);
    } else {
        void* m = nullptr;
        e = hipMalloc(&m, total);
        if (e != hipSuccess) {
            delete b;
            return fail(SW_ENOMEM, "hipMalloc(%zu): %s", total, hipGetErrorString(e));
        }
        b->base = static_cast<char*>(m);
        b->owns = true;
    }
    auto cleanup = [&](int st) {
        if (b->owns) (void)hipFree(b->base);
        delete b;
        return st;
    };
    b->reps.resize(static_cast<size_t>(n));
    size_t off = 0;
    for (int32_t r = 0; r < n; ++r) {
        Replica& rp = b->reps[static_cast<size_t>(r)];
        rp.p = ps[r];
        rp.lay = layout_of(ps[r]);
        rp.offset = off;
        off += rp.lay.total;
        char* rb = b->base + rp.offset;
        rp.args = make_args(ps[r], rb, rp.lay);
        rp.args.count_row = reinterpret_cast<int64_t*>(rb + rp.lay.ring);
        rp.table.resize(table_entries(ps[r]));
        build_table(ps[r], rp.table.data());
        e = hipMemcpyAsync(rb + rp.lay.ctl, &kFreshControl, sizeof(Control), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(rb + rp.lay.table, rp.table.data(), rp.table.size() * 4, hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = launch_init(rp.args, b->stream);
        if (e != hipSuccess) return cleanup(fail(SW_EDEVICE, "sw_batch_init: %s", hipGetErrorString(e)));
    }
    int st = upload_lists(b);
    if (st) return cleanup(st);
    *out = b;
    return SW_OK;
}

int sw_batch_set_schedule(sw_batch* b, int32_t merge_tiles) {
    const int st = check_batch(b);
    if (st) return st;
    bool ok = false;
    for (int mt : kSchedules) ok = ok || (mt == merge_tiles);
    if (!ok) return fail(SW_EINVAL, "merge_tiles must be 1, 2 or 4");
    if (merge_tiles == b->merge_tiles) return SW_OK;
    b->merge_tiles = merge_tiles;
    return upload_lists(b);
}

int sw_batch_set_tile_waves(sw_batch* b, int32_t waves) {
    const int st = check_batch(b);
    if (st) return st;
    if (waves != kWaves && waves != kWavesSmall) return fail(SW_EINVAL, "waves per tile must be 4 or 8");
    if (waves == b->tile_waves) return SW_OK;
    b->tile_waves = waves;
    drop_graphs(b);  // the captured launches name the bond kernel
    return SW_OK;
}

int sw_batch_sweep(sw_batch* b, int32_t nsweeps, uint32_t flags) {
    int st = check_batch(b);
    if (st) return st;
    if (nsweeps < 0) return fail(SW_EINVAL, "nsweeps must be >= 0");
    if (flags & ~(SW_MEASURE | SW_VERIFY | SW_PROFILE | SW_NO_GRAPH | SW_HASH))
        return fail(SW_EINVAL, "unknown flag bits");
    const bool measure = flags & SW_MEASURE;
    const bool profile = flags & SW_PROFILE;
    const bool verify = flags & SW_VERIFY;
    const bool hash = flags & SW_HASH;
    if (!measure && !profile && !hash && !(flags & SW_NO_GRAPH)) {
        // replay the captured sweep; a verify sweep (the last one) runs uncaptured
        const int32_t plain = verify ? nsweeps - 1 : nsweeps;
        // runs of up to kMaxGraphSweeps sweeps, each one graph launch
        for (int32_t done = 0; done < plain;) {
            const int32_t k = (plain - done < kMaxGraphSweeps) ? plain - done : kMaxGraphSweeps;
            hipGraphExec_t exec = nullptr;
            st = graph_of(b, k, &exec);
            if (st) return st;
            SWB_HIP(b, hipGraphLaunch(exec, b->stream));
            done += k;
        }
        if (verify && nsweeps > 0) {
            st = enqueue_sweep(b, false, true);
            if (st) return st;
            for (auto& rp : b->reps) rp.have_canon = true;
        }
        return SW_OK;
    }
    int rows = 0, hrows = 0;
    for (int32_t s = 0; s < nsweeps; ++s) {
        const bool v = verify && (s == nsweeps - 1);
        st = enqueue_sweep(b, profile, v, hash ? hrows : -1);
        if (st) return st;
        if (hash && ++hrows == kRing) {
            st = flush_hashes(b, hrows);
            if (st) return st;
            hrows = 0;
        }
        if (v)
            for (auto& rp : b->reps) rp.have_canon = true;
        if (measure) {
            st = launch_list(b, kLCounts, profile, static_cast<uint32_t>(rows));
            if (st) return st;
            st = launch_list(b, kLCountSum, profile, static_cast<uint32_t>(rows));
            if (st) return st;
            if (++rows == kRing) {
                st = flush_rings(b, rows);
                if (st) return st;
                rows = 0;
            }
        }
    }
    st = flush_hashes(b, hrows);
    if (st) return st;
    return flush_rings(b, rows);
}

int sw_batch_read_hashes(sw_batch* b, int32_t replica, uint64_t* out, size_t cap, size_t* n) {
    int st = check_replica(b, replica);
    if (st) return st;
    if (!n || (cap > 0 && !out)) return fail(SW_EINVAL, "bad output arrays");
    Replica& rp = b->reps[static_cast<size_t>(replica)];
    const size_t k = rp.hashes.size() < cap ? rp.hashes.size() : cap;
    for (size_t r = 0; r < k; ++r) {
        out[3 * r] = rp.hashes[r].t;
        out[3 * r + 1] = rp.hashes[r].hs;
        out[3 * r + 2] = rp.hashes[r].hl;
    }
    rp.hashes.erase(rp.hashes.begin(), rp.hashes.begin() + static_cast<std::ptrdiff_t>(k));
    *n = k;
    return SW_OK;
}

int sw_batch_measure(sw_batch* b, int32_t replica, sw_obs* out) {
    int st = check_replica(b, replica);
    if (st) return st;
    if (!out) return fail(SW_EINVAL, "null sw_obs");
    Replica& rp = b->reps[static_cast<size_t>(replica)];
    SweepArgs a = rp.args;
    a.count_row = reinterpret_cast<int64_t*>(b->base + rp.offset + rp.lay.scratch_row);
    SWB_HIP(b, launch_counts(a, b->stream));
    const uint32_t N = static_cast<uint32_t>(rp.p.L) * static_cast<uint32_t>(rp.p.L);
    SWB_HIP(b, launch_hash_state(a.spins, rp.have_canon ? a.canon : nullptr, N, a.hash_partial, b->stream));
    int64_t row[kRowWords];
    uint64_t h[2];
    Control ctl;
    SWB_HIP(b, hipStreamSynchronize(b->stream));
    SWB_HIP(b, hipMemcpy(&ctl, b->base + rp.offset + rp.lay.ctl, sizeof ctl, hipMemcpyDeviceToHost));
    st = fault_status(ctl.fault);
    if (st) {
        b->sticky = true;
        return st;
    }
    SWB_HIP(b, hipMemcpy(row, a.count_row, sizeof row, hipMemcpyDeviceToHost));
    SWB_HIP(b, hipMemcpy(h, a.hash_partial + 2 * static_cast<size_t>(hash_state_blocks(N)), sizeof h,
                         hipMemcpyDeviceToHost));
    fill_obs(rp.p, row, ctl.t, rp.sums, out);
    out->hash_spins = h[0];
    out->hash_labels = rp.have_canon ? h[1] : 0u;
    return SW_OK;
}

int sw_batch_read_spins(sw_batch* b, int32_t replica, int8_t* host, size_t n) {
    int st = check_replica(b, replica);
    if (st) return st;
    const Replica& rp = b->reps[static_cast<size_t>(replica)];
    const size_t N = static_cast<size_t>(rp.p.L) * rp.p.L;
    if (!host || n != N) return fail(SW_EINVAL, "n must be N = %zu", N);
    SWB_HIP(b, hipStreamSynchronize(b->stream));
    SWB_HIP(b, hipMemcpy(host, b->base + rp.offset + rp.lay.spins, N, hipMemcpyDeviceToHost));
    return SW_OK;
}

int sw_batch_read_labels(sw_batch* b, int32_t replica, int32_t* host, size_t n) {
    int st = check_replica(b, replica);
    if (st) return st;
    const Replica& rp = b->reps[static_cast<size_t>(replica)];
    const size_t N = static_cast<size_t>(rp.p.L) * rp.p.L;
    if (!host || n != N) return fail(SW_EINVAL, "n must be N = %zu", N);
    if (!rp.have_canon) return fail(SW_ESTATE, "no sweep was run with SW_VERIFY");
    SWB_HIP(b, hipStreamSynchronize(b->stream));
    SWB_HIP(b, hipMemcpy(host, b->base + rp.offset + rp.lay.canon, N * 4, hipMemcpyDeviceToHost));
    return SW_OK;
}

int sw_batch_tune(sw_batch* b, int32_t sweeps, int32_t* merge_tiles, int32_t* waves) {
    int st = check_batch(b);
    if (st) return st;
    if (sweeps <= 0 || !merge_tiles) return fail(SW_EINVAL, "need sweeps > 0 and an output pointer");
    std::vector<sw_lattice> ps;
    for (auto& rp : b->reps) ps.push_back(rp.p);
    const std::string key = tune_key_batch(b->arch, ps.data(), static_cast<int32_t>(ps.size()));
    int cached = 0;
    if (tune_cache_get(key, &cached)) {
        const int mt = cached / 16, w = cached % 16;
        bool ok = (w == kWaves || w == kWavesSmall);
        bool mt_ok = false;
        for (int m : kSchedules) mt_ok = mt_ok || m == mt;
        if (ok && mt_ok) {
            st = sw_batch_set_tile_waves(b, w);
            if (!st) st = sw_batch_set_schedule(b, mt);
            if (st) return st;
            *merge_tiles = mt;
            if (waves) *waves = w;
            return SW_OK;
        }
    }
    // Snapshot every replica's spins and control block, time each choice of
    // waves per tile and merge schedule on the same states (one captured run
    // of `sweeps` sweeps each, after a warm-up sweep), restore: the chain is
    // left exactly as it was.
    size_t snap = 0;
    for (auto& rp : b->reps) snap += up(static_cast<size_t>(rp.p.L) * rp.p.L) + up(sizeof(Control));
    void* tmp = nullptr;
    SWB_HIP(b, hipMalloc(&tmp, snap));
    auto save_restore = [&](bool save) -> hipError_t {
        char* p = static_cast<char*>(tmp);
        for (auto& rp : b->reps) {
            const size_t N = static_cast<size_t>(rp.p.L) * rp.p.L;
            char* sp = b->base + rp.offset + rp.lay.spins;
            char* cp = b->base + rp.offset + rp.lay.ctl;
            hipError_t e = save ? hipMemcpyAsync(p, sp, N, hipMemcpyDeviceToDevice, b->stream)
                                : hipMemcpyAsync(sp, p, N, hipMemcpyDeviceToDevice, b->stream);
            if (e != hipSuccess) return e;
            p += up(N);
            e = save ? hipMemcpyAsync(p, cp, sizeof(Control), hipMemcpyDeviceToDevice, b->stream)
                     : hipMemcpyAsync(cp, p, sizeof(Control), hipMemcpyDeviceToDevice, b->stream);
            if (e != hipSuccess) return e;
            p += up(sizeof(Control));
        }
        return hipSuccess;
    };
    int best_mt = b->merge_tiles, best_w = b->tile_waves;
    float best_ms = 0.0f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = save_restore(true);
    for (int w : kTileWavesChoices) {
        for (int mt : kSchedules) {
            if (e != hipSuccess || st) break;
            st = sw_batch_set_tile_waves(b, w);
            if (!st) st = sw_batch_set_schedule(b, mt);
            if (!st) st = sw_batch_sweep(b, 1, 0);  // capture and warm
            if (!st) st = sw_batch_sweep(b, sweeps, 0);  // capture the timed run
            if (!st) e = save_restore(false);
            if (st || e != hipSuccess) break;
            e = hipEventRecord(e0, b->stream);
            if (e == hipSuccess) st = sw_batch_sweep(b, sweeps, 0);
            if (e == hipSuccess && !st) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess && !st) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess && !st) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && !st && (best_ms == 0.0f || ms < best_ms)) {
                best_ms = ms;
                best_mt = mt;
                best_w = w;
            }
            if (e == hipSuccess && !st) e = save_restore(false);
        }
    }
    if (e == hipSuccess && !st) e = hipStreamSynchronize(b->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(tmp);
    if (st) return st;
    if (e != hipSuccess) return bfail(b, e, "sw_batch_tune");
    for (auto& rp : b->reps) rp.have_canon = false;
    st = sw_batch_set_tile_waves(b, best_w);
    if (!st) st = sw_batch_set_schedule(b, best_mt);
    if (st) return st;
    tune_cache_put(key, best_mt * 16 + best_w);
    *merge_tiles = best_mt;
    if (waves) *waves = best_w;
    return SW_OK;
}

int sw_batch_profile_read(sw_batch* b, const char** names, int64_t* launches, double* total_ms, int32_t cap,
                          int32_t* nk) {
    int st = check_batch(b);
    if (st) return st;
    if (!nk || cap < 0 || (cap > 0 && (!names || !launches || !total_ms))) return fail(SW_EINVAL, "bad output arrays");
    SWB_HIP(b, hipStreamSynchronize(b->stream));
    for (auto& pe : b->pending) {
        float ms = 0.0f;
        SWB_HIP(b, hipEventElapsedTime(&ms, pe.second.first, pe.second.second));
        b->prof_ms[pe.first] += ms;
        b->prof_launches[pe.first] += 1;
        b->free_events.push_back(pe.second.first);
        b->free_events.push_back(pe.second.second);
    }
    b->pending.clear();
    const int k = cap < kNumLists ? cap : kNumLists;
    for (int i = 0; i < k; ++i) {
        names[i] = kListNames[i];
        launches[i] = b->prof_launches[i];
        total_ms[i] = b->prof_ms[i];
    }
    *nk = k;
    for (int i = 0; i < kNumLists; ++i) {
        b->prof_launches[i] = 0;
        b->prof_ms[i] = 0.0;
    }
    return SW_OK;
}

int32_t sw_batch_size(sw_batch* b) { return b ? static_cast<int32_t>(b->reps.size()) : 0; }

void sw_batch_free(sw_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (auto& pe : b->pending) {
        (void)hipEventDestroy(pe.second.first);
        (void)hipEventDestroy(pe.second.second);
    }
    for (hipEvent_t e : b->free_events) (void)hipEventDestroy(e);
    if (b->owns) (void)hipFree(b->base);
    delete b;
}

}  // extern "C"
