// Host runtime of libswmc for single lattices: the device arena, kernel
// sequencing and the C-ABI of include/sw.h (parameter checks, the cutoff
// table and the arena layout are in sw_host.cpp).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sw.h"
#include "sw_host.hpp"
#include "sw_internal.hpp"

using namespace swmc;
using namespace swmc::host;

struct sw_ctx {
    sw_lattice p{};
    hipStream_t stream = nullptr;
    char* base = nullptr;
    bool owns = false;
    bool sticky = false;
    bool have_canon = false;
    Layout lay{};
    SweepArgs args{};
    std::vector<uint32_t> table;
    // running sums over measured sweeps
    Sums sums;
    std::vector<int64_t> ring_host;
    // per-kernel timing
    std::vector<hipEvent_t> free_events;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    int labeler = kUnionFind;
    std::string arch;  // gcnArchName of the device, for the autotuner cache
    // counts of measured sweeps run on a second stream (made on first use,
    // default priority), ordered against the sweep by events
    hipStream_t side = nullptr;
    hipEvent_t ev_state = nullptr, ev_count[2] = {nullptr, nullptr};
    uint64_t le_iterations = 0, le_sweeps = 0;
    // per-sweep state hashes (SW_HASH) moved to the host, not yet read
    std::vector<HashRecord> hashes;
    std::vector<uint64_t> hash_host;
    int64_t prof_launches[kNumKernels] = {};
    double prof_ms[kNumKernels] = {};
};

namespace {

int device_fail(sw_ctx* c, hipError_t e, const char* what) {
    if (c) c->sticky = true;
    return fail(SW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define SW_HIP(ctx, call)                                      \
    do {                                                      \
        const hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return device_fail(ctx, e_, #call); \
    } while (0)

hipEvent_t take_event(sw_ctx* c) {
    if (!c->free_events.empty()) {
        hipEvent_t e = c->free_events.back();
        c->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch one kernel of the sweep, optionally bracketed by timing events.
template <typename F>
int timed(sw_ctx* c, bool profile, int kid, F&& launch) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (profile) {
        e0 = take_event(c);
        e1 = take_event(c);
        if (!e0 || !e1) return device_fail(c, hipErrorOutOfMemory, "hipEventCreate");
        SW_HIP(c, hipEventRecord(e0, c->stream));
    }
    SW_HIP(c, launch());
    if (profile) {
        SW_HIP(c, hipEventRecord(e1, c->stream));
        c->pending.push_back({kid, {e0, e1}});
    }
    return SW_OK;
}

int check_ctx(sw_ctx* c) {
    if (!c) return fail(SW_EINVAL, "null context");
    if (c->sticky) return fail(SW_ESTATE, "context had a device error earlier");
    return SW_OK;
}

// After a synchronisation: the control block's fault bits (a kernel met a
// broken forest) make the context sticky.
int check_fault(sw_ctx* c, Control* ctl_out = nullptr) {
    Control ctl;
    SW_HIP(c, hipMemcpy(&ctl, c->base + c->lay.ctl, sizeof ctl, hipMemcpyDeviceToHost));
    if (ctl_out) *ctl_out = ctl;
    const int st = fault_status(ctl.fault);
    if (st) c->sticky = true;
    return st;
}

// Fold count rows [0, rows) of the device ring into the running averages.
int flush_ring(sw_ctx* c, int rows) {
    if (rows <= 0) return SW_OK;
    if (c->side) SW_HIP(c, hipStreamSynchronize(c->side));
    SW_HIP(c, hipStreamSynchronize(c->stream));
    const int st = check_fault(c);
    if (st) return st;
    c->ring_host.resize(static_cast<size_t>(rows) * kRowWords);
    SW_HIP(c, hipMemcpy(c->ring_host.data(), c->base + c->lay.ring, c->ring_host.size() * 8, hipMemcpyDeviceToHost));
    for (int r = 0; r < rows; ++r) {
        c->sums.add(observables_of(c->p, c->ring_host.data() + static_cast<size_t>(r) * kRowWords));
    }
    return SW_OK;
}

}  // namespace

extern "C" {

size_t sw_state_bytes(const sw_lattice* p) {
    std::string why;
    if (!lattice_ok(p, &why, kMaxSide)) {
        fail(SW_EINVAL, "%s", why.c_str());
        return 0;
    }
    return layout_of(*p, true).total;
}

int sw_cutoff_table(const sw_lattice* p, uint32_t* out, size_t n) {
    std::string why;
    if (!lattice_ok(p, &why, kMaxSide)) return fail(SW_EINVAL, "%s", why.c_str());
    if (!out || n != table_entries(*p)) return fail(SW_EINVAL, "table size must be %zu", table_entries(*p));
    build_table(*p, out);
    return SW_OK;
}

int sw_init(const sw_lattice* p, void* dev_mem, size_t bytes, void* stream, sw_ctx** out) {
    if (!out) return fail(SW_EINVAL, "null output pointer");
    *out = nullptr;
    std::string why;
    if (!lattice_ok(p, &why, kMaxSide)) return fail(SW_EINVAL, "%s", why.c_str());
    const Layout lay = layout_of(*p, true);
    if (dev_mem) {
        if (reinterpret_cast<uintptr_t>(dev_mem) % kAlign != 0) return fail(SW_EINVAL, "dev_mem must be 256-byte aligned");
        if (bytes < lay.total) return fail(SW_ENOMEM, "dev_mem has %zu bytes, need %zu", bytes, lay.total);
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SW_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fail(SW_EDEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SW_EDEVICE, "libswmc is built for gfx950; device %d is %s", dev, prop.gcnArchName);

    sw_ctx* c = new sw_ctx();
    c->p = *p;
    c->arch = std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':'));
    c->stream = static_cast<hipStream_t>(stream);
    c->lay = lay;
    if (dev_mem) {
        c->base = static_cast<char*>(dev_mem);
    } else {
        void* m = nullptr;
        e = hipMalloc(&m, lay.total);
        if (e != hipSuccess) {
            delete c;
            return fail(SW_ENOMEM, "hipMalloc(%zu): %s", lay.total, hipGetErrorString(e));
        }
        c->base = static_cast<char*>(m);
        c->owns = true;
    }
    c->table.resize(table_entries(*p));
    build_table(*p, c->table.data());

    c->args = make_args(*p, c->base, lay);
    SweepArgs& a = c->args;

    auto cleanup = [&](int st) {
        if (c->owns) (void)hipFree(c->base);
        delete c;
        return st;
    };
    e = hipMemcpyAsync(c->base + lay.ctl, &kFreshControl, sizeof(Control), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->base + lay.table, c->table.data(), c->table.size() * 4, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_init(a, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    // the side stream of measured sweeps and its events (default priority),
    // made here so that no measured call pays for them
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_state, hipEventDisableTiming);
    for (auto& ev : c->ev_count)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (c->side) (void)hipStreamDestroy(c->side);
        if (c->ev_state) (void)hipEventDestroy(c->ev_state);
        for (auto& ev : c->ev_count)
            if (ev) (void)hipEventDestroy(ev);
        return cleanup(fail(SW_EDEVICE, "sw_init: %s", hipGetErrorString(e)));
    }
    *out = c;
    return SW_OK;
}

int sw_sweep(sw_ctx* c, int32_t nsweeps, uint32_t flags) {
    int st = check_ctx(c);
    if (st) return st;
    if (nsweeps < 0) return fail(SW_EINVAL, "nsweeps must be >= 0");
    if (flags & ~(SW_MEASURE | SW_VERIFY | SW_PROFILE | SW_HASH)) return fail(SW_EINVAL, "unknown flag bits");
    const bool measure = flags & SW_MEASURE;
    const bool profile = flags & SW_PROFILE;
    const bool hash = flags & SW_HASH;
    // Per-sweep hashes (SW_HASH): hash_sweep reads the forest after a sweep's
    // border merge; rows of the device hash ring are moved to the host when
    // the ring is full and at the end of the call.
    int hrows = 0;
    auto flush_hashes = [&]() -> int {
        if (hrows == 0) return SW_OK;
        SW_HIP(c, hipStreamSynchronize(c->stream));
        Control ctl;
        const int st2 = check_fault(c, &ctl);
        if (st2) return st2;
        c->hash_host.resize(2 * static_cast<size_t>(hrows));
        SW_HIP(c, hipMemcpy(c->hash_host.data(), c->base + c->lay.hash_ring, c->hash_host.size() * 8,
                            hipMemcpyDeviceToHost));
        // every enqueued sweep has finished: the last record is the state ctl.t
        for (int r = 0; r < hrows; ++r)
            c->hashes.push_back({ctl.t - static_cast<uint64_t>(hrows - 1 - r), c->hash_host[2 * r],
                                 c->hash_host[2 * r + 1]});
        hrows = 0;
        return SW_OK;
    };
    auto hash_sweep = [&](const SweepArgs& a) -> int {
        if (!hash) return SW_OK;
        const int st2 = timed(c, profile, kKHash, [&] { return launch_hash_sweep(a, static_cast<uint32_t>(hrows), c->stream); });
        if (st2) return st2;
        if (++hrows == kRing) return flush_hashes();
        return SW_OK;
    };
    int64_t* const ring = reinterpret_cast<int64_t*>(c->base + c->lay.ring);
    int rows = 0;
    auto next_row = [&](int64_t** row) -> int {
        *row = ring + static_cast<size_t>(rows) * kRowWords;
        return SW_OK;
    };
    auto row_done = [&]() -> int {
        if (++rows < kRing) return SW_OK;
        const int st2 = flush_ring(c, rows);
        rows = 0;
        return st2;
    };
    // The primary spin buffer and the second one that measured sweeps
    // alternate with.
    int8_t* const spins0 = c->args.spins;
    int8_t* const spins1 = reinterpret_cast<int8_t*>(c->base + c->lay.spins2);
    // Union-find path with measurement (not profiled): the count of a state
    // runs on the side stream after the kernel that wrote the state, and the
    // next kernel that overwrites that spin buffer (two sweeps later, or the
    // call's final flip) waits for it, so counting overlaps the merges and
    // the next sweep's bond kernel.
    const bool overlap = measure && !profile && c->labeler == kUnionFind;
    bool pending[2] = {false, false};  // a count of spin buffer 0 / 1 may still run
    auto buffer_of = [&](const int8_t* p) { return p == spins0 ? 0 : 1; };
    auto before_write = [&](const int8_t* p) -> int {
        const int b = buffer_of(p);
        if (pending[b]) {
            SW_HIP(c, hipStreamWaitEvent(c->stream, c->ev_count[b], 0));
            pending[b] = false;
        }
        return SW_OK;
    };
    auto count_state = [&](SweepArgs a) -> int {
        st = next_row(&a.count_row);
        if (st) return st;
        if (overlap) {
            SW_HIP(c, hipEventRecord(c->ev_state, c->stream));
            SW_HIP(c, hipStreamWaitEvent(c->side, c->ev_state, 0));
            SW_HIP(c, launch_counts(a, c->side));
            const int b = buffer_of(a.spins);
            SW_HIP(c, hipEventRecord(c->ev_count[b], c->side));
            pending[b] = true;
        } else {
            st = timed(c, profile, kKCounts, [&] { return launch_counts(a, c->stream); });
            if (st) return st;
        }
        return row_done();
    };
    if (c->labeler != kUnionFind) {
        // The paper's labelers: every sweep is bonds, label equivalence until
        // a scan changes nothing, root words, flip.
        SweepArgs a = c->args;
        // Hawick et al.'s temporary array lives in the canonical-label buffer,
        // which the flip of a verified sweep fills only after the labeling
        uint32_t* R = (c->labeler == kHawick) ? c->args.canon : nullptr;
        if (R) c->have_canon = false;
        uint32_t* changed = &a.ctl->changed;
        const int64_t cap = 4ll * c->p.L + 64;  // labels fall at every pass that continues
        for (int32_t s = 0; s < nsweeps; ++s) {
            const bool verify = (flags & SW_VERIFY) && s == nsweeps - 1;
            st = timed(c, profile, kKBondsOnly, [&] { return launch_bonds_only(a, c->stream); });
            if (st) return st;
            SW_HIP(c, launch_le_init(a, R, c->stream));
            int64_t it = 0;
            for (;;) {
                SW_HIP(c, hipMemsetAsync(changed, 0, sizeof(uint32_t), c->stream));
                st = timed(c, profile, kKLeIteration, [&] { return launch_le_iteration(a, c->labeler, R, c->stream); });
                if (st) return st;
                uint32_t flag = 0;
                SW_HIP(c, hipMemcpyAsync(&flag, changed, sizeof flag, hipMemcpyDeviceToHost, c->stream));
                SW_HIP(c, hipStreamSynchronize(c->stream));
                ++it;
                if (!flag) break;
                if (it >= cap) {
                    c->sticky = true;
                    return fail(SW_EDEVICE, "label equivalence did not converge in %lld passes",
                                static_cast<long long>(cap));
                }
            }
            c->le_iterations += static_cast<uint64_t>(it);
            c->le_sweeps += 1;
            st = timed(c, profile, kKLeRoots, [&] { return launch_le_roots(a, c->stream); });
            if (st) return st;
            st = hash_sweep(a);
            if (st) return st;
            st = timed(c, profile, kKFlip, [&] { return launch_flip(a, verify, c->stream); });
            if (st) return st;
            if (verify) c->have_canon = true;
            if (measure) {
                st = count_state(a);
                if (st) return st;
            }
        }
        st = flush_hashes();
        if (st) return st;
        return flush_ring(c, rows);
    }
    // Union-find with two-level labels.  The first sweep of a call reads the
    // spins; every later one reads the previous sweep's codes and node forest
    // (the flip of that sweep, fused into the bond kernel), so codes, node
    // forests and node counts alternate between two buffers.  The merge joins
    // the node forest across tile borders; the call ends with the flip of its
    // last sweep into the primary spin buffer.  Measured sweeps have their
    // state stored by the fused kernel, alternately in the two spin buffers.
    uint16_t* const codes[2] = {reinterpret_cast<uint16_t*>(c->base + c->lay.codes[0]),
                                reinterpret_cast<uint16_t*>(c->base + c->lay.codes[1])};
    uint64_t* const nodes[2] = {reinterpret_cast<uint64_t*>(c->base + c->lay.nodes[0]),
                                reinterpret_cast<uint64_t*>(c->base + c->lay.nodes[1])};
    uint32_t* const nslots[2] = {reinterpret_cast<uint32_t*>(c->base + c->lay.nslots[0]),
                                 reinterpret_cast<uint32_t*>(c->base + c->lay.nslots[1])};
    SweepArgs a = c->args;
    a.border_slots = reinterpret_cast<uint8_t*>(c->base + c->lay.border_slots);
    for (int32_t s = 0; s < nsweeps; ++s) {
        const bool last = s == nsweeps - 1;
        const bool verify = (flags & SW_VERIFY) && last;
        const int b = s & 1;
        SweepArgs f = a;
        f.codes = codes[b];
        f.nodes = nodes[b];
        f.nslots = nslots[b];
        f.lroot = (hash || verify) ? c->args.labels : nullptr;  // tile-local roots, for canonical labels
        f.spins_out = nullptr;
        if (s == 0) {
            f.spins = spins0;
            st = timed(c, profile, kKCodeBond, [&] { return launch_code_bond(f, false, c->stream); });
            if (st) return st;
        } else {
            f.codes_prev = codes[b ^ 1];
            f.nodes_prev = nodes[b ^ 1];
            f.nslots_prev = nslots[b ^ 1];
            if (measure) {
                f.spins_out = b ? spins1 : spins0;
                st = before_write(f.spins_out);
                if (st) return st;
            }
            st = timed(c, profile, kKCodeFlipBond, [&] { return launch_code_bond(f, true, c->stream); });
            if (st) return st;
            if (measure) {  // the state after sweep s - 1, which the fused kernel stored
                SweepArgs m = f;
                m.spins = f.spins_out;
                st = count_state(m);
                if (st) return st;
            }
        }
        st = timed(c, profile, kKNodeMerge, [&] { return launch_node_merge(f, c->stream); });
        if (st) return st;
        if (hash) {
            st = timed(c, profile, kKHash, [&] { return launch_code_hash(f, static_cast<uint32_t>(hrows), c->stream); });
            if (st) return st;
            if (++hrows == kRing) {
                st = flush_hashes();
                if (st) return st;
            }
        }
        if (last) {
            SweepArgs g = f;
            g.flip_out = spins0;
            st = before_write(spins0);
            if (st) return st;
            st = timed(c, profile, kKCodeFlip, [&] { return launch_code_flip(g, verify, c->stream); });
            if (st) return st;
            if (verify) c->have_canon = true;
            if (measure) {
                g.spins = spins0;
                st = count_state(g);
                if (st) return st;
            }
        }
    }
    // later work on the context's stream comes after every count of the call
    for (int b = 0; b < 2; ++b)
        if (pending[b]) SW_HIP(c, hipStreamWaitEvent(c->stream, c->ev_count[b], 0));
    st = flush_hashes();
    if (st) return st;
    return flush_ring(c, rows);
}

int sw_read_hashes(sw_ctx* c, uint64_t* out, size_t cap, size_t* n) {
    int st = check_ctx(c);
    if (st) return st;
    if (!n || (cap > 0 && !out)) return fail(SW_EINVAL, "bad output arrays");
    SW_HIP(c, hipStreamSynchronize(c->stream));
    st = check_fault(c);
    if (st) return st;
    const size_t k = c->hashes.size() < cap ? c->hashes.size() : cap;
    for (size_t r = 0; r < k; ++r) {
        out[3 * r] = c->hashes[r].t;
        out[3 * r + 1] = c->hashes[r].hs;
        out[3 * r + 2] = c->hashes[r].hl;
    }
    c->hashes.erase(c->hashes.begin(), c->hashes.begin() + static_cast<std::ptrdiff_t>(k));
    *n = k;
    return SW_OK;
}

int sw_measure(sw_ctx* c, sw_obs* out) {
    int st = check_ctx(c);
    if (st) return st;
    if (!out) return fail(SW_EINVAL, "null sw_obs");
    SweepArgs a = c->args;
    a.count_row = reinterpret_cast<int64_t*>(c->base + c->lay.scratch_row);
    SW_HIP(c, launch_counts(a, c->stream));
    const uint32_t N = static_cast<uint32_t>(c->p.L) * static_cast<uint32_t>(c->p.L);
    SW_HIP(c, launch_hash_state(a.spins, c->have_canon ? a.canon : nullptr, N, a.hash_partial, c->stream));
    int64_t row[kRowWords];
    uint64_t h[2];
    Control ctl;
    SW_HIP(c, hipStreamSynchronize(c->stream));
    st = check_fault(c, &ctl);
    if (st) return st;
    SW_HIP(c, hipMemcpy(row, a.count_row, sizeof row, hipMemcpyDeviceToHost));
    SW_HIP(c, hipMemcpy(h, a.hash_partial + 2 * static_cast<size_t>(hash_state_blocks(N)), sizeof h,
                        hipMemcpyDeviceToHost));
    fill_obs(c->p, row, ctl.t, c->sums, out);
    out->hash_spins = h[0];
    out->hash_labels = c->have_canon ? h[1] : 0u;
    return SW_OK;
}

int sw_read_spins(sw_ctx* c, int8_t* host, size_t n) {
    int st = check_ctx(c);
    if (st) return st;
    const size_t N = static_cast<size_t>(c->p.L) * c->p.L;
    if (!host || n != N) return fail(SW_EINVAL, "n must be N = %zu", N);
    SW_HIP(c, hipStreamSynchronize(c->stream));
    st = check_fault(c);
    if (st) return st;
    SW_HIP(c, hipMemcpy(host, c->base + c->lay.spins, N, hipMemcpyDeviceToHost));
    return SW_OK;
}

int sw_read_labels(sw_ctx* c, int32_t* host, size_t n) {
    int st = check_ctx(c);
    if (st) return st;
    const size_t N = static_cast<size_t>(c->p.L) * c->p.L;
    if (!host || n != N) return fail(SW_EINVAL, "n must be N = %zu", N);
    if (!c->have_canon) return fail(SW_ESTATE, "no sweep was run with SW_VERIFY");
    SW_HIP(c, hipStreamSynchronize(c->stream));
    st = check_fault(c);
    if (st) return st;
    SW_HIP(c, hipMemcpy(host, c->base + c->lay.canon, N * 4, hipMemcpyDeviceToHost));
    return SW_OK;
}

int sw_read_bonds(sw_ctx* c, uint8_t* host_right, uint8_t* host_down, size_t n) {
    int st = check_ctx(c);
    if (st) return st;
    const size_t L = static_cast<size_t>(c->p.L);
    const size_t N = L * L;
    if (!host_right || !host_down || n != N) return fail(SW_EINVAL, "n must be N = %zu", N);
    const size_t w64 = static_cast<size_t>(c->args.w64);
    std::vector<uint64_t> r(L * w64), d(L * w64);
    SW_HIP(c, hipStreamSynchronize(c->stream));
    SW_HIP(c, hipMemcpy(r.data(), c->base + c->lay.bond_r, r.size() * 8, hipMemcpyDeviceToHost));
    SW_HIP(c, hipMemcpy(d.data(), c->base + c->lay.bond_d, d.size() * 8, hipMemcpyDeviceToHost));
    for (size_t y = 0; y < L; ++y)
        for (size_t x = 0; x < L; ++x) {
            host_right[y * L + x] = static_cast<uint8_t>((r[y * w64 + x / 64] >> (x % 64)) & 1u);
            host_down[y * L + x] = static_cast<uint8_t>((d[y * w64 + x / 64] >> (x % 64)) & 1u);
        }
    return SW_OK;
}

int sw_write_spins(sw_ctx* c, const int8_t* host, size_t n, uint64_t t) {
    int st = check_ctx(c);
    if (st) return st;
    const size_t N = static_cast<size_t>(c->p.L) * c->p.L;
    if (!host || n != N) return fail(SW_EINVAL, "n must be N = %zu", N);
    for (size_t i = 0; i < N; ++i)
        if (host[i] < 0 || host[i] >= c->p.q) return fail(SW_EINVAL, "spin %zu = %d is not in [0, q)", i, host[i]);
    Control ctl = kFreshControl;
    ctl.t = t;
    SW_HIP(c, hipStreamSynchronize(c->stream));
    SW_HIP(c, hipMemcpy(c->base + c->lay.spins, host, N, hipMemcpyHostToDevice));
    SW_HIP(c, hipMemcpy(c->base + c->lay.ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice));
    c->have_canon = false;
    return SW_OK;
}

int sw_device_spins(sw_ctx* c, void** dev_ptr) {
    int st = check_ctx(c);
    if (st) return st;
    if (!dev_ptr) return fail(SW_EINVAL, "null output pointer");
    *dev_ptr = c->base + c->lay.spins;
    return SW_OK;
}

int sw_profile_read(sw_ctx* c, const char** names, int64_t* launches, double* total_ms, int32_t cap, int32_t* nk) {
    int st = check_ctx(c);
    if (st) return st;
    if (!nk || cap < 0 || (cap > 0 && (!names || !launches || !total_ms))) return fail(SW_EINVAL, "bad output arrays");
    SW_HIP(c, hipStreamSynchronize(c->stream));
    for (auto& pe : c->pending) {
        float ms = 0.0f;
        SW_HIP(c, hipEventElapsedTime(&ms, pe.second.first, pe.second.second));
        c->prof_ms[pe.first] += ms;
        c->prof_launches[pe.first] += 1;
        c->free_events.push_back(pe.second.first);
        c->free_events.push_back(pe.second.second);
    }
    c->pending.clear();
    const int k = cap < kNumKernels ? cap : kNumKernels;
    for (int i = 0; i < k; ++i) {
        names[i] = kKernelNames[i];
        launches[i] = c->prof_launches[i];
        total_ms[i] = c->prof_ms[i];
    }
    *nk = k;
    for (int i = 0; i < kNumKernels; ++i) {
        c->prof_launches[i] = 0;
        c->prof_ms[i] = 0.0;
    }
    return SW_OK;
}

int sw_set_labeler(sw_ctx* c, int32_t labeler) {
    const int st = check_ctx(c);
    if (st) return st;
    if (labeler != SW_LABEL_UNION_FIND && labeler != SW_LABEL_HAWICK && labeler != SW_LABEL_KALENTEV)
        return fail(SW_EINVAL, "labeler must be SW_LABEL_UNION_FIND, SW_LABEL_HAWICK or SW_LABEL_KALENTEV");
    if (labeler != SW_LABEL_UNION_FIND && c->p.L > kMaxSideFlagged)
        return fail(SW_EINVAL, "the label-equivalence labelers take L <= %d", kMaxSideFlagged);
    c->labeler = labeler;
    return SW_OK;
}

int sw_labeler_stats(sw_ctx* c, uint64_t* iterations, uint64_t* sweeps) {
    const int st = check_ctx(c);
    if (st) return st;
    if (!iterations || !sweeps) return fail(SW_EINVAL, "null output pointer");
    *iterations = c->le_iterations;
    *sweeps = c->le_sweeps;
    return SW_OK;
}

int sw_set_tile_waves(sw_ctx* c, int32_t waves) {
    const int st = check_ctx(c);
    if (st) return st;
    if (waves != kWaves && waves != kWavesSmall) return fail(SW_EINVAL, "waves per tile must be 4 or 8");
    c->args.tile_waves = waves;
    return SW_OK;
}

int sw_tune(sw_ctx* c, int32_t sweeps, int32_t* waves) {
    int st = check_ctx(c);
    if (st) return st;
    if (sweeps <= 0 || !waves) return fail(SW_EINVAL, "need sweeps > 0 and an output pointer");
    const std::string key = tune_key_lattice(c->arch, c->p);
    int cached = 0;
    if (tune_cache_get(key, &cached) && (cached == kWaves || cached == kWavesSmall)) {
        c->args.tile_waves = cached;
        *waves = cached;
        return SW_OK;
    }
    const size_t N = static_cast<size_t>(c->p.L) * c->p.L;
    void* tmp = nullptr;
    SW_HIP(c, hipMalloc(&tmp, up(N) + up(sizeof(Control))));
    char* spins = c->base + c->lay.spins;
    char* ctl = c->base + c->lay.ctl;
    char* s_spins = static_cast<char*>(tmp);
    char* s_ctl = s_spins + up(N);
    hipError_t e = hipMemcpyAsync(s_spins, spins, N, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s_ctl, ctl, sizeof(Control), hipMemcpyDeviceToDevice, c->stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // Three rounds, each timing every choice from the same saved state; a
    // choice's time is its fastest round.
    const int kChoices[2] = {kWaves, kWavesSmall};
    float best_of[2] = {0.0f, 0.0f};
    for (int round = 0; round < 3; ++round) {
        for (int k = 0; k < 2; ++k) {
            if (e != hipSuccess || st) break;
            c->args.tile_waves = kChoices[k];
            st = sw_sweep(c, 1, 0);
            if (!st) e = hipEventRecord(e0, c->stream);
            if (!st && e == hipSuccess) st = sw_sweep(c, sweeps, 0);
            if (!st && e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (!st && e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (!st && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (!st && e == hipSuccess && (best_of[k] == 0.0f || ms < best_of[k])) best_of[k] = ms;
            if (!st && e == hipSuccess) e = hipMemcpyAsync(spins, s_spins, N, hipMemcpyDeviceToDevice, c->stream);
            if (!st && e == hipSuccess) e = hipMemcpyAsync(ctl, s_ctl, sizeof(Control), hipMemcpyDeviceToDevice, c->stream);
        }
    }
    int best = c->args.tile_waves;
    float best_ms = 0.0f;
    for (int k = 0; k < 2; ++k)
        if (best_of[k] > 0.0f && (best_ms == 0.0f || best_of[k] < best_ms)) {
            best_ms = best_of[k];
            best = kChoices[k];
        }
    if (e == hipSuccess && !st) e = hipStreamSynchronize(c->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(tmp);
    if (st) return st;
    if (e != hipSuccess) return device_fail(c, e, "sw_tune");
    c->args.tile_waves = best;
    c->have_canon = false;
    tune_cache_put(key, best);
    *waves = best;
    return SW_OK;
}

void sw_free(sw_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& pe : c->pending) {
        (void)hipEventDestroy(pe.second.first);
        (void)hipEventDestroy(pe.second.second);
    }
    for (hipEvent_t e : c->free_events) (void)hipEventDestroy(e);
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipEventDestroy(c->ev_state);
        for (hipEvent_t e : c->ev_count) (void)hipEventDestroy(e);
        (void)hipStreamDestroy(c->side);
    }
    if (c->owns) (void)hipFree(c->base);
    delete c;
}

const char* sw_strerror(int s) {
    switch (s) {
        case SW_OK: return "ok";
        case SW_EINVAL: return "invalid argument";
        case SW_ENOMEM: return "out of device memory";
        case SW_EDEVICE: return "device error";
        case SW_ESTATE: return "invalid state";
        case SW_EBUDGET: return "over memory budget";
        case SW_EBUSY: return "busy";
        default: return "unknown status";
    }
}

const char* sw_last_error(void) { return last_error_text(); }

}  // extern "C"
