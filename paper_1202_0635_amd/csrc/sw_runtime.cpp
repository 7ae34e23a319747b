// Host runtime of libswmc: parameter checks, the FP64 cutoff table, the
// device arena, kernel sequencing and the C-ABI of include/sw.h.
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

namespace swmc {
namespace host {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

bool lattice_ok(const sw_lattice* p, std::string* why) {
    if (!p) return *why = "null sw_lattice", false;
    if (p->L < 2 || p->L > 46340) return *why = "L must be in [2, 46340]", false;
    if (p->q < 2 || p->q > 32) return *why = "q must be in [2, 32]", false;
    if (p->model != SW_POTTS && p->model != SW_CLOCK) return *why = "model must be SW_POTTS or SW_CLOCK", false;
    if (p->reserved != 0) return *why = "reserved must be 0", false;
    if (!(p->T > 0.0) || !std::isfinite(p->T)) return *why = "T must be positive and finite", false;
    if (!(p->J > 0.0) || !std::isfinite(p->J)) return *why = "J must be positive and finite", false;
    return true;
}

// ---------------------------------------------------------------------------
// Cutoff table (Sec. 2 step (ii); Sec. 4 embedded cluster).  A bond is active
// iff its 32-bit uniform u < C, C = floor(2^32 p) with p = -expm1(-x) in FP64.
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;

// cos / sin of the angle 2 pi n / q; angles that are multiples of 30 degrees
// with a rational cosine (sine) are exact, the rest come from libm.
double turn_cos(int n, int q) {
    n = ((n % q) + q) % q;
    if ((12 * n) % q == 0) {
        static const double exact[12] = {1.0, NAN, 0.5, 0.0, -0.5, NAN, -1.0, NAN, -0.5, 0.0, 0.5, NAN};
        const double v = exact[(12 * n) / q];
        if (!std::isnan(v)) return v;
    }
    return std::cos(2.0 * kPi * static_cast<double>(n) / static_cast<double>(q));
}

double turn_sin(int n, int q) {
    n = ((n % q) + q) % q;
    if ((12 * n) % q == 0) {
        static const double exact[12] = {0.0, 0.5, NAN, 1.0, NAN, 0.5, 0.0, -0.5, NAN, -1.0, NAN, -0.5};
        const double v = exact[(12 * n) / q];
        if (!std::isnan(v)) return v;
    }
    return std::sin(2.0 * kPi * static_cast<double>(n) / static_cast<double>(q));
}

uint32_t cutoff(double x) {
    const double c = std::floor(std::ldexp(-std::expm1(-x), 32));
    if (c >= 4294967295.0) return 0xFFFFFFFFu;
    if (c <= 0.0) return 0u;
    return static_cast<uint32_t>(c);
}

size_t table_entries(const sw_lattice& p) {
    return p.model == SW_POTTS ? static_cast<size_t>(p.q) * p.q : static_cast<size_t>(p.q) * p.q * p.q;
}

void build_table(const sw_lattice& p, uint32_t* out) {
    const int q = p.q;
    if (p.model == SW_POTTS) {
        const uint32_t c = cutoff(p.J / p.T);
        for (int s = 0; s < q; ++s)
            for (int u = 0; u < q; ++u) out[s * q + u] = (s == u) ? c : 0u;
        return;
    }
    // Mirror m reflects state k to (m - k) mod q; the projection of two states
    // on the mirror normal multiplies to [cos(a-b) - cos(a+b-m)] / 2 (angles in
    // units of 2 pi / q); only positive products can bond, with x = 2 J P / T.
    for (int m = 0; m < q; ++m)
        for (int s = 0; s < q; ++s)
            for (int u = 0; u < q; ++u) {
                const double P = 0.5 * (turn_cos(s - u, q) - turn_cos(s + u - m, q));
                out[(static_cast<size_t>(m) * q + s) * q + u] = P > 0.0 ? cutoff(2.0 * p.J * P / p.T) : 0u;
            }
}

// ---------------------------------------------------------------------------
// Device arena layout.
// ---------------------------------------------------------------------------
size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

Layout layout_of(const sw_lattice& p, bool with_pair) {
    const size_t L = static_cast<size_t>(p.L);
    const size_t N = L * L;
    const size_t w64 = (L + 63) / 64;
    Layout l{};
    size_t o = 0;
    l.ctl = o; o += up(sizeof(Control));
    l.spins = o; o += up(N);
    l.bond_r = o; o += up(L * w64 * 8);
    l.bond_d = o; o += up(L * w64 * 8);
    l.labels = o; o += up(N * 4);
    l.canon = o; o += up(N * 4);
    l.count_partial = o; o += up(static_cast<size_t>(count_blocks(p.L)) * kRowWords * 4);
    const size_t tiles = ((L + kTileW - 1) / kTileW) * ((L + kTileH - 1) / kTileH);
    l.border_roots = o; o += up(tiles * 4 * kTileW * 4);
    l.border_bonds = o; o += up(tiles * kBorderMasks * 8);
    l.ring = o; o += up(static_cast<size_t>(kRing) * kRowWords * 8);
    l.scratch_row = o; o += up(kRowWords * 8);
    l.table = o; o += up(table_entries(p) * 4);
    if (with_pair) {
        l.spins2 = o; o += up(N);
        l.labels2 = o; o += up(N * 4);
    }
    l.total = o;
    return l;
}

Observables observables_of(const sw_lattice& p, const int64_t* row) {
    const double N = static_cast<double>(p.L) * static_cast<double>(p.L);
    const int q = p.q;
    const int64_t* hist = row + kRowHist;
    const int64_t* pair = row + kRowPair;
    Observables o;
    if (p.model == SW_POTTS) {
        o.e = p.J * (2.0 * N - static_cast<double>(pair[0])) / N;
        double s2 = 0.0;
        for (int k = 0; k < q; ++k) s2 += static_cast<double>(hist[k]) * static_cast<double>(hist[k]);
        o.m2 = (static_cast<double>(q) * s2 - N * N) / (static_cast<double>(q - 1) * N * N);
    } else {
        double e = 0.0;
        for (int d = 0; d < q; ++d) e += static_cast<double>(pair[d]) * turn_cos(d, q);
        o.e = -p.J * e / N;
        double mx = 0.0, my = 0.0;
        for (int k = 0; k < q; ++k) {
            mx += static_cast<double>(hist[k]) * turn_cos(k, q);
            my += static_cast<double>(hist[k]) * turn_sin(k, q);
        }
        o.m2 = (mx * mx + my * my) / (N * N);
        // G(r): mean over the 2N displaced pairs of cos(theta_j - theta_i)
        double g1 = 0.0, g2 = 0.0;
        for (int d = 0; d < q; ++d) {
            g1 += static_cast<double>(row[kRowCorr1 + d]) * turn_cos(d, q);
            g2 += static_cast<double>(row[kRowCorr2 + d]) * turn_cos(d, q);
        }
        o.g1 = g1 / (2.0 * N);
        o.g2 = g2 / (2.0 * N);
    }
    return o;
}

const Control kFreshControl = {0ull, ~0ull, 0u, 1u, {}};

static uint32_t div_up(uint64_t a, uint64_t b) { return static_cast<uint32_t>((a + b - 1) / b); }

uint32_t blocks_for(int l, const SweepArgs& a) {
    const uint64_t L = static_cast<uint64_t>(a.L);
    const int mt = a.merge_tiles;
    switch (l) {
        case kLBondPotts: return a.model == SW_POTTS ? static_cast<uint32_t>(a.tiles_x * a.tiles_y) : 0u;
        case kLBondClock: return a.model == SW_CLOCK ? static_cast<uint32_t>(a.tiles_x * a.tiles_y) : 0u;
        case kLBlockMerge: return mt > 1 ? merge_blocks_x(a.tiles_x, mt) * merge_blocks_x(a.tiles_y, mt) : 0u;
        case kLBorderMerge: return div_up((merge_blocks_x(a.tiles_x, mt) + merge_blocks_x(a.tiles_y, mt)) * L, 256);
        case kLFlatten: return div_up((static_cast<uint64_t>(a.tiles_x) + a.tiles_y) * L, 256);
        case kLFlip: return static_cast<uint32_t>(a.tiles_x * a.tiles_y);
        case kLCounts: return count_blocks(a.L);
        case kLCountSum: return 1u;
        default: return 0u;
    }
}

SweepArgs make_args(const sw_lattice& p, char* base, const Layout& lay) {
    SweepArgs a{};
    a.spins = reinterpret_cast<int8_t*>(base + lay.spins);
    a.flip_out = a.spins;
    a.bond_r = reinterpret_cast<uint64_t*>(base + lay.bond_r);
    a.bond_d = reinterpret_cast<uint64_t*>(base + lay.bond_d);
    a.labels = reinterpret_cast<uint32_t*>(base + lay.labels);
    a.canon = reinterpret_cast<uint32_t*>(base + lay.canon);
    a.count_partial = reinterpret_cast<uint32_t*>(base + lay.count_partial);
    a.border_roots = reinterpret_cast<uint32_t*>(base + lay.border_roots);
    a.border_bonds = reinterpret_cast<uint64_t*>(base + lay.border_bonds);
    a.table = reinterpret_cast<const uint32_t*>(base + lay.table);
    a.ctl = reinterpret_cast<Control*>(base + lay.ctl);
    a.count_row = nullptr;
    a.L = p.L;
    a.q = p.q;
    a.model = p.model;
    a.w64 = (p.L + 63) / 64;
    a.tiles_x = (p.L + kTileW - 1) / kTileW;
    a.tiles_y = (p.L + kTileH - 1) / kTileH;
    a.tile_waves = (a.tiles_x * a.tiles_y < kSmallTiles) ? kWavesSmall : kWaves;
    a.merge_tiles = kMergeTiles;
    a.key0 = static_cast<uint32_t>(p.seed);
    a.key1 = static_cast<uint32_t>(p.seed >> 32);
    return a;
}

void fill_obs(const sw_lattice& p, const int64_t* row, uint64_t t, const Sums& sums, sw_obs* out) {
    std::memset(out, 0, sizeof *out);
    out->sweeps_done = t;
    out->samples = sums.samples;
    for (int k = 0; k < 32; ++k) {
        out->hist[k] = row[kRowHist + k];
        out->pair_hist[k] = row[kRowPair + k];
        if (p.model == SW_CLOCK) {
            out->corr_hist[0][k] = row[kRowCorr1 + k];
            out->corr_hist[1][k] = row[kRowCorr2 + k];
        }
    }
    const Observables o = observables_of(p, row);
    out->e_per_site = o.e;
    out->m2 = o.m2;
    out->g_quarter = o.g1;
    out->g_half = o.g2;
    if (sums.samples) {
        const double n = static_cast<double>(sums.samples);
        out->mean_e = sums.e / n;
        out->mean_m2 = sums.m2 / n;
        out->mean_m4 = sums.m4 / n;
        out->binder_u = out->mean_m2 > 0.0 ? out->mean_m4 / (out->mean_m2 * out->mean_m2) : 0.0;
        out->mean_g_quarter = sums.g1 / n;
        out->mean_g_half = sums.g2 / n;
        out->corr_ratio = out->mean_g_quarter != 0.0 ? out->mean_g_half / out->mean_g_quarter : 0.0;
    }
}

}  // namespace host
}  // namespace swmc

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
    // counts of measured sweeps run on a second stream (made on first use,
    // default priority), ordered against the sweep by events
    hipStream_t side = nullptr;
    hipEvent_t ev_state = nullptr, ev_count[2] = {nullptr, nullptr};
    uint64_t le_iterations = 0, le_sweeps = 0;
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

// Fold count rows [0, rows) of the device ring into the running averages.
int flush_ring(sw_ctx* c, int rows) {
    if (rows <= 0) return SW_OK;
    if (c->side) SW_HIP(c, hipStreamSynchronize(c->side));
    SW_HIP(c, hipStreamSynchronize(c->stream));
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
    if (!lattice_ok(p, &why)) {
        fail(SW_EINVAL, "%s", why.c_str());
        return 0;
    }
    return layout_of(*p, true).total;
}

int sw_cutoff_table(const sw_lattice* p, uint32_t* out, size_t n) {
    std::string why;
    if (!lattice_ok(p, &why)) return fail(SW_EINVAL, "%s", why.c_str());
    if (!out || n != table_entries(*p)) return fail(SW_EINVAL, "table size must be %zu", table_entries(*p));
    build_table(*p, out);
    return SW_OK;
}

int sw_init(const sw_lattice* p, void* dev_mem, size_t bytes, void* stream, sw_ctx** out) {
    if (!out) return fail(SW_EINVAL, "null output pointer");
    *out = nullptr;
    std::string why;
    if (!lattice_ok(p, &why)) return fail(SW_EINVAL, "%s", why.c_str());
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
    if (e != hipSuccess) return cleanup(fail(SW_EDEVICE, "sw_init: %s", hipGetErrorString(e)));
    *out = c;
    return SW_OK;
}

int sw_sweep(sw_ctx* c, int32_t nsweeps, uint32_t flags) {
    int st = check_ctx(c);
    if (st) return st;
    if (nsweeps < 0) return fail(SW_EINVAL, "nsweeps must be >= 0");
    if (flags & ~(SW_MEASURE | SW_VERIFY | SW_PROFILE)) return fail(SW_EINVAL, "unknown flag bits");
    const bool measure = flags & SW_MEASURE;
    const bool profile = flags & SW_PROFILE;
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
    // Sweeps after the first of a call fuse the previous sweep's flip into
    // their bond kernel: spins and labels alternate between the context's two
    // buffers, and the call ends with a flip into the primary spin buffer.
    int8_t* const spins0 = c->args.spins;
    int8_t* const spins1 = reinterpret_cast<int8_t*>(c->base + c->lay.spins2);
    uint32_t* const labels0 = c->args.labels;
    uint32_t* const labels1 = reinterpret_cast<uint32_t*>(c->base + c->lay.labels2);
    // Union-find path with measurement (not profiled): the count of a state
    // runs on the side stream after the kernel that wrote the state, and the
    // next kernel that overwrites that spin buffer (two sweeps later, or the
    // call's final flip) waits for it, so counting overlaps the merges and
    // the next sweep's bond kernel.
    const bool overlap = measure && !profile && c->labeler == kUnionFind;
    if (overlap && !c->side) {
        SW_HIP(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        SW_HIP(c, hipEventCreateWithFlags(&c->ev_state, hipEventDisableTiming));
        for (auto& ev : c->ev_count) SW_HIP(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
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
        uint32_t* R = (c->labeler == kHawick) ? reinterpret_cast<uint32_t*>(c->base + c->lay.labels2) : nullptr;
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
            st = timed(c, profile, kKFlip, [&] { return launch_flip(a, verify, c->stream); });
            if (st) return st;
            if (verify) c->have_canon = true;
            if (measure) {
                st = count_state(a);
                if (st) return st;
            }
        }
        return flush_ring(c, rows);
    }
    SweepArgs a = c->args;
    for (int32_t s = 0; s < nsweeps; ++s) {
        const bool last = s == nsweeps - 1;
        const bool verify = (flags & SW_VERIFY) && last;
        if (s == 0) {
            st = timed(c, profile, kKBondLocal, [&] { return launch_bond_local(a, c->stream); });
            if (st) return st;
        } else {
            SweepArgs f = a;
            f.labels_prev = a.labels;
            f.spins_prev = a.spins;
            f.labels = (a.labels == labels0) ? labels1 : labels0;
            f.spins = (a.spins == spins0) ? spins1 : spins0;
            st = before_write(f.spins);
            if (st) return st;
            st = timed(c, profile, kKFlipBond, [&] { return launch_flip_bond(f, c->stream); });
            if (st) return st;
            a = f;
            if (measure) {  // the state after sweep s - 1, which the fused kernel wrote
                st = count_state(a);
                if (st) return st;
            }
        }
        if (a.merge_tiles > 1) {
            st = timed(c, profile, kKBlockMerge, [&] { return launch_block_merge(a, c->stream); });
            if (st) return st;
        }
        st = timed(c, profile, kKBorderMerge, [&] { return launch_border_merge(a, c->stream); });
        if (st) return st;
        // a verified sweep's canonical labels need the links; otherwise the
        // flatten leaves root words where the next flip looks
        a.root_copies = verify ? 0 : 1;
        st = timed(c, profile, kKFlatten, [&] { return launch_flatten(a, c->stream); });
        if (st) return st;
        if (last) {
            SweepArgs f = a;
            f.flip_out = spins0;
            st = before_write(spins0);
            if (st) return st;
            st = timed(c, profile, kKFlip, [&] { return launch_flip(f, verify, c->stream); });
            if (st) return st;
            if (verify) c->have_canon = true;
            if (measure) {
                f.spins = spins0;
                st = count_state(f);
                if (st) return st;
            }
        }
    }
    // later work on the context's stream comes after every count of the call
    for (int b = 0; b < 2; ++b)
        if (pending[b]) SW_HIP(c, hipStreamWaitEvent(c->stream, c->ev_count[b], 0));
    return flush_ring(c, rows);
}

int sw_measure(sw_ctx* c, sw_obs* out) {
    int st = check_ctx(c);
    if (st) return st;
    if (!out) return fail(SW_EINVAL, "null sw_obs");
    SweepArgs a = c->args;
    a.count_row = reinterpret_cast<int64_t*>(c->base + c->lay.scratch_row);
    SW_HIP(c, launch_counts(a, c->stream));
    int64_t row[kRowWords];
    Control ctl;
    SW_HIP(c, hipStreamSynchronize(c->stream));
    SW_HIP(c, hipMemcpy(row, a.count_row, sizeof row, hipMemcpyDeviceToHost));
    SW_HIP(c, hipMemcpy(&ctl, c->base + c->lay.ctl, sizeof ctl, hipMemcpyDeviceToHost));
    fill_obs(c->p, row, ctl.t, c->sums, out);
    return SW_OK;
}

int sw_read_spins(sw_ctx* c, int8_t* host, size_t n) {
    int st = check_ctx(c);
    if (st) return st;
    const size_t N = static_cast<size_t>(c->p.L) * c->p.L;
    if (!host || n != N) return fail(SW_EINVAL, "n must be N = %zu", N);
    SW_HIP(c, hipStreamSynchronize(c->stream));
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

int sw_set_schedule(sw_ctx* c, int32_t merge_tiles) {
    const int st = check_ctx(c);
    if (st) return st;
    if (merge_tiles != 1 && merge_tiles != 2 && merge_tiles != 4)
        return fail(SW_EINVAL, "merge_tiles must be 1, 2 or 4");
    c->args.merge_tiles = merge_tiles;
    return SW_OK;
}

int sw_tune(sw_ctx* c, int32_t sweeps, int32_t* merge_tiles) {
    int st = check_ctx(c);
    if (st) return st;
    if (sweeps <= 0 || !merge_tiles) return fail(SW_EINVAL, "need sweeps > 0 and an output pointer");
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
    // Three rounds, each timing every schedule from the same saved state; a
    // schedule's time is its fastest round (the schedules' times differ by a
    // few per cent, about as much as one timing varies).
    const int kSchedules[3] = {1, 2, 4};
    float best_of[3] = {0.0f, 0.0f, 0.0f};
    for (int round = 0; round < 3; ++round) {
        for (int k = 0; k < 3; ++k) {
            if (e != hipSuccess || st) break;
            c->args.merge_tiles = kSchedules[k];
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
    int best = c->args.merge_tiles;
    float best_ms = 0.0f;
    for (int k = 0; k < 3; ++k)
        if (best_of[k] > 0.0f && (best_ms == 0.0f || best_of[k] < best_ms)) {
            best_ms = best_of[k];
            best = kSchedules[k];
        }
    if (e == hipSuccess && !st) e = hipStreamSynchronize(c->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(tmp);
    if (st) return st;
    if (e != hipSuccess) return device_fail(c, e, "sw_tune");
    c->args.merge_tiles = best;
    c->have_canon = false;
    *merge_tiles = best;
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

const char* sw_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
