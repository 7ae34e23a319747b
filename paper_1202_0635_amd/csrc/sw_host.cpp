// Pure host pieces of libswmc (no HIP runtime calls): parameter checks, the
// FP64 cutoff table (Sec. 2 step (ii); Sec. 4 embedded cluster), the device
// arena layout, kernel-argument setup, observables from integer counts and
// the decoding of device fault bits.  Built into the library and, on its own,
// into the sanitized host tests.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <string>

#include "sw.h"
#include "sw_host.hpp"
#include "sw_internal.hpp"

namespace swmc {
namespace host {

thread_local std::string g_last_error;

const char* last_error_text() { return g_last_error.c_str(); }

int fail(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

bool lattice_ok(const sw_lattice* p, std::string* why, int max_side) {
    if (!p) return *why = "null sw_lattice", false;
    if (p->L < 2 || p->L > max_side) return *why = "L must be in [2, " + std::to_string(max_side) + "]", false;
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
    l.hash_ring = o; o += up(static_cast<size_t>(kRing) * 2 * 8);
    l.hash_partial = o; o += up(kHashPartWords * 8);
    l.table = o; o += up(table_entries(p) * 4);
    if (with_pair) {
        l.spins2 = o; o += up(N);
        for (int b = 0; b < 2; ++b) {
            l.codes[b] = o; o += up(N * 2);
            l.nodes[b] = o; o += up(tiles * kSlotsPerTile * 8);
            l.nslots[b] = o; o += up(tiles * 4);
        }
        l.border_slots = o; o += up(tiles * 4 * kTileW);
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

const Control kFreshControl = {0ull, ~0ull, 0u, 1u, 0u, 0u, {}};

const char* fault_text(uint32_t bits) {
    if (bits & kFaultLds) return "a tile-forest walk in LDS exceeded its step bound (broken tile forest)";
    if (bits & kFaultGlobal) return "a global forest walk exceeded its step bound (broken label forest)";
    if (bits & kFaultFlip) return "a flip walk exceeded its step bound (broken label forest)";
    if (bits & kFaultHash) return "a hash walk exceeded its step bound (broken label forest)";
    return nullptr;
}

int fault_status(uint32_t bits) {
    const char* t = fault_text(bits);
    if (!t) return SW_OK;
    return fail(SW_EDEVICE, "kernel fault 0x%x: %s", bits, t);
}

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
        case kLHash: return hash_blocks(a.L);
        case kLHashSum: return 1u;
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
    a.hash_ring = reinterpret_cast<uint64_t*>(base + lay.hash_ring);
    a.hash_partial = reinterpret_cast<uint64_t*>(base + lay.hash_partial);
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
    a.node_cap = static_cast<uint32_t>(a.tiles_x) * static_cast<uint32_t>(a.tiles_y) * kSlotsPerTile;
    a.key0 = static_cast<uint32_t>(p.seed);
    a.key1 = static_cast<uint32_t>(p.seed >> 32);
    return a;
}

// ---------------------------------------------------------------------------
// Autotuner cache.
// ---------------------------------------------------------------------------
namespace {
std::mutex g_tune_mutex;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

const char* tune_file() {
    const char* f = std::getenv("SWMC_TUNE_CACHE");
    return (f && *f) ? f : nullptr;
}

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* f = tune_file();
    if (!f) return;
    std::ifstream in(f);
    std::string line;
    while (std::getline(in, line)) {
        const size_t sp = line.rfind(' ');
        if (sp == std::string::npos || sp == 0) continue;
        char* end = nullptr;
        const long v = std::strtol(line.c_str() + sp + 1, &end, 10);
        if (end == line.c_str() + sp + 1) continue;
        g_tune[line.substr(0, sp)] = static_cast<int>(v);
    }
}

int ceil_log2(uint64_t v) {
    int k = 0;
    while ((1ull << k) < v) ++k;
    return k;
}
}  // namespace

bool tune_cache_get(const std::string& key, int* choice) {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    tune_load_locked();
    const auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *choice = it->second;
    return true;
}

void tune_cache_put(const std::string& key, int choice) {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    tune_load_locked();
    g_tune[key] = choice;
    if (const char* f = tune_file()) {
        std::ofstream out(f, std::ios::app);
        out << key << ' ' << choice << '\n';
    }
}

std::string tune_key_lattice(const std::string& arch, const sw_lattice& p) {
    return "lattice " + arch + " L2^" + std::to_string(ceil_log2(static_cast<uint64_t>(p.L))) + " model" +
           std::to_string(p.model) + " q" + std::to_string(p.q);
}

std::string tune_key_batch(const std::string& arch, const sw_lattice* ps, int32_t n) {
    uint64_t sites = 0;
    int lmax = 0, models = 0;
    for (int32_t r = 0; r < n; ++r) {
        sites += static_cast<uint64_t>(ps[r].L) * static_cast<uint64_t>(ps[r].L);
        lmax = ps[r].L > lmax ? ps[r].L : lmax;
        models |= 1 << ps[r].model;
    }
    return "batch " + arch + " sites2^" + std::to_string(ceil_log2(sites)) + " Lmax2^" +
           std::to_string(ceil_log2(static_cast<uint64_t>(lmax))) + " models" + std::to_string(models);
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
    out->absm = std::sqrt(o.m2 > 0.0 ? o.m2 : 0.0);
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
