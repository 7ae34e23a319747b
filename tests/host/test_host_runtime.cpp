// Host-only tests of libswmc's runtime pieces, built with g++ under
// AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_host_sanitized.py):
//   * parameter checks, the cutoff table, the arena layout, observables from
//     counts, the decoding of device fault bits and the autotuner cache
//     (sw_host.cpp);
//   * the request server's policy (sw_sched.hpp) driven by a recording fake
//     executor: arrival-order admission with head-of-line waiting, the memory
//     budget, slot reuse, retirement after exactly the requested sweeps,
//     rejection of requests that can never fit.
// Nothing here calls the HIP runtime.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "sw.h"
#include "sw_host.hpp"
#include "sw_internal.hpp"
#include "sw_sched.hpp"

using namespace swmc;
using namespace swmc::host;

static int g_failures = 0;
#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #cond); \
            ++g_failures;                                                        \
        }                                                                        \
    } while (0)

static sw_lattice lat(int L, int q, int model, double T, uint64_t seed = 1) {
    sw_lattice p{};
    p.L = L;
    p.q = q;
    p.model = model;
    p.T = T;
    p.J = 1.0;
    p.seed = seed;
    return p;
}

static void test_params() {
    std::string why;
    sw_lattice p = lat(64, 2, SW_POTTS, 1.0);
    CHECK(lattice_ok(&p, &why));
    for (int L : {1, 0, -3, 46341}) {
        sw_lattice b = p;
        b.L = L;
        CHECK(!lattice_ok(&b, &why));
    }
    // single lattices (two-level labels) go up to 65535
    for (int L : {46341, 65535}) {
        sw_lattice b = p;
        b.L = L;
        CHECK(lattice_ok(&b, &why, kMaxSide));
    }
    {
        sw_lattice b = p;
        b.L = 65536;
        CHECK(!lattice_ok(&b, &why, kMaxSide));
    }
    for (int q : {1, 33}) {
        sw_lattice b = p;
        b.q = q;
        CHECK(!lattice_ok(&b, &why));
    }
    sw_lattice b = p;
    b.T = 0.0;
    CHECK(!lattice_ok(&b, &why));
    b = p;
    b.T = NAN;
    CHECK(!lattice_ok(&b, &why));
    b = p;
    b.J = -1.0;
    CHECK(!lattice_ok(&b, &why));
    b = p;
    b.reserved = 1;
    CHECK(!lattice_ok(&b, &why));
    b = p;
    b.model = 2;
    CHECK(!lattice_ok(&b, &why));
    CHECK(!lattice_ok(nullptr, &why));
}

static void test_tables() {
    for (int q : {2, 3, 4, 6, 7, 32}) {
        for (double T : {0.05, 0.9, 3.0}) {
            sw_lattice p = lat(16, q, SW_POTTS, T);
            std::vector<uint32_t> t(table_entries(p));
            CHECK(t.size() == static_cast<size_t>(q * q));
            build_table(p, t.data());
            for (int a = 0; a < q; ++a)
                for (int c = 0; c < q; ++c) CHECK(t[a * q + c] == (a == c ? t[0] : 0u));
            // equal spins: p = 1 - exp(-J/T), so the cutoff is floor(2^32 p)
            const double pe = -std::expm1(-1.0 / T);
            CHECK(std::fabs(static_cast<double>(t[0]) - std::floor(std::ldexp(pe, 32))) <= 1.0);
            p.model = SW_CLOCK;
            std::vector<uint32_t> c(table_entries(p));
            CHECK(c.size() == static_cast<size_t>(q * q * q));
            build_table(p, c.data());
            // the bond rule is symmetric in the two spins, and two spins that
            // the mirror maps onto each other never bond (zero projection product)
            for (int m = 0; m < q; ++m)
                for (int a = 0; a < q; ++a) {
                    for (int d = 0; d < q; ++d) CHECK(c[(m * q + a) * q + d] == c[(m * q + d) * q + a]);
                    const int fa = ((m - a) % q + q) % q;
                    CHECK(c[(m * q + a) * q + fa] == 0u);
                }
        }
    }
}

static void test_layout() {
    for (int L : {2, 3, 63, 64, 65, 100, 1030, 4096, 65535}) {
        for (bool pair : {false, true}) {
            sw_lattice p = lat(L, 6, SW_CLOCK, 0.9);
            const Layout l = layout_of(p, pair);
            const size_t N = static_cast<size_t>(L) * L;
            std::vector<std::pair<size_t, size_t>> r = {
                {l.ctl, sizeof(Control)}, {l.spins, N}, {l.bond_r, static_cast<size_t>(L) * ((L + 63) / 64) * 8},
                {l.bond_d, static_cast<size_t>(L) * ((L + 63) / 64) * 8}, {l.labels, N * 4}, {l.canon, N * 4},
                {l.ring, static_cast<size_t>(kRing) * kRowWords * 8}, {l.scratch_row, kRowWords * 8},
                {l.hash_ring, static_cast<size_t>(kRing) * 16}, {l.hash_partial, kHashPartWords * 8},
                {l.table, table_entries(p) * 4}};
            if (pair) {
                const size_t tiles = static_cast<size_t>((L + kTileW - 1) / kTileW) * ((L + kTileH - 1) / kTileH);
                r.push_back({l.spins2, N});
                for (int b = 0; b < 2; ++b) {
                    r.push_back({l.codes[b], N * 2});
                    r.push_back({l.nodes[b], tiles * kSlotsPerTile * 8});
                    r.push_back({l.nslots[b], tiles * 4});
                }
                r.push_back({l.border_slots, tiles * 4 * kTileW});
            }
            for (auto& a : r) {
                CHECK(a.first % kAlign == 0);
                CHECK(a.first + a.second <= l.total);
            }
            for (size_t i = 0; i < r.size(); ++i)
                for (size_t j = i + 1; j < r.size(); ++j)
                    CHECK(r[i].first + r[i].second <= r[j].first || r[j].first + r[j].second <= r[i].first);
        }
    }
}

static void test_faults() {
    CHECK(fault_status(0u) == SW_OK);
    const uint32_t bits[] = {kFaultLds, kFaultGlobal, kFaultFlip, kFaultHash, kFaultGlobal | kFaultFlip};
    for (uint32_t bit : bits) {
        CHECK(fault_status(bit) == SW_EDEVICE);
        CHECK(std::strstr(last_error_text(), "step bound") != nullptr);
        CHECK(fault_text(bit) != nullptr);
    }
}

static void test_observables() {
    // an all-equal Ising state: E = 0, M^2 = 1; half and half: M^2 = 0
    sw_lattice p = lat(8, 2, SW_POTTS, 1.0);
    std::vector<int64_t> row(kRowWords, 0);
    row[kRowHist + 0] = 64;
    row[kRowPair + 0] = 128;
    Observables o = observables_of(p, row.data());
    CHECK(o.e == 0.0 && o.m2 == 1.0);
    row[kRowHist + 0] = 32;
    row[kRowHist + 1] = 32;
    row[kRowPair + 0] = 64;
    row[kRowPair + 1] = 64;
    o = observables_of(p, row.data());
    CHECK(o.m2 == 0.0 && o.e == 1.0);
    sw_obs out;
    Sums s;
    s.add(o);
    fill_obs(p, row.data(), 7, s, &out);
    CHECK(out.sweeps_done == 7 && out.samples == 1 && out.absm == 0.0);
}

// ---------------------------------------------------------------------------
// Pool allocator: random allocations and releases never overlap, the used
// count is exact, and releasing everything coalesces the pool into one extent.
// ---------------------------------------------------------------------------
static void test_pool() {
    std::mt19937_64 rng(5);
    const uint64_t size = 64ull << 20;
    sched::PoolAllocator pool(size);
    std::map<uint64_t, uint64_t> live;  // off -> rounded size
    uint64_t used = 0;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3) {
            const uint64_t n = 1 + rng() % (1u << 20);
            uint64_t off = 0;
            if (pool.alloc(n, &off)) {
                const uint64_t rn = sched::PoolAllocator::rounded(n);
                CHECK(off % sched::kPoolAlign == 0);
                CHECK(off + rn <= size);
                auto nx = live.lower_bound(off);
                if (nx != live.end()) CHECK(off + rn <= nx->first);
                if (nx != live.begin()) {
                    auto pv = std::prev(nx);
                    CHECK(pv->first + pv->second <= off);
                }
                live[off] = rn;
                used += rn;
            } else {
                CHECK(pool.largest_free() < sched::PoolAllocator::rounded(n));
            }
        } else {
            auto it2 = live.begin();
            std::advance(it2, static_cast<long>(rng() % live.size()));
            pool.release(it2->first, it2->second);
            used -= it2->second;
            live.erase(it2);
        }
        CHECK(pool.used() == used);
    }
    for (auto& kv : live) pool.release(kv.first, kv.second);
    CHECK(pool.used() == 0);
    CHECK(pool.extents() == 1 && pool.largest_free() == size);
}

// ---------------------------------------------------------------------------
// Server policy with a fake executor.
// ---------------------------------------------------------------------------
struct FakeExec {
    double clock = 0.0;
    int64_t steps = 0;
    std::vector<uint64_t> admitted;  // tags in admission order
    std::vector<uint64_t> retired;
    std::vector<uint64_t> rejected;
    std::map<uint64_t, int64_t> admit_step, retire_step;
    std::map<int, uint64_t> slot_tag;      // slot -> tag of the lattice it holds
    std::set<int> slots_seen;
    uint64_t live_bytes = 0, max_live = 0, budget = 0;
    int drains = 0, end_steps = 0;

    uint64_t bytes_of(const sw_request& r) const {
        return static_cast<uint64_t>(r.lattice.L) * r.lattice.L * 10 + 4096;
    }
    double now() const { return clock; }
    int admit(int slot, const sched::Slot& sl) {
        CHECK(slot_tag.count(slot) == 0);  // a slot holds one lattice at a time
        slot_tag[slot] = sl.req.tag;
        slots_seen.insert(slot);
        admitted.push_back(sl.req.tag);
        admit_step[sl.req.tag] = steps;
        live_bytes += sched::PoolAllocator::rounded(sl.bytes);
        max_live = live_bytes > max_live ? live_bytes : max_live;
        CHECK(sl.off + sl.bytes <= budget);
        return SW_OK;
    }
    int run(int) {
        ++steps;
        return SW_OK;
    }
    int retire(int slot, const sched::Slot& sl) {
        CHECK(slot_tag.count(slot) && slot_tag[slot] == sl.req.tag);
        slot_tag.erase(slot);
        retired.push_back(sl.req.tag);
        retire_step[sl.req.tag] = steps;
        live_bytes -= sched::PoolAllocator::rounded(sl.bytes);
        CHECK(sl.done >= sl.req.sweeps);
        return SW_OK;
    }
    void reject(const sw_request& r) { rejected.push_back(r.tag); }
    int end_step() {
        ++end_steps;
        clock += 1.0;
        return SW_OK;
    }
    int drain() {
        ++drains;
        return SW_OK;
    }
};

static sw_request req(uint64_t tag, int L, int64_t sweeps) {
    sw_request r{};
    r.lattice = lat(L, 2, SW_POTTS, 1.0, tag);
    r.sweeps = sweeps;
    r.tag = tag;
    return r;
}

static void test_server_policy() {
    const uint64_t budget = 1ull << 20;  // 1 MiB: lattices of L = 100 take ~100 KB, L = 300 ~900 KB
    const int slots = 4, k = 7;
    FakeExec ex;
    ex.budget = budget;
    sched::ServerCore<FakeExec> core(budget, slots, k, &ex);
    std::mt19937_64 rng(11);
    std::vector<sw_request> reqs;
    for (uint64_t t = 0; t < 60; ++t) {
        const int L = (t % 13 == 5) ? 300 : 20 + static_cast<int>(rng() % 90);
        reqs.push_back(req(t, L, 1 + static_cast<int64_t>(rng() % 40)));
    }
    reqs.push_back(req(999, 400, 5));  // 1.6 MB: can never fit
    for (auto& r : reqs) core.submit(r);
    CHECK(ex.rejected.size() == 1 && ex.rejected[0] == 999);
    int guard = 0;
    while (ex.retired.size() < 60 && guard++ < 10000) {
        int32_t active = 0;
        CHECK(core.step(&active) == SW_OK);
        CHECK(active <= slots);
        const sw_server_stats st = core.stats();
        CHECK(st.used_bytes <= budget);
        CHECK(st.active == static_cast<int64_t>(ex.slot_tag.size()));
    }
    CHECK(ex.retired.size() == 60);
    // arrival order of admission (head-of-line waiting: nothing overtakes)
    for (size_t i = 0; i < ex.admitted.size(); ++i) CHECK(ex.admitted[i] == i);
    // every lattice ran exactly ceil(sweeps / k) steps
    for (const sw_request& r : reqs) {
        if (r.tag == 999) continue;
        const int64_t steps = ex.retire_step[r.tag] - ex.admit_step[r.tag];
        CHECK(steps == (r.sweeps + k - 1) / k);
    }
    CHECK(ex.max_live <= budget);
    CHECK(ex.slots_seen.size() == static_cast<size_t>(slots));  // slots are reused
    const sw_server_stats st = core.stats();
    CHECK(st.completed == 60 && st.rejected == 1 && st.submitted == 61);
    CHECK(st.active == 0 && st.waiting == 0 && st.used_bytes == 0);
    CHECK(core.pool().extents() == 1);
    int32_t active = -1;
    CHECK(core.step(&active) == SW_OK && active == 0);
    CHECK(ex.drains >= 1);
}

// A head that does not fit waits, and the requests behind it wait too.
static void test_head_of_line() {
    FakeExec ex;
    const uint64_t budget = 1ull << 20;
    ex.budget = budget;
    sched::ServerCore<FakeExec> core(budget, 8, 10, &ex);
    core.submit(req(0, 250, 30));  // ~630 KB
    core.submit(req(1, 250, 10));  // does not fit beside request 0
    core.submit(req(2, 16, 10));   // would fit, but waits behind request 1
    int32_t active = 0;
    CHECK(core.step(&active) == SW_OK && active == 1);
    CHECK(ex.admitted.size() == 1 && core.waiting() == 2);
    CHECK(core.step(&active) == SW_OK && active == 1);
    CHECK(core.step(&active) == SW_OK && active == 1);  // request 0 retires at the end of this step
    CHECK(ex.retired.size() == 1 && ex.retired[0] == 0);
    CHECK(core.step(&active) == SW_OK && active == 2);  // 1 and 2 both fit now
    CHECK(ex.admitted.size() == 3 && ex.admitted[1] == 1 && ex.admitted[2] == 2);
}

// The autotuner cache: keys bucket lattices by ceil(log2 L) (batches by total
// sites and largest L) and separate models, q and architectures; the file
// named by SWMC_TUNE_CACHE (the test driver seeds it with one good line and
// malformed ones) is read once, and every new choice is appended to it.
static void test_tune_cache() {
    const std::string f = std::getenv("SWMC_TUNE_CACHE") ? std::getenv("SWMC_TUNE_CACHE") : "";
    CHECK(!f.empty());
    CHECK(tune_key_lattice("gfx950", lat(33, 2, SW_POTTS, 1.0)) == tune_key_lattice("gfx950", lat(64, 2, SW_POTTS, 1.0)));
    CHECK(tune_key_lattice("gfx950", lat(64, 2, SW_POTTS, 1.0)) != tune_key_lattice("gfx950", lat(65, 2, SW_POTTS, 1.0)));
    CHECK(tune_key_lattice("gfx950", lat(64, 2, SW_POTTS, 1.0)) != tune_key_lattice("gfx950", lat(64, 3, SW_POTTS, 1.0)));
    CHECK(tune_key_lattice("gfx950", lat(64, 6, SW_POTTS, 1.0)) != tune_key_lattice("gfx950", lat(64, 6, SW_CLOCK, 1.0)));
    CHECK(tune_key_lattice("gfx950", lat(64, 2, SW_POTTS, 1.0)) != tune_key_lattice("gfx942", lat(64, 2, SW_POTTS, 1.0)));
    // temperature, coupling and seed do not enter the key
    CHECK(tune_key_lattice("gfx950", lat(64, 2, SW_POTTS, 1.0, 1)) == tune_key_lattice("gfx950", lat(64, 2, SW_POTTS, 2.0, 9)));
    const sw_lattice one[1] = {lat(32, 2, SW_POTTS, 1.0)};
    const sw_lattice mix[2] = {lat(32, 2, SW_POTTS, 1.0), lat(20, 6, SW_CLOCK, 1.0)};
    CHECK(tune_key_batch("gfx950", one, 1) == "batch gfx950 sites2^10 Lmax2^5 models1");
    CHECK(tune_key_batch("gfx950", mix, 2) != tune_key_batch("gfx950", one, 1));
    int v = -1;
    CHECK(tune_cache_get("batch gfx950 sites2^10 Lmax2^5 models1", &v) && v == 33);  // seeded in the file
    CHECK(!tune_cache_get(tune_key_batch("gfx950", mix, 2), &v));
    CHECK(!tune_cache_get("junk", &v));
    const std::string k = tune_key_lattice("gfx950", lat(4096, 2, SW_POTTS, 1.0));
    CHECK(!tune_cache_get(k, &v));
    tune_cache_put(k, 4);
    CHECK(tune_cache_get(k, &v) && v == 4);
    tune_cache_put(k, 8);  // a later choice wins, here and when the file is read again
    CHECK(tune_cache_get(k, &v) && v == 8);
    std::ifstream in(f);
    std::string line, last;
    int lines = 0;
    while (std::getline(in, line)) {
        ++lines;
        last = line;
    }
    CHECK(last == k + " 8");
    CHECK(lines >= 3);
}

int main() {
    test_params();
    test_tables();
    test_layout();
    test_faults();
    test_observables();
    test_pool();
    test_server_policy();
    test_head_of_line();
    test_tune_cache();
    if (g_failures) {
        std::fprintf(stderr, "%d check(s) failed\n", g_failures);
        return 1;
    }
    std::printf("host runtime tests passed\n");
    return 0;
}
