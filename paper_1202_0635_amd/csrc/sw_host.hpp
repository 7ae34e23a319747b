// Host-side helpers shared by the single-lattice and the batched runtimes.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include "sw.h"
#include "sw_internal.hpp"

namespace swmc {
namespace host {

// Record a status with a formatted reason (thread-local, read by sw_last_error).
int fail(int status, const char* fmt, ...);
const char* last_error_text();
// max_side: kMaxSide for single-lattice contexts (two-level labels), else
// kMaxSideFlagged (one-level label words with a root flag).
bool lattice_ok(const sw_lattice* p, std::string* why, int max_side = kMaxSideFlagged);

double turn_cos(int n, int q);
double turn_sin(int n, int q);
size_t table_entries(const sw_lattice& p);
void build_table(const sw_lattice& p, uint32_t* out);

constexpr size_t kAlign = 256;
size_t up(size_t v);

struct Layout {
    size_t ctl, spins, bond_r, bond_d, labels, canon, count_partial, border_roots, border_bonds, ring, scratch_row,
        hash_ring, hash_partial, table, spins2, codes[2], nodes[2], nslots[2], border_slots, total;
};
// Arena layout; with_pair adds what single-lattice contexts use beside the
// one-level forest: the two-level labels (codes, node forests and node counts,
// two of each, alternating from sweep to sweep), the border records of slots,
// and a second spin buffer for the states of measured sweeps.
Layout layout_of(const sw_lattice& p, bool with_pair = false);

struct Observables {
    double e = 0.0, m2 = 0.0;
    double g1 = 0.0, g2 = 0.0;  // clock: G(L/4), G(L/2)
};
Observables observables_of(const sw_lattice& p, const int64_t* row);
// Running sums over the measured sweeps, folded in sweep order.
struct Sums {
    uint64_t samples = 0;
    double e = 0.0, m2 = 0.0, m4 = 0.0, g1 = 0.0, g2 = 0.0;
    void add(const Observables& o) {
        samples += 1;
        e += o.e;
        m2 += o.m2;
        m4 += o.m2 * o.m2;
        g1 += o.g1;
        g2 += o.g2;
    }
};
void fill_obs(const sw_lattice& p, const int64_t* row, uint64_t t, const Sums& sums, sw_obs* out);

SweepArgs make_args(const sw_lattice& p, char* base, const Layout& lay);
// Control block of a fresh lattice: t = 0, no sweep target.
extern const Control kFreshControl;
// A control block's fault bits (set by a kernel whose forest walk exceeded its
// step bound): SW_OK if none, else SW_EDEVICE with the reason recorded.
const char* fault_text(uint32_t bits);
int fault_status(uint32_t bits);

// Autotuner choices, remembered per key for the life of the process and, when
// the environment variable SWMC_TUNE_CACHE names a file, across processes
// (one "key choice" line per entry; later lines win).  Keys name what the
// choice depends on: the GPU architecture, the lattice size bucket
// (ceil(log2 L), or of the total sites of a batch), the model and q.
bool tune_cache_get(const std::string& key, int* choice);
void tune_cache_put(const std::string& key, int choice);
std::string tune_key_lattice(const std::string& arch, const sw_lattice& p);
std::string tune_key_batch(const std::string& arch, const sw_lattice* ps, int32_t n);

// One record of a per-sweep hash stream: the sweep index of the state after
// the sweep, H_s of that state and H_l of its canonical labels.
struct HashRecord {
    uint64_t t, hs, hl;
};

// Launch lists of the batched kernels: one launch per list and sweep covers
// the workgroups of every lattice in a set.
enum ListId {
    kLBondPotts, kLBondClock, kLBlockMerge, kLBorderMerge, kLFlatten, kLFlip, kLCounts, kLCountSum, kLHash, kLHashSum, kNumLists
};
// Workgroups list l needs for one lattice.
uint32_t blocks_for(int l, const SweepArgs& a);

}  // namespace host
}  // namespace swmc
