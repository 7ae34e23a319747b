// HIP kernels of the Swendsen-Wang sweep for gfx950 (wave64, LDS union-find).
//
// One sweep (Sec. 2 steps (1)-(3); the GPU organisation of Sec. 3 is replaced
// by a non-iterative union-find).  Single lattices use two-level labels:
//   k_code_bond     per 64 x 64 tile: FK bonds from Philox draws, row runs by
//                   wave ballots, a Hoshen-Kopelman pass per wave and unions
//                   in an LDS forest.  Every tile-local component draws its
//                   cluster value; a component off the tile's perimeter writes
//                   its sites' new values straight into their 16-bit codes,
//                   one that reaches the perimeter becomes a node of the
//                   global forest (a slot of the tile) and its sites' codes
//                   name the slot.  Border records hold the perimeter sites'
//                   slots and the bond masks.  From a call's second sweep on,
//                   the kernel takes the state from the previous sweep's codes
//                   and node forest (the flip of that sweep fused in).
//   k_node_merge    the tile borders and the torus wrap: lock-free unions of
//                   node roots, the larger key (smallest site index of the
//                   component) linked under the smaller by compare-and-swap.
//   k_code_flip     the last sweep of a call: codes and merged nodes to spins
//                   (and canonical labels in verify mode).
//   k_code_hash     per-sweep state hashes from codes and merged nodes.
// Batches and the static entry point use one-level labels (a 32-bit forest
// over all sites with root words):
//   k_bond_local    the same tile kernel writing the label forest and border
//                   records of edge roots; tile-local roots hold their draw.
//   k_block_merge   (schedules 2 and 4) the inner borders of blocks of tiles,
//                   joined in LDS.
//   k_border_merge  the remaining tile borders and the wrap, as k_node_merge.
//   k_flatten       every linked tile-local root gets its cluster's root word
//                   (or, for a verified sweep, a link straight to the root).
//   k_flip          each site reaches its root word and takes the cluster's
//                   value (Potts) or reflection (clock).
//   k_counts        measured sweeps: n[k], neighbour differences and, for the
//                   clock model, the correlation counts at L/4 and L/2.
// The paper's own label-equivalence labelers (k_bonds_only, k_le_*) are kept
// as an ablation; kb_* are the batched versions (one launch for all replicas).
#include "sw_device.hpp"
#include "sw_internal.hpp"

namespace swmc {

const char* const kKernelNames[kNumKernels] = {"k_bond_local", "k_block_merge",   "k_border_merge", "k_flatten",
                                               "k_flip",       "k_counts",        "k_flip_bond",    "k_bonds_only",
                                               "k_le_iteration", "k_le_roots",    "k_hash",
                                               "k_code_bond",    "k_code_flip_bond", "k_node_merge", "k_code_flip"};

namespace {

__device__ __forceinline__ uint32_t lds_load(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_store(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Lane k of v takes the wave-uniform value s: one VALU instruction, no
// branch on the lane.  The lane is an immediate (with the value in a scalar
// register it is the instruction's one scalar operand), so k must fold to a
// constant below 16, as an unrolled loop index does; the switch then folds.
template <int K>
__device__ __forceinline__ void write_lane_k(uint32_t& v, uint32_t s) {
    asm("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(s), "i"(K));
}
__device__ __forceinline__ void write_lane(uint32_t& v, uint32_t s, int k) {
    switch (k) {
        case 0: write_lane_k<0>(v, s); break;
        case 1: write_lane_k<1>(v, s); break;
        case 2: write_lane_k<2>(v, s); break;
        case 3: write_lane_k<3>(v, s); break;
        case 4: write_lane_k<4>(v, s); break;
        case 5: write_lane_k<5>(v, s); break;
        case 6: write_lane_k<6>(v, s); break;
        case 7: write_lane_k<7>(v, s); break;
        case 8: write_lane_k<8>(v, s); break;
        case 9: write_lane_k<9>(v, s); break;
        case 10: write_lane_k<10>(v, s); break;
        case 11: write_lane_k<11>(v, s); break;
        case 12: write_lane_k<12>(v, s); break;
        case 13: write_lane_k<13>(v, s); break;
        case 14: write_lane_k<14>(v, s); break;
        case 15: write_lane_k<15>(v, s); break;
        default: break;
    }
}

// A walk that has taken more steps than its forest has nodes has met a broken
// forest (links must point to smaller indices): it records a fault bit in the
// control block and stops, so a kernel ends instead of looping.
__device__ __forceinline__ void record_fault(Control* ctl, uint32_t bit) {
    __hip_atomic_fetch_or(&ctl->fault, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x in the tile forest (parents always have smaller indices), with
// path halving: a visited node is pointed at its grandparent.  A halving store
// may overwrite a concurrent lowering of that node; the union that lowered it
// continues with the node's previous parent, so no connection is lost.
// p is P[x], already loaded by the caller.
__device__ __forceinline__ uint32_t lds_find_from(uint32_t* P, uint32_t x, uint32_t p, Control* ctl) {
    for (uint32_t n = 0; p != x; ++n) {
        if (n >= kLdsWalkCap) {
            record_fault(ctl, kFaultLds);
            return x;
        }
        const uint32_t gp = lds_load(&P[p]);
        if (gp == p) return p;
        lds_store(&P[x], gp);
        x = gp;
        p = lds_load(&P[x]);
    }
    return x;
}

__device__ __forceinline__ uint32_t lds_find(uint32_t* P, uint32_t x, Control* ctl) {
    return lds_find_from(P, x, lds_load(&P[x]), ctl);
}

// Join the sets of a and b: the larger root is lowered to the smaller with an
// LDS atomic min; if that root had meanwhile been linked elsewhere, its old
// parent still has to be joined, so the loop continues with it (each round
// lowers a root, so a correct forest ends it within its node count).
__device__ __forceinline__ void lds_union(uint32_t* P, uint32_t a, uint32_t b, Control* ctl) {
    for (uint32_t n = 0;; ++n) {
        if (n >= kLdsWalkCap) {
            record_fault(ctl, kFaultLds);
            return;
        }
        a = lds_find(P, a, ctl);
        b = lds_find(P, b, ctl);
        if (a == b) return;
        if (a < b) {
            const uint32_t tmp = a;
            a = b;
            b = tmp;
        }
        const uint32_t old = __hip_atomic_fetch_min(&P[a], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == a) return;
        a = old;
    }
}

__device__ __forceinline__ uint32_t g_load(const uint32_t* p) {
    return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void g_store(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x in the global forest, from x's word w (read coherently by the
// caller); *word receives the root word.  Path halving: a visited non-root
// is pointed at its grandparent.  Only non-root words are rewritten and only
// with an ancestor's index, so a concurrent compare-and-swap (which targets
// root words) is never disturbed.
__device__ __forceinline__ uint32_t g_find_from(uint32_t* lab, uint32_t x, uint32_t w, uint32_t* word,
                                                Control* ctl) {
    for (uint32_t n = 0; !(w & kRootFlag); ++n) {
        if (n >= kGlobalWalkCap) {
            record_fault(ctl, kFaultGlobal);
            break;
        }
        const uint32_t w2 = g_load(&lab[w]);
        if (w2 & kRootFlag) {
            *word = w2;
            return w;
        }
        g_store(&lab[x], w2);
        x = w2;
        w = g_load(&lab[x]);
    }
    *word = w;
    return x;
}

// Root of x, whose word w the caller has loaded, through ordinary (cached)
// loads, halving the path on the way.  Every word written before this kernel
// is visible; a word linked meanwhile may be seen stale, which at worst makes
// the following compare-and-swap fail.  A word read as a non-root can no
// longer be a root, so the halving stores never touch the root words the
// compare-and-swap works on.
__device__ __forceinline__ uint32_t c_find_from(uint32_t* lab, uint32_t x, uint32_t w, uint32_t* word,
                                                Control* ctl) {
    for (uint32_t n = 0; !(w & kRootFlag); ++n) {
        if (n >= kGlobalWalkCap) {
            record_fault(ctl, kFaultGlobal);
            break;
        }
        const uint32_t w2 = lab[w];
        if (w2 & kRootFlag) {
            *word = w2;
            return w;
        }
        lab[x] = w2;
        x = w2;
        w = lab[x];
    }
    *word = w;
    return x;
}

// Join the clusters whose roots were found (through the caches) as a and b,
// with root words wa and wb: the larger root is linked under the smaller one
// by compare-and-swap on its root word; after a failed swap the walk uses
// coherent loads (and halves the paths it visits).
__device__ void g_union_roots(uint32_t* lab, uint32_t a, uint32_t wa, uint32_t b, uint32_t wb, Control* ctl) {
    for (uint32_t n = 0; a != b; ++n) {
        if (n >= kGlobalWalkCap || !(wa & wb & kRootFlag)) {  // a walk gave up: the forest is broken
            record_fault(ctl, kFaultGlobal);
            return;
        }
        if (a > b) {
            uint32_t tmp = a;
            a = b;
            b = tmp;
            tmp = wa;
            wa = wb;
            wb = tmp;
        }
        uint32_t expected = wb;
        if (__hip_atomic_compare_exchange_strong(&lab[b], &expected, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        // the failed swap returned b's current word; a's first load is
        // issued before b's walk goes on
        const uint32_t wa0 = g_load(&lab[a]);
        b = g_find_from(lab, b, expected, &wb, ctl);
        a = g_find_from(lab, a, wa0, &wa, ctl);
    }
}

__device__ __forceinline__ int mirror_of(uint64_t t, int q, uint32_t k0, uint32_t k1) {
    return static_cast<int>(qmap(draw(0u, t, kMirror, k0, k1).w0, static_cast<uint32_t>(q)));
}

// The cluster draw of canonical label rho (Sec. 2 step (vi); the paper draws
// a new value for every label).  Potts q >= 3: qmap of word 0 of the draw
// with c0 = rho.  Two outcomes (Potts q = 2: the new value; clock: reflect or
// not): one bit, bit rho mod 128 of the draw with c0 = rho div 128 (word k
// holds bits 32k .. 32k + 31), so one draw serves 128 consecutive sites.
__device__ __forceinline__ bool two_outcomes(int model, int q) { return model == 1 || q == 2; }
__device__ __forceinline__ uint32_t group_bit(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t rho) {
    const uint32_t k = (rho >> 5) & 3u;
    const uint32_t word = (k == 0) ? w0 : (k == 1) ? w1 : (k == 2) ? w2 : w3;
    return (word >> (rho & 31u)) & 1u;
}


// ---------------------------------------------------------------------------
// Bonds that leave a tile (or wrap around the torus), read from the tiles'
// border records.  A bond is skipped when the bond before it on the same
// border joins the same two tile-local sets (both its ends are tile-internal
// neighbours of the skipped bond's ends).  The ends are returned as their
// tile-local roots.
// ---------------------------------------------------------------------------
struct BorderBond {
    bool active;
    uint32_t i, j;
};

__device__ __forceinline__ uint32_t bit(uint64_t m, int k) { return static_cast<uint32_t>(m >> k) & 1u; }

// Right-edge bond of tile column tx in row y (wrapping to column 0 after the
// last column).  The record words are loaded unconditionally, so their loads
// are issued together instead of one after another behind each test.
__device__ __forceinline__ BorderBond vertical_border_bond(const SweepArgs& a, int tx, int y) {
    const int ty = y / kTileH, ly = y - ty * kTileH;
    const int t = ty * a.tiles_x + tx;
    const int tr = ty * a.tiles_x + ((tx + 1 == a.tiles_x) ? 0 : tx + 1);
    const uint64_t* m = a.border_bonds + static_cast<size_t>(t) * kBorderMasks;
    const uint64_t rr = m[kRightR], rd = m[kRightD];
    const uint64_t ld = a.border_bonds[static_cast<size_t>(tr) * kBorderMasks + kLeftD];
    const uint32_t i = a.border_roots[(static_cast<size_t>(t) * 4 + 0) * kTileW + ly];
    const uint32_t j = a.border_roots[(static_cast<size_t>(tr) * 4 + 2) * kTileW + ly];
    const bool skip = ly != 0 && bit(rr, ly - 1) && bit(rd, ly - 1) && bit(ld, ly - 1);
    return {bit(rr, ly) && !skip, i, j};
}

// Bottom-edge bond of tile row ty in column x (wrapping to row 0).
__device__ __forceinline__ BorderBond horizontal_border_bond(const SweepArgs& a, int ty, int x) {
    const int tx = x / kTileW, lx = x - tx * kTileW;
    const int t = ty * a.tiles_x + tx;
    const int td = ((ty + 1 == a.tiles_y) ? 0 : ty + 1) * a.tiles_x + tx;
    const uint64_t* m = a.border_bonds + static_cast<size_t>(t) * kBorderMasks;
    const uint64_t bd = m[kBottomD], br = m[kBottomR];
    const uint64_t tr = a.border_bonds[static_cast<size_t>(td) * kBorderMasks + kTopR];
    const uint32_t i = a.border_roots[(static_cast<size_t>(t) * 4 + 1) * kTileW + lx];
    const uint32_t j = a.border_roots[(static_cast<size_t>(td) * 4 + 3) * kTileW + lx];
    const bool skip = lx != 0 && bit(bd, lx - 1) && bit(br, lx - 1) && bit(tr, lx - 1);
    return {bit(bd, lx) && !skip, i, j};
}

// ---------------------------------------------------------------------------
// Random start: s_i = qmap(draw(i, 0, init)).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_init(SweepArgs a) {
    const uint32_t N = __umul24(a.L, a.L);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const Words4 w = draw(i, 0, kInit, a.key0, a.key1);
    a.spins[i] = static_cast<int8_t>(qmap(w.w0, static_cast<uint32_t>(a.q)));
}

// ---------------------------------------------------------------------------
// The previous sweep's flip of one site, for the fused kernel: the root word
// of the site's cluster in the previous forest gives the new value (Potts) or
// the reflection bit for the old value (clock, mirror m).
// ---------------------------------------------------------------------------
template <bool kClock>
__device__ __forceinline__ int flipped(uint32_t root_word, int old, int m, int q) {
    if (!kClock) return static_cast<int>(root_word & 0xFFu);
    int v = old;
    if (root_word & 1u) {
        v = m - old;
        if (v < 0) v += q;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Bonds + tile-local labeling.  Lane = column; each wave owns kTileH/4
// consecutive rows.  Each spin is loaded once: its right neighbour comes from
// the next lane, its lower neighbour from the next row held in registers.
// The 32-bit bond uniforms are u = (hi << 24) | lo: one draw gives the high
// bytes of eight rows of a column; the low 24 bits only matter when a high
// byte equals the cutoff's high byte (probability 2^-8), so those ties are
// collected in a tile-wide list and resolved with one draw per tied site.
// ---------------------------------------------------------------------------
// kSpinTile (the clock model writing codes): the tile's state and the row
// below it stay in LDS for the tie resolutions and the codes.
template <bool kSpinTile>
struct BondShared {
    uint32_t P[kTileH * kTileW];          // tie list, then the tile forest, then per-root records
    uint64_t raw_r[kTileH];               // right-bond masks of the tile's rows
    uint64_t raw_d[kTileH];               // down-bond masks
    alignas(16) uint8_t halo[kTileH];     // spins of the column right of the tile
    uint8_t tbl[kSlotsPerTile];           // codes: the previous sweep's draw of each node of the tile
    uint8_t sp[kSpinTile ? (kTileH + 1) * kTileW : 4];
    uint32_t ntie;
    uint32_t nslots;
};

// Where the bond kernel takes the state from, and what it writes.
enum BondSource { kFromSpins = 0, kFromCodes = 1 };
enum BondOutput { kWriteLabels = 0, kWriteCodes = 1, kWriteBonds = 2 };

// Perimeter mark of a per-root record in the tile forest (code output): the
// record's low half then holds the mark and the component's slot, else the
// root's draw; the high half of the forest words of a wave's rows holds that
// wave's list of roots while they draw.
constexpr uint32_t kMarkPerimeter = 0x8000u;

// kFull: the tile lies inside the lattice (no column or row beyond L), which
// removes the bounds tests from every row.
template <int kModel, int kSrc, int kOut, bool kFull, int kW>
__device__ __forceinline__ void bond_local_tile(const SweepArgs& a, const int tx, const int ty,
                                                BondShared<kModel == 1 && kOut == kWriteCodes>& sh) {
    constexpr bool kClock = kModel == 1;
    constexpr bool kSpinTile = kClock && kOut == kWriteCodes;
    constexpr bool kFused = kSrc == kFromCodes;
    constexpr int RPW = kTileH / kW;  // rows per wave (kW waves per tile)
    static_assert(RPW % 8 == 0, "a wave's rows must be whole 8-row draw groups");
    static_assert(RPW <= 16, "phase 1 gathers a wave's row masks in lanes 0 .. 15");
    uint32_t* const P = sh.P;
    uint64_t* const raw_r = sh.raw_r;
    uint64_t* const raw_d = sh.raw_d;
    uint8_t* const halo = sh.halo;
    uint32_t& ntie = sh.ntie;
    extern __shared__ uint32_t cut[];  // clock: the q x q cutoff slice (sized at launch)

    const int lane = threadIdx.x & 63;
    const uint32_t ulane = threadIdx.x & 63u;
    // the wave index is uniform: keeping it (and every row index derived from
    // it) in scalar registers lets row accesses take a scalar row pointer and
    // the lane as a 32-bit offset
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int L = a.L, q = a.q;
    const int x0 = tx * kTileW, y0 = ty * kTileH;
    const int x = x0 + lane;
    // Site indices stay below 2^32 (L < 2^16), so 32-bit arithmetic with
    // 24-bit multiplies replaces 64-bit address products.
    const uint32_t tile_base = __umul24(y0, L) + static_cast<uint32_t>(x0);
    const size_t tile = static_cast<size_t>(ty) * a.tiles_x + tx;
    const bool col_ok = kFull || x < L;
    const int nvalid = kFull ? kTileW : min(kTileW, L - x0);
    const int nrows = kFull ? kTileH : min(kTileH, L - y0);
    // lanes whose right bond stays inside the tile (not the last column, no wrap)
    const uint64_t in_tile_r = (nvalid >= 64) ? (~0ull >> 1) : ((1ull << (nvalid - 1)) - 1ull);
    const uint64_t t = a.ctl->t;
    const uint32_t k0 = a.key0, k1 = a.key1;
    // A lattice whose sweep target is reached sits this sweep out; the later
    // kernels of the sweep read the decision from the control block.
    const bool live = t < a.ctl->target;
    if (tx == 0 && ty == 0 && threadIdx.x == 0) a.ctl->live = live ? 1u : 0u;
    if (!live) return;

    // Cutoffs of this sweep: Potts needs only the equal-spin cutoff; the clock
    // model reads the q x q slice of its mirror m from LDS.
    const uint32_t c_eq = a.table[0];
    const int m_cur = kClock ? mirror_of(t, q, k0, k1) : 0;
    if (kClock) {
        const uint32_t* src = a.table + static_cast<size_t>(m_cur) * q * q;
        for (int k = threadIdx.x; k < q * q; k += kW * 64) cut[k] = src[k];
        if (tx == 0 && ty == 0 && threadIdx.x == 0) a.ctl->mirror = static_cast<uint32_t>(m_cur);
    }
    if (threadIdx.x == 0) {
        ntie = 0;
        sh.nslots = 0;
    }
    // Fused kernel: the spins this tile reads are the previous sweep's flip of
    // the previous state (mirror of sweep t - 1 for the clock model).
    const int m_prev = (kFused && kClock) ? mirror_of(t - 1, q, k0, k1) : 0;
    // the column right of the tile: one site per lane of wave 0
    const int xh = (x0 + nvalid == L) ? 0 : x0 + nvalid;
    const int yh = y0 + lane;
    const bool halo_lane = wave == 0 && (kFull || yh < L);
    const uint32_t ih = __umul24(kFull ? yh : min(yh, L - 1), L) + static_cast<uint32_t>(xh);
    if (!kFused && wave == 0) halo[lane] = halo_lane ? static_cast<uint8_t>(a.spins[ih]) : 0;

    const int ly_base = wave * RPW;
    const int y_base = y0 + ly_base;
    int sreg[RPW + 1];
    // row r of the strip (r == RPW: the row below it); row L is row 0, the
    // periodic neighbour of row L - 1 (in a full tile only the row below a
    // strip can be row L)
    auto row_of = [&](int r) -> int {
        const int yr = y_base + r;
        return ((!kFull || r == RPW) && yr == L) ? 0 : yr;
    };
    auto row_ok = [&](int r) -> bool { return kFull || (col_ok && y_base + r <= L); };
    uint32_t cw[RPW + 1];  // fused: the previous codes of this lane's sites
    // Phase 1's bond draws depend only on the site and the sweep: one draw per
    // 8-row group of the lane's column, taken while the state loads are in
    // flight.
    Words4 hiw[RPW / 8];
    auto bond_draws = [&]() {
#pragma unroll
        for (int g = 0; g < RPW / 8; ++g) {
            const int yb = y0 + ly_base + g * 8;  // multiple of 8
            hiw[g] = {0, 0, 0, 0};
            if (kFull || (col_ok && yb < L)) hiw[g] = draw(__umul24(yb >> 3, L) + static_cast<uint32_t>(x), t, kBondHi, k0, k1);
        }
    };
    if (kFused) {
        // The loads that depend on nothing are issued first: this lane's
        // previous codes, the halo site's, and for thread k below the tile's
        // node count the word of node k.  Then the walks to node roots advance
        // together, one load each per step: node k's (its draw goes to LDS for
        // this tile's sites), the halo site's and that of the one row of the
        // strip that lies in another tile (the row below the strip, in the
        // tile below or row 0 through the wrap, or in a ragged tile the
        // wrapped row L), whose nodes lie in other tiles' forests.
        const uint32_t ns = min(a.nslots_prev[tile], kSlotsPerTile);
        if (kFull) {
            // the strip's rows through one row pointer advanced by L (a
            // scalar base and the lane's offset per load), the row below
            // through its own (it may wrap to row 0)
            const uint16_t* row = a.codes_prev + (__umul24(y_base, L) + static_cast<uint32_t>(x0));
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                cw[r] = row[ulane];
                row += L;
            }
            cw[RPW] = (a.codes_prev + (__umul24(row_of(RPW), L) + static_cast<uint32_t>(x0)))[ulane];
        } else {
#pragma unroll
            for (int r = 0; r <= RPW; ++r) {
                const uint16_t* row = a.codes_prev + (__umul24(row_of(r), L) + static_cast<uint32_t>(x0));
                cw[r] = row_ok(r) ? row[ulane] : 0u;
            }
        }
        const uint32_t hc = halo_lane ? static_cast<uint32_t>(a.codes_prev[ih]) : 0u;
        const bool t_walk = threadIdx.x < ns;
        uint64_t tw = t_walk ? a.nodes_prev[static_cast<uint32_t>(tile) * kSlotsPerTile + threadIdx.x] : kNodeRoot;
        bond_draws();
        int rf = -1;  // uniform
#pragma unroll
        for (int r = 0; r <= RPW; ++r)
            if ((!kFull || r == RPW) && y_base + r <= L && (row_of(r) >> 6) != ty) rf = r;
        uint32_t fc = 0u;
#pragma unroll
        for (int r = 0; r <= RPW; ++r)
            if (r == rf && row_ok(r)) fc = cw[r];
        const int yf = (rf >= 0) ? row_of(rf) : 0;
        const uint32_t fn = static_cast<uint32_t>((yf >> 6) * a.tiles_x + (x >> 6)) * kSlotsPerTile + (fc & 0xFFu);
        const uint32_t hn = static_cast<uint32_t>((yh >> 6) * a.tiles_x + (xh >> 6)) * kSlotsPerTile + (hc & 0xFFu);
        uint64_t fw = (fc & kCodeNode) ? a.nodes_prev[min(fn, a.node_cap - 1u)] : kNodeRoot;
        uint64_t hw = (hc & kCodeNode) ? a.nodes_prev[min(hn, a.node_cap - 1u)] : kNodeRoot;
        for (uint32_t k = 0; !(static_cast<uint32_t>(tw) & static_cast<uint32_t>(fw) & static_cast<uint32_t>(hw) & kNodeRoot);
             ++k) {
            if (k >= a.node_cap) {
                record_fault(a.ctl, kFaultGlobal);
                tw = fw = hw = kNodeRoot;
                break;
            }
            // (clamped: a broken forest stays in bounds)
            if (!(static_cast<uint32_t>(tw) & kNodeRoot)) tw = a.nodes_prev[min(static_cast<uint32_t>(tw), a.node_cap - 1u)];
            if (!(static_cast<uint32_t>(fw) & kNodeRoot)) fw = a.nodes_prev[min(static_cast<uint32_t>(fw), a.node_cap - 1u)];
            if (!(static_cast<uint32_t>(hw) & kNodeRoot)) hw = a.nodes_prev[min(static_cast<uint32_t>(hw), a.node_cap - 1u)];
        }
        if (t_walk) sh.tbl[threadIdx.x] = static_cast<uint8_t>(tw);
        // the state at a site from its code and, for a node's site, the root word
        auto value_of = [&](uint32_t c, uint64_t w) -> int {
            if (!(c & kCodeNode)) return static_cast<int>(c & 31u);
            const uint32_t v = static_cast<uint32_t>(w) & 0xFFu;
            return kClock ? flipped<true>(v, static_cast<int>((c >> 8) & 31u), m_prev, q) : static_cast<int>(v);
        };
        const int sf = value_of(fc, fw);
        if (wave == 0) halo[lane] = halo_lane ? static_cast<uint8_t>(value_of(hc, hw)) : 0;
        __syncthreads();  // the node draws, the halo and the cutoffs in LDS
        // (Potts: an inner site's code is its value; the table is read for
        // every site and used for a node's.)
        auto own = [&](uint32_t c) -> int {
            const uint32_t v = sh.tbl[c & 0xFFu];
            if (!kClock) return static_cast<int>((c & kCodeNode) ? v : c);
            if (!(c & kCodeNode)) return static_cast<int>(c & 31u);
            return flipped<true>(v, static_cast<int>((c >> 8) & 31u), m_prev, q);
        };
#pragma unroll
        for (int r = 0; r <= RPW; ++r) sreg[r] = !row_ok(r) ? 0 : (r == rf) ? sf : own(cw[r]);
        if (a.spins_out) {
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const uint32_t rb = __umul24(row_of(r), L) + static_cast<uint32_t>(x0);
                if (kFull || (col_ok && y_base + r < L)) (a.spins_out + rb)[ulane] = static_cast<int8_t>(sreg[r]);
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r <= RPW; ++r) {
            sreg[r] = row_ok(r) ? (a.spins + (__umul24(row_of(r), L) + static_cast<uint32_t>(x0)))[ulane] : 0;
        }
        bond_draws();
    }
    if (!kFused) __syncthreads();  // halo and cutoffs in LDS (the fused prologue's barrier covers them)
    const bool edge_lane = (lane == nvalid - 1);
    // The clock model's tile state (rows 0 .. nrows, the last one the row
    // below the tile) for the tie resolutions and the codes, which carry each
    // site's value before the flip; phase 1's barrier orders the stores.
    if (kSpinTile) {
#pragma unroll
        for (int r = 0; r <= RPW; ++r)
            if (ly_base + r <= nrows) sh.sp[(ly_base + r) * kTileW + lane] = static_cast<uint8_t>(sreg[r]);
    }

    // Phase 1: decisions on the high bytes; ties go to the list.  The right
    // neighbour comes from the next lane by a DPP wave shift; the edge lane
    // takes it from the halo, whose RPW bytes for this wave are read once.
    uint32_t hv[RPW / 4];  // four rows' halo bytes per word
#pragma unroll
    for (int k = 0; k < RPW / 4; ++k) hv[k] = *reinterpret_cast<const uint32_t*>(&halo[ly_base + 4 * k]);
    const uint32_t chi = c_eq >> 24;                    // Potts: high byte of the cutoff
    const bool lo_matters = (c_eq & 0xFFFFFFu) != 0u;   // ties need the low 24 bits
    // the strip's row masks gather in lanes: lane r holds row r's (low and
    // high halves, right and down bonds), stored to LDS after the loop
    uint32_t mrl = 0u, mrh = 0u, mdl = 0u, mdh = 0u;
#pragma unroll
    for (int g = 0; g < RPW / 8; ++g) {
        const int ly0 = ly_base + g * 8;
        const int yb = y0 + ly0;  // multiple of 8
        const Words4 hi = hiw[g];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int r = g * 8 + k;
            const int ly = ly0 + k;
            const bool ok = kFull || (col_ok && (yb + k < L));
            const int s = sreg[r];
            const int sd = sreg[r + 1];
            const int sr_next = __builtin_amdgcn_mov_dpp(s, 0x130, 0xF, 0xF, false);  // wave_shl:1, lane i <- i+1
            const uint32_t hword = hv[r >> 2];
            const int sr = edge_lane ? static_cast<int>((hword >> (8 * (r & 3))) & 0xFFu) : sr_next;
            const uint32_t word = (k < 2) ? hi.w0 : (k < 4) ? hi.w1 : (k < 6) ? hi.w2 : hi.w3;
            const uint32_t hr = (k & 1) ? ((word >> 8) & 0xFFu) : (word >> 24);
            const uint32_t hd = (k & 1) ? (word & 0xFFu) : ((word >> 16) & 0xFFu);
            uint64_t mr, md;
            bool tr, td;
            if (kClock) {
                const uint32_t cr = cut[s * q + sr];
                const uint32_t cd = cut[s * q + sd];
                mr = __ballot(ok && (hr < (cr >> 24)));
                md = __ballot(ok && (hd < (cd >> 24)));
                tr = ok && (hr == (cr >> 24)) && (cr & 0xFFFFFFu);
                td = ok && (hd == (cd >> 24)) && (cd & 0xFFFFFFu);
            } else {
                // Potts: a bond needs equal spins and a high byte below the cutoff's
                const uint64_t okm = kFull ? ~0ull : __ballot(ok);
                const uint64_t er = __ballot(s == sr), ed = __ballot(s == sd);
                mr = okm & er & __ballot(hr < chi);
                md = okm & ed & __ballot(hd < chi);
                tr = lo_matters && ok && (s == sr) && (hr == chi);
                td = lo_matters && ok && (s == sd) && (hd == chi);
            }
            write_lane(mrl, static_cast<uint32_t>(mr), r);
            write_lane(mrh, static_cast<uint32_t>(mr >> 32), r);
            write_lane(mdl, static_cast<uint32_t>(md), r);
            write_lane(mdh, static_cast<uint32_t>(md >> 32), r);
            if (tr || td) {
                const uint32_t pos = atomicAdd(&ntie, 1u);
                P[pos] = static_cast<uint32_t>(ly * kTileW + lane) | (tr ? 1u << 12 : 0u) | (td ? 1u << 13 : 0u);
            }
        }
    }
    if (lane < RPW) {
        raw_r[ly_base + lane] = (static_cast<uint64_t>(mrh) << 32) | mrl;
        raw_d[ly_base + lane] = (static_cast<uint64_t>(mdh) << 32) | mdl;
    }
    __syncthreads();

    // Phase 1b: ties resolved by the low 24 bits of the per-site draw.
    const uint32_t nt = ntie;
    for (uint32_t j = threadIdx.x; j < nt; j += kW * 64) {
        const uint32_t e = P[j];
        const int ly = static_cast<int>((e & 0xFFFu) >> 6), lx = static_cast<int>(e & 63u);
        const int y = y0 + ly, xx = x0 + lx;
        const uint32_t row = __umul24(y, L);
        const uint32_t i = row + static_cast<uint32_t>(xx);
        const Words4 lo = draw(i, t, kBondLo, k0, k1);
        // (the clock model's codes kernel has the tile's state in LDS; the
        // other clock kernels read the spin array)
        auto spin_at = [&](int yy, int xc) -> int { return a.spins[__umul24(yy, L) + static_cast<uint32_t>(xc)]; };
        const int s = !kClock ? 0 : kSpinTile ? sh.sp[ly * kTileW + lx] : spin_at(y, xx);  // a Potts tie implies equal spins
        if (e & (1u << 12)) {
            const int sr = !kClock ? 0
                           : kSpinTile ? ((lx + 1 < nvalid) ? sh.sp[ly * kTileW + lx + 1] : halo[ly])
                                       : spin_at(y, (xx + 1 == L) ? 0 : xx + 1);
            const uint32_t c = kClock ? cut[s * q + sr] : c_eq;
            if ((lo.w0 & 0xFFFFFFu) < (c & 0xFFFFFFu)) atomicOr(&raw_r[ly], 1ull << lx);
        }
        if (e & (1u << 13)) {
            const int sd = !kClock ? 0 : kSpinTile ? sh.sp[(ly + 1) * kTileW + lx] : spin_at((y + 1 == L) ? 0 : y + 1, xx);
            const uint32_t c = kClock ? cut[s * q + sd] : c_eq;
            if ((lo.w1 & 0xFFFFFFu) < (c & 0xFFFFFFu)) atomicOr(&raw_d[ly], 1ull << lx);
        }
    }
    __syncthreads();

    // Final bond masks to memory: one 64-bit word per row and direction.
    if (threadIdx.x < 2 * kTileH) {
        const int ly = threadIdx.x & (kTileH - 1);
        const int y = y0 + ly;
        if (kFull || y < L) {
            const uint32_t wi = __umul24(y, a.w64) + static_cast<uint32_t>(tx);
            if (threadIdx.x < kTileH)
                a.bond_r[wi] = raw_r[ly];
            else
                a.bond_d[wi] = raw_d[ly];
        }
    }
    if (kOut == kWriteBonds) return;  // the label-equivalence labelers start from the bonds alone
    // Border record, bond masks (lane = row of the tile for the column masks).
    if (wave == kW - 1) {
        const bool rowok = kFull || lane < nrows;
        const uint64_t rr = raw_r[lane], dd = raw_d[lane];
        const uint64_t right_r = __ballot(rowok && ((rr >> (nvalid - 1)) & 1ull));
        const uint64_t right_d = __ballot(rowok && ((dd >> (nvalid - 1)) & 1ull));
        const uint64_t left_d = __ballot(rowok && (dd & 1ull));
        uint64_t v = 0;
        if (lane == kRightR) v = right_r;
        if (lane == kRightD) v = right_d;
        if (lane == kLeftD) v = left_d;
        if (lane == kBottomD) v = raw_d[nrows - 1];
        if (lane == kBottomR) v = raw_r[nrows - 1];
        if (lane == kTopR) v = raw_r[0];
        if (lane < kBorderMasks) a.border_bonds[tile * kBorderMasks + lane] = v;
    }
    // Phase 2: each wave labels its strip of rows in raster order, as the
    // Hoshen-Kopelman scan does (Sec. 2).  P holds, for each site, its run's
    // first site, and for a run's first site, the run's label (a link to a
    // smaller index, or itself).  A bond mask held in scalar registers tests
    // a lane's bit with no vector instruction.
    const uint64_t le_lane = ~0ull >> (63 - lane);  // this lane and the lanes below it
    {
        // The wave's row masks are read once, one row per lane, and taken row
        // by row into scalar registers with lane reads.
        const uint64_t rr_lane = (lane < RPW) ? raw_r[ly_base + lane] : 0ull;
        const uint64_t dd_lane = (lane < RPW) ? raw_d[ly_base + lane] : 0ull;
        auto lane64 = [](uint64_t v, int k) -> uint64_t {
            const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(v), k);
            const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(v >> 32), k);
            return (static_cast<uint64_t>(hi) << 32) | lo;
        };
        // Every site points at its run's first site, which starts as the
        // run's own label.
        uint32_t node[RPW];
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int ly = ly_base + r;
            const uint64_t starts = ~((lane64(rr_lane, r) & in_tile_r) << 1);  // first sites of the runs
            node[r] = static_cast<uint32_t>(ly * kTileW + 63 - __clzll(starts & le_lane));
            P[ly * kTileW + lane] = node[r];
        }
        // Rows in raster order: a run takes the smallest label among the runs
        // above it that it is bonded to (labels of earlier rows are smaller),
        // and each other label it touches is lowered to that one.  A label
        // that has been lowered before is no longer a root: lowering it again
        // returns its parent, which must then be joined as well.  That check
        // of a row waits until the next row's loads are issued.
        // (Lane sets are kept as 64-bit masks in scalar registers.)
        uint32_t lab_prev = node[0];
        uint32_t old_p = 0, tgt_p = 0, lab_p = 0;
        uint64_t need_p = 0;
        auto join_parent = [&](uint64_t need, uint32_t old, uint32_t tgt, uint32_t lab) {
            const uint64_t bad = need & __ballot(old != tgt) & __ballot(old != lab);
            if (bad) {
                if (__builtin_amdgcn_inverse_ballot_w64(bad)) lds_union(P, old, lab, a.ctl);
            }
        };
#pragma unroll
        for (int r = 1; r < RPW; ++r) {
            const int ly = ly_base + r;
            const uint64_t up = (kFull || y0 + ly < L) ? lane64(dd_lane, r - 1) : 0ull;
            __builtin_amdgcn_wave_barrier();
            if (__builtin_amdgcn_inverse_ballot_w64(up)) atomicMin(&P[node[r]], lab_prev);
            __builtin_amdgcn_wave_barrier();
            const uint32_t lab = lds_load(&P[node[r]]);
            if (r > 1) join_parent(need_p, old_p, tgt_p, lab_p);
            const uint64_t need = up & __ballot(lab_prev != lab);
            uint32_t old = lab_prev;
            if (__builtin_amdgcn_inverse_ballot_w64(need))
                old = __hip_atomic_fetch_min(&P[lab_prev], lab, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            need_p = need;
            old_p = old;
            tgt_p = lab_prev;
            lab_p = lab;
            lab_prev = lab;
        }
        join_parent(need_p, old_p, tgt_p, lab_p);
    }
    __syncthreads();

    // Phase 2b: vertical bonds between the strips of consecutive waves.  A
    // bond is skipped when the lane to its left carries a vertical bond
    // between the same two runs.  The union starts from the two sites' run
    // entries (their run's first site, or its label), so the walks touch only
    // run starts and roots: every other site keeps pointing at its run's
    // first site, in its own row.
    if (wave + 1 < kW) {
        const int ly = ly_base + RPW - 1;
        const uint64_t d = (kFull || y0 + ly + 1 < L) ? raw_d[ly] : 0ull;
        if (((d >> lane) & 1ull) &&
            !(lane > 0 && ((d >> (lane - 1)) & 1ull) && ((raw_r[ly] >> (lane - 1)) & 1ull) &&
              ((raw_r[ly + 1] >> (lane - 1)) & 1ull)))
            lds_union(P, lds_load(&P[ly * kTileW + lane]), lds_load(&P[(ly + 1) * kTileW + lane]), a.ctl);
    }
    __syncthreads();

    // Roots.  After phase 2b the forest is final and is only read: a site
    // follows its parents (its run's first site, the run's label, ...) to the
    // root.  The walks of all rows of a wave advance together, one level per
    // step, with every level's loads issued at once; a root is its own parent,
    // so a walk that has arrived stays put, and the steps end when no site of
    // the wave moved.  The code output also walks from the perimeter sites
    // (edges as in the border record: right column, bottom row, left column,
    // top row), one edge per wave.
    constexpr bool kCodes = kOut == kWriteCodes;
    const uint32_t e = threadIdx.x >> 6, pos = ulane;
    const bool perim = kCodes && threadIdx.x < 4 * kTileW && static_cast<int>(pos) < ((e & 1u) ? nvalid : nrows);
    uint32_t proot = 0;
    if (perim) {
        const uint32_t col = (e == 0) ? static_cast<uint32_t>(nvalid - 1) : (e == 2) ? 0u : pos;
        const uint32_t row = (e == 1) ? static_cast<uint32_t>(nrows - 1) : (e == 3) ? 0u : pos;
        proot = row * kTileW + col;
    }
    // The walks step two levels per round, between two register sets, so
    // that no copies are needed; a set that did not move holds the roots.
    // (Entries are tile indices; LDS reads out of range return zero, and the
    // round count is bounded, so a broken forest cannot fault or hang here.)
    uint32_t rootreg[RPW], nxt[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) rootreg[r] = P[(ly_base + r) * kTileW + lane];
    if (kCodes) proot = P[proot];
    for (uint32_t n = 0;; n += 2) {
        uint64_t moved = 0;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            nxt[r] = P[rootreg[r]];
            moved |= __ballot(nxt[r] != rootreg[r]);
        }
        uint32_t pnxt = 0;
        if (kCodes) {
            pnxt = P[proot];
            moved |= __ballot(pnxt != proot);
        }
        if (moved == 0ull) break;
        moved = 0;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            rootreg[r] = P[nxt[r]];
            moved |= __ballot(rootreg[r] != nxt[r]);
        }
        if (kCodes) {
            proot = P[pnxt];
            moved |= __ballot(proot != pnxt);
        }
        if (moved == 0ull) break;
        if (n >= kLdsWalkCap) {
            record_fault(a.ctl, kFaultLds);
            break;
        }
    }
    __syncthreads();  // every root is read: P may now be rewritten
    if (kCodes) {
        // Every component that reaches the perimeter becomes a node: the
        // first perimeter site to mark its root takes the next slot.
        if (perim) {
            const uint32_t old = atomicOr(&P[proot], kMarkPerimeter);
            if (!(old & kMarkPerimeter)) P[proot] = kMarkPerimeter | atomicAdd(&sh.nslots, 1u);
        }
        __syncthreads();
        if (perim) a.border_slots[tile * (4 * kTileW) + threadIdx.x] = static_cast<uint8_t>(P[proot] & 0xFFu);
        if (threadIdx.x == 0) a.nslots[tile] = sh.nslots;
        // Each wave lists the roots of its rows in the high halves of its rows'
        // forest words; then one lane per root draws the cluster value (Sec. 3
        // assigns a new value to every label index; here only roots draw).  A
        // perimeter root's draw goes to its node, the others' to their record.
        uint16_t* const P16 = reinterpret_cast<uint16_t*>(P);
        const uint32_t list0 = static_cast<uint32_t>(ly_base * kTileW);
        uint32_t nroots = 0;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const bool ok = kFull || (col_ok && (y_base + r < L));
            const uint32_t self = static_cast<uint32_t>((ly_base + r) * kTileW + lane);
            const uint64_t rm = __ballot(ok && rootreg[r] == self);
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(rm >> 32),
                                                             __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(rm), 0u));
            if (__builtin_amdgcn_inverse_ballot_w64(rm)) P16[2 * (list0 + nroots + below) + 1] = static_cast<uint16_t>(self);
            nroots += static_cast<uint32_t>(__popcll(rm));
        }
        __builtin_amdgcn_wave_barrier();  // the list is read by other lanes of this wave only
        uint64_t* const nodes = a.nodes + tile * kSlotsPerTile;
        // Two outcomes: lane k < 2 RPW draws the (k & 1)-th 128-site group
        // that row ly_base + k / 2 of the tile meets, and a root reads its
        // group's words from that lane (all lanes take part in the reads).
        const bool one_bit = two_outcomes(kModel, q);
        Words4 gw = {0u, 0u, 0u, 0u};
        if (one_bit && ulane < 2u * RPW) {
            const uint32_t rf = tile_base + __umul24(static_cast<uint32_t>(ly_base) + (ulane >> 1), L);
            gw = draw((rf >> 7) + (ulane & 1u), t, kCluster, k0, k1);
        }
        for (uint32_t j0 = 0; j0 < nroots; j0 += 64) {
            const uint32_t j = j0 + ulane;
            const bool valid = j < nroots;
            const uint32_t root =
                valid ? (P16[2 * (list0 + j) + 1] & (kLdsWalkCap - 1u)) : static_cast<uint32_t>(ly_base * kTileW);
            const uint32_t gi = tile_base + __umul24(root >> 6, L) + (root & 63u);
            uint32_t v;
            if (one_bit) {
                const uint32_t rf = gi - (root & 63u);  // the row's first site in the tile
                const int src = static_cast<int>(2u * ((root >> 6) - static_cast<uint32_t>(ly_base)) + ((gi >> 7) - (rf >> 7)));
                v = group_bit(__shfl(gw.w0, src, 64), __shfl(gw.w1, src, 64), __shfl(gw.w2, src, 64),
                              __shfl(gw.w3, src, 64), gi);
            } else {
                v = valid ? qmap(draw(gi, t, kCluster, k0, k1).w0, static_cast<uint32_t>(q)) : 0u;
            }
            if (valid) {
                const uint32_t rec = P[root];
                if (rec & kMarkPerimeter)
                    nodes[rec & 0xFFu] = (static_cast<uint64_t>(gi) << 32) | kNodeRoot | v;
                else
                    P16[2 * root] = static_cast<uint16_t>(v);
            }
        }
        __syncthreads();
        // Codes: the new value of an inner component's sites, or the slot of
        // the node (and, clock, the old value) of a perimeter component's.
        // (Potts: the low half of a root's record is the code itself, the
        // mark being the node bit.)  Row pointers advance by L.
        const uint32_t rb = __umul24(y_base, L) + static_cast<uint32_t>(x0);
        uint16_t* crow = a.codes + rb;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int y = y_base + r;
            if (kFull || (col_ok && y < L)) {
                uint32_t code;
                if (kClock) {
                    const uint32_t rec = P[rootreg[r]] & 0xFFFFu;
                    const int old = static_cast<int>(sh.sp[(ly_base + r) * kTileW + lane]);
                    if (rec & kMarkPerimeter)
                        code = kCodeNode | (static_cast<uint32_t>(old) << 8) | (rec & 0xFFu);
                    else
                        code = static_cast<uint32_t>(flipped<true>(rec, old, m_cur, q));
                } else {
                    code = P16[2 * rootreg[r]];
                }
                crow[ulane] = static_cast<uint16_t>(code);
            }
            crow += L;
        }
        if (a.lroot) {  // (verify sweeps) every site's tile-local root
            uint32_t* lrow = a.lroot + rb;
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                if (kFull || (col_ok && y_base + r < L))
                    lrow[ulane] = tile_base + __umul24(rootreg[r] >> 6, L) + (rootreg[r] & 63u);
                lrow += L;
            }
        }
        return;
    }
    // Border record, edge roots (global site indices), from the registers of
    // the waves that own the rows: right column (edge 0) by the lane of the
    // last column, left column (edge 2) by lane 0, top row (edge 3) by wave 0,
    // bottom row (edge 1) by the wave holding row nrows - 1.
    {
        auto global_of = [&](uint32_t root) { return tile_base + __umul24(root >> 6, L) + (root & 63u); };
        uint32_t* const rec = a.border_roots + tile * 4 * kTileW;
        if (lane == nvalid - 1 || lane == 0) {
#pragma unroll
            for (int r = 0; r < RPW; ++r)
                if (kFull || ly_base + r < nrows) {
                    const uint32_t g = global_of(rootreg[r]);
                    if (lane == nvalid - 1) rec[0 * kTileW + ly_base + r] = g;
                    if (lane == 0) rec[2 * kTileW + ly_base + r] = g;
                }
        }
        if (lane < nvalid) {
            if (wave == 0) rec[3 * kTileW + lane] = global_of(rootreg[0]);
            if (ly_base <= nrows - 1 && nrows - 1 < ly_base + RPW) {
                uint32_t v = rootreg[0];
#pragma unroll
                for (int r = 1; r < RPW; ++r)
                    if (ly_base + r == nrows - 1) v = rootreg[r];
                rec[1 * kTileW + lane] = global_of(v);
            }
        }
    }
    uint32_t* list = P + ly_base * kTileW;  // this wave's rows of P hold its root list
    uint32_t nroots = 0;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int y = y_base + r;
        const bool ok = kFull || (col_ok && (y < L));
        const uint32_t self = static_cast<uint32_t>((ly_base + r) * kTileW + lane);
        const uint32_t root = rootreg[r];
        const uint64_t rm = __ballot(ok && root == self);  // the row's roots
        const bool is_root = __builtin_amdgcn_inverse_ballot_w64(rm);
        // every site of the row is stored (a root gets a placeholder root word
        // that its draw below overwrites), so label lines are written whole
        if (ok) (a.labels + (__umul24(y, L) + static_cast<uint32_t>(x0)))[ulane] =
            is_root ? kRootFlag : tile_base + __umul24(root >> 6, L) + (root & 63u);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(rm >> 32),
                                                         __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(rm), 0u));
        if (is_root) list[nroots + below] = self;
        nroots += static_cast<uint32_t>(__popcll(rm));
    }
    __builtin_amdgcn_wave_barrier();  // the list is read by other lanes of this wave only
    // Every tile-local root draws its cluster's value (Sec. 3 assigns a new
    // value to every label index; here only roots draw, one lane per root;
    // two outcomes: one draw per row group, as in the code output).
    const bool one_bit = two_outcomes(kModel, q);
    Words4 gw = {0u, 0u, 0u, 0u};
    if (one_bit && ulane < 2u * RPW) {
        const uint32_t rf = tile_base + __umul24(static_cast<uint32_t>(ly_base) + (ulane >> 1), L);
        gw = draw((rf >> 7) + (ulane & 1u), t, kCluster, k0, k1);
    }
    for (uint32_t j0 = 0; j0 < nroots; j0 += 64) {
        const uint32_t j = j0 + ulane;
        const bool valid = j < nroots;
        const uint32_t root = valid ? list[j] : static_cast<uint32_t>(ly_base * kTileW);
        const uint32_t i = tile_base + __umul24(root >> 6, L) + (root & 63u);
        uint32_t v;
        if (one_bit) {
            const uint32_t rf = i - (root & 63u);
            const int src = static_cast<int>(2u * ((root >> 6) - static_cast<uint32_t>(ly_base)) + ((i >> 7) - (rf >> 7)));
            v = group_bit(__shfl(gw.w0, src, 64), __shfl(gw.w1, src, 64), __shfl(gw.w2, src, 64),
                          __shfl(gw.w3, src, 64), i);
        } else {
            v = valid ? qmap(draw(i, t, kCluster, k0, k1).w0, static_cast<uint32_t>(q)) : 0u;
        }
        if (valid) a.labels[i] = kRootFlag | v;
    }
}

template <int kModel, int kSrc, int kOut, int kW>
__device__ __forceinline__ void bond_tile(const SweepArgs& a, const int tx, const int ty) {
    __shared__ BondShared<kModel == 1 && kOut == kWriteCodes> sh;
    if ((tx + 1) * kTileW <= a.L && (ty + 1) * kTileH <= a.L)
        bond_local_tile<kModel, kSrc, kOut, true, kW>(a, tx, ty, sh);
    else
        bond_local_tile<kModel, kSrc, kOut, false, kW>(a, tx, ty, sh);
}

// Thread g of a launch over the bonds that cross every step-th tile border
// (the right edge of tile columns step-1, 2 step-1, ... and the last column;
// likewise for tile rows).  g < nvb * L is row g % L of vertical border
// g / L; the rest is column h % L of horizontal border h / L.  Neighbouring
// threads take neighbouring sites of one border, which mostly share their
// tile-local roots, so their finds meet in the same cache lines.
__device__ __forceinline__ BorderBond border_bond(const SweepArgs& a, uint32_t g, const int step) {
    const uint32_t L = static_cast<uint32_t>(a.L);
    const uint32_t nvb = static_cast<uint32_t>((a.tiles_x + step - 1) / step);
    const uint32_t nhb = static_cast<uint32_t>((a.tiles_y + step - 1) / step);
    if (g < nvb * L) {
        const uint32_t k = g / L, y = g - k * L;
        return vertical_border_bond(a, min(static_cast<int>(k) * step + step - 1, a.tiles_x - 1), static_cast<int>(y));
    }
    g -= nvb * L;
    if (g < nhb * L) {
        const uint32_t r = g / L, x = g - r * L;
        return horizontal_border_bond(a, min(static_cast<int>(r) * step + step - 1, a.tiles_y - 1), static_cast<int>(x));
    }
    return {false, 0u, 0u};
}

// ---------------------------------------------------------------------------
// Merge, level 1: one workgroup per block of mt x mt tiles (mt <= 4) joins
// the block's inner tile borders in LDS.  The tile-local roots at the ends of
// every active inner border bond (from the border records) are entered in an
// LDS hash table (slot = node), and the unions run on an LDS forest whose
// links always go from the larger site index to the smaller.  Finally every node
// that is no longer a root has its global root word replaced by a link to
// its block root.  The nodes belong to this block only, so nothing here
// races with another workgroup.
// ---------------------------------------------------------------------------
constexpr int kHashBits = 13;
constexpr uint32_t kHashSlots = 1u << kHashBits;  // >= 2x the most nodes: 2 ends x 2 (mt-1) mt 64 bonds at mt = 4
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;
static_assert(kHashSlots >= 2u * 2u * 2u * 3u * 4u * 64u, "hash table sized for 4 x 4 tile blocks");

// Slot of key in a table of 2^kBits slots, inserting it if absent (linear
// probing; the tables are sized so that they never fill, so a free slot is
// always reached).
template <int kBits>
__device__ __forceinline__ uint32_t hash_insert(uint32_t* keys, uint32_t key) {
    constexpr uint32_t kSlots = 1u << kBits;
    uint32_t s = (key * 2654435761u) >> (32 - kBits);
    for (uint32_t n = 0; n < kSlots; ++n) {
        const uint32_t old = atomicCAS(&keys[s], kEmptyKey, key);
        if (old == kEmptyKey || old == key) return s;
        s = (s + 1) & (kSlots - 1);
    }
    return kSlots;  // unreachable: the table never fills
}

__device__ __forceinline__ uint32_t node_find(uint32_t* par, uint32_t x, Control* ctl) {
    uint32_t p = lds_load(&par[x]);
    for (uint32_t n = 0; p != x; ++n) {
        if (n >= kHashSlots) {
            record_fault(ctl, kFaultLds);
            return x;
        }
        const uint32_t gp = lds_load(&par[p]);
        if (gp == p) return p;
        lds_store(&par[x], gp);
        x = gp;
        p = lds_load(&par[x]);
    }
    return x;
}

// Join the sets of nodes a and b: the root with the larger key (site index)
// is linked under the other by compare-and-swap; a lost race retries.
__device__ __forceinline__ void node_union(uint32_t* par, const uint32_t* keys, uint32_t a, uint32_t b, Control* ctl) {
    for (uint32_t n = 0;; ++n) {
        if (n >= kHashSlots) {
            record_fault(ctl, kFaultLds);
            return;
        }
        a = node_find(par, a, ctl);
        b = node_find(par, b, ctl);
        if (a == b) return;
        if (keys[a] > keys[b]) {
            const uint32_t tmp = a;
            a = b;
            b = tmp;
        }
        if (atomicCAS(&par[b], b, a) == b) return;
    }
}

__device__ __forceinline__ void block_merge(const SweepArgs& a, const int bx, const int by) {
    __shared__ uint32_t keys[kHashSlots];
    __shared__ uint32_t par[kHashSlots];
    if (!a.ctl->live) return;
    for (uint32_t k = threadIdx.x; k < kHashSlots; k += blockDim.x) {
        keys[k] = kEmptyKey;
        par[k] = k;
    }
    __syncthreads();
    const int L = a.L;
    const int mt = a.merge_tiles;
    const int txa = bx * mt, tya = by * mt;
    const int ntx = min(mt, a.tiles_x - txa), nty = min(mt, a.tiles_y - tya);
    const int ya = tya * kTileH, xa = txa * kTileW;
    const int nrows = min((tya + nty) * kTileH, L) - ya;
    const int ncols = min((txa + ntx) * kTileW, L) - xa;
    const int nv = (ntx - 1) * nrows;  // bonds across the block's inner vertical tile borders
    const int nh = (nty - 1) * ncols;
    // at most 2 (mt-1) mt 64 <= 1536 bonds: two per thread of a 1024-thread workgroup
    constexpr int kPer = 2;
    static_assert(kPer * kMergeThreads >= 2 * 3 * 4 * 64, "bonds per thread");
    uint32_t ends[kPer][2];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int k = static_cast<int>(threadIdx.x) + r * kMergeThreads;
        ends[r][0] = ends[r][1] = kHashSlots;
        if (k >= nv + nh) continue;
        BorderBond b;
        if (k < nv)
            b = vertical_border_bond(a, txa + k / nrows, ya + k % nrows);
        else
            b = horizontal_border_bond(a, tya + (k - nv) / ncols, xa + (k - nv) % ncols);
        if (!b.active) continue;
        ends[r][0] = hash_insert<kHashBits>(keys, b.i);
        ends[r][1] = hash_insert<kHashBits>(keys, b.j);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPer; ++r)
        if (ends[r][0] < kHashSlots && ends[r][1] < kHashSlots) node_union(par, keys, ends[r][0], ends[r][1], a.ctl);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < kHashSlots; k += blockDim.x) {
        const uint32_t key = keys[k];
        if (key == kEmptyKey) continue;
        const uint32_t r = node_find(par, k, a.ctl);
        if (r != k) a.labels[key] = keys[r];
    }
}

// ---------------------------------------------------------------------------
// Merge, level 2: bonds across block borders and the periodic wrap, with the
// device-wide lock-free union.  Thread g < nbx*L: right edge of the last tile
// column of block column g / L; the rest: bottom edges of block rows.
// ---------------------------------------------------------------------------
// True in the lowest lane of the wave that wants a given key (ka, kb); the
// other wanting lanes with the same key get false.  The loop runs once per
// distinct key among the wanting lanes.
__device__ __forceinline__ bool wave_first(bool want, uint32_t ka, uint32_t kb) {
    const uint32_t lane = threadIdx.x & 63;
    uint64_t m = __ballot(want);
    while (m) {
        const int j = __ffsll(static_cast<unsigned long long>(m)) - 1;
        // (j is uniform: lane reads, not a permute through LDS)
        const uint32_t ja = __builtin_amdgcn_readlane(ka, j), jb = __builtin_amdgcn_readlane(kb, j);
        if (want && lane > static_cast<uint32_t>(j) && ka == ja && kb == jb) want = false;
        m &= __ballot(want) & ~((2ull << j) - 1ull);
    }
    return want;
}

// Neighbouring lanes take neighbouring sites of one border and mostly find
// the same two roots: of the lanes of a wave that found the same pair of
// roots only the lowest does the union.  (Every link ever stored points to an
// ancestor, so equal found roots mean equal sets.)
__device__ __forceinline__ void border_merge(const SweepArgs& a, const uint32_t gid) {
    if (!a.ctl->live) return;
    const BorderBond b = border_bond(a, gid, a.merge_tiles);
    uint32_t ra = kRootFlag, rb = kRootFlag, wa = 0, wb = 0;
    if (b.active) {
        // the two first loads are issued together; most walks end there
        const uint32_t wi = a.labels[b.i], wj = a.labels[b.j];
        ra = c_find_from(a.labels, b.i, wi, &wa, a.ctl);
        rb = c_find_from(a.labels, b.j, wj, &wb, a.ctl);
        if (ra > rb) {
            uint32_t tmp = ra;
            ra = rb;
            rb = tmp;
            tmp = wa;
            wa = wb;
            wb = tmp;
        }
    }
    if (wave_first(b.active && ra != rb, ra, rb)) g_union_roots(a.labels, ra, wa, rb, wb, a.ctl);
}

// ---------------------------------------------------------------------------
// Two-level labels: the unions across tile borders on the node forest.  A
// bond that leaves a tile joins the nodes of its two end sites' components
// (from the tiles' border records of slots); the bond-skipping rule is that
// of the one-level records.  Nodes are linked by their keys (smallest site
// indices): the root with the larger key goes under the other by a 64-bit
// compare-and-swap on its root word, so every cluster's root is the node of
// its smallest site, which carries the cluster's draw.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lo32(uint64_t w) { return static_cast<uint32_t>(w); }
__device__ __forceinline__ uint32_t hi32(uint64_t w) { return static_cast<uint32_t>(w >> 32); }

__device__ __forceinline__ uint64_t n_load(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of node x, whose word w the caller has loaded, through ordinary
// (cached) loads with path halving: a visited non-root gets its grandparent
// in its low half.  A word read as a non-root can no longer be a root, so the
// halving stores never touch a word a compare-and-swap works on.  kCoherent:
// loads see every swap made so far (used after a failed swap).
template <bool kCoherent>
__device__ __forceinline__ uint32_t n_find_from(uint64_t* nodes, uint32_t x, uint64_t w, uint64_t* word,
                                                const SweepArgs& a) {
    for (uint32_t k = 0; !(lo32(w) & kNodeRoot); ++k) {
        if (k >= a.node_cap) {
            record_fault(a.ctl, kFaultGlobal);
            break;
        }
        const uint32_t p = min(lo32(w), a.node_cap - 1u);  // (clamped: a broken forest stays in bounds)
        const uint64_t wp = kCoherent ? n_load(&nodes[p]) : nodes[p];
        if (lo32(wp) & kNodeRoot) {
            *word = wp;
            return p;
        }
        reinterpret_cast<uint32_t*>(&nodes[x])[0] = lo32(wp);
        x = min(lo32(wp), a.node_cap - 1u);
        w = kCoherent ? n_load(&nodes[x]) : nodes[x];
    }
    *word = w;
    return x;
}

// Join the clusters of roots a and b (root words wa and wb).
__device__ void n_union_roots(uint64_t* nodes, uint32_t a, uint64_t wa, uint32_t b, uint64_t wb, const SweepArgs& args) {
    for (uint32_t k = 0; a != b; ++k) {
        if (k >= args.node_cap || !(lo32(wa) & lo32(wb) & kNodeRoot)) {  // a walk gave up: the forest is broken
            record_fault(args.ctl, kFaultGlobal);
            return;
        }
        if (hi32(wa) > hi32(wb)) {
            uint32_t tn = a;
            a = b;
            b = tn;
            const uint64_t tw = wa;
            wa = wb;
            wb = tw;
        }
        uint64_t expected = wb;
        const uint64_t link = (wb & 0xFFFFFFFF00000000ull) | a;
        if (__hip_atomic_compare_exchange_strong(&nodes[b], &expected, link, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        // the failed swap returned b's current word; a's first load is
        // issued before b's walk goes on
        const uint64_t wa0 = n_load(&nodes[a]);
        b = n_find_from<true>(nodes, b, expected, &wb, args);
        a = n_find_from<true>(nodes, a, wa0, &wa, args);
    }
}

// Node-forest ends of the bond that leaves tile (tx, row y) to the right, or
// tile (ty, column x) downwards.
__device__ __forceinline__ BorderBond vertical_node_bond(const SweepArgs& a, int tx, int y) {
    const int ty = y / kTileH, ly = y - ty * kTileH;
    const int t = ty * a.tiles_x + tx;
    const int tr = ty * a.tiles_x + ((tx + 1 == a.tiles_x) ? 0 : tx + 1);
    const uint64_t* m = a.border_bonds + static_cast<size_t>(t) * kBorderMasks;
    const uint64_t rr = m[kRightR], rd = m[kRightD];
    const uint64_t ld = a.border_bonds[static_cast<size_t>(tr) * kBorderMasks + kLeftD];
    const uint32_t si = a.border_slots[static_cast<size_t>(t) * (4 * kTileW) + 0 * kTileW + ly];
    const uint32_t sj = a.border_slots[static_cast<size_t>(tr) * (4 * kTileW) + 2 * kTileW + ly];
    const bool skip = ly != 0 && bit(rr, ly - 1) && bit(rd, ly - 1) && bit(ld, ly - 1);
    return {bit(rr, ly) && !skip, static_cast<uint32_t>(t) * kSlotsPerTile + si,
            static_cast<uint32_t>(tr) * kSlotsPerTile + sj};
}

__device__ __forceinline__ BorderBond horizontal_node_bond(const SweepArgs& a, int ty, int x) {
    const int tx = x / kTileW, lx = x - tx * kTileW;
    const int t = ty * a.tiles_x + tx;
    const int td = ((ty + 1 == a.tiles_y) ? 0 : ty + 1) * a.tiles_x + tx;
    const uint64_t* m = a.border_bonds + static_cast<size_t>(t) * kBorderMasks;
    const uint64_t bd = m[kBottomD], br = m[kBottomR];
    const uint64_t tr = a.border_bonds[static_cast<size_t>(td) * kBorderMasks + kTopR];
    const uint32_t si = a.border_slots[static_cast<size_t>(t) * (4 * kTileW) + 1 * kTileW + lx];
    const uint32_t sj = a.border_slots[static_cast<size_t>(td) * (4 * kTileW) + 3 * kTileW + lx];
    const bool skip = lx != 0 && bit(bd, lx - 1) && bit(br, lx - 1) && bit(tr, lx - 1);
    return {bit(bd, lx) && !skip, static_cast<uint32_t>(t) * kSlotsPerTile + si,
            static_cast<uint32_t>(td) * kSlotsPerTile + sj};
}

// Thread g: row g % L of vertical border g / L (every tile column's right
// edge), then column h % L of horizontal border h / L.
__device__ __forceinline__ void node_merge(const SweepArgs& a, uint32_t g) {
    if (!a.ctl->live) return;
    // every kernel that reads this sweep's index has run (stream order)
    if (g == 0) a.ctl->t += 1;
    const uint32_t L = static_cast<uint32_t>(a.L);
    const uint32_t nv = static_cast<uint32_t>(a.tiles_x) * L, nh = static_cast<uint32_t>(a.tiles_y) * L;
    BorderBond b = {false, 0u, 0u};
    if (g < nv) {
        const uint32_t k = g / L;
        b = vertical_node_bond(a, static_cast<int>(k), static_cast<int>(g - k * L));
    } else if (g - nv < nh) {
        const uint32_t h = g - nv, k = h / L;
        b = horizontal_node_bond(a, static_cast<int>(k), static_cast<int>(h - k * L));
    }
    uint32_t ra = 0, rb = 0;
    uint64_t wa = 0, wb = 0;
    if (b.active) {
        // the two first loads are issued together; most walks end there
        const uint64_t wi = a.nodes[b.i], wj = a.nodes[b.j];
        ra = n_find_from<false>(a.nodes, b.i, wi, &wa, a);
        rb = n_find_from<false>(a.nodes, b.j, wj, &wb, a);
        if (ra > rb) {
            const uint32_t tn = ra;
            ra = rb;
            rb = tn;
            const uint64_t tw = wa;
            wa = wb;
            wb = tw;
        }
    }
    if (wave_first(b.active && ra != rb, ra, rb)) n_union_roots(a.nodes, ra, wa, rb, wb, a);
}

// The last sweep's flip from its codes and merged node forest: one tile per
// workgroup, the tile's node draws (and keys) resolved once into LDS, then
// sixteen consecutive sites of a row per thread.  With kVerify the canonical
// labels follow: the tile-local root of an inner component's sites, the key
// of the cluster root for a perimeter component's.
template <bool kVerify>
__device__ __forceinline__ void code_flip(const SweepArgs& a, const int tx, const int ty) {
    __shared__ uint32_t val[kSlotsPerTile];
    __shared__ uint32_t key[kSlotsPerTile];
    if (!a.ctl->live) return;
    const int L = a.L;
    const uint32_t tile = static_cast<uint32_t>(ty * a.tiles_x + tx);
    const uint32_t ns = min(a.nslots[tile], kSlotsPerTile);
    for (uint32_t k = threadIdx.x; k < ns; k += blockDim.x) {
        const uint32_t n = tile * kSlotsPerTile + k;
        uint64_t w = a.nodes[n];
        for (uint32_t s = 0; !(lo32(w) & kNodeRoot); ++s) {
            if (s >= a.node_cap) {
                record_fault(a.ctl, kFaultFlip);
                w = kNodeRoot;
                break;
            }
            w = a.nodes[min(lo32(w), a.node_cap - 1u)];
        }
        val[k] = lo32(w) & 0xFFu;
        key[k] = hi32(w);
    }
    __syncthreads();
    const int ly = static_cast<int>(threadIdx.x >> 2), lx = static_cast<int>(threadIdx.x & 3) * 16;
    const int y = ty * kTileH + ly;
    const int xs = tx * kTileW + lx;
    const int nx = (y < L) ? max(0, min(16, L - xs)) : 0;
    if (nx == 0) return;
    const uint32_t base = __umul24(y, L) + static_cast<uint32_t>(xs);
    const int m = static_cast<int>(a.ctl->mirror);
    const bool full = (nx == 16) && ((base & 15u) == 0);
    uint32_t c[16];
    if (full) {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const uint4 v = *reinterpret_cast<const uint4*>(a.codes + base + 8 * g);
            c[8 * g] = v.x & 0xFFFFu; c[8 * g + 1] = v.x >> 16;
            c[8 * g + 2] = v.y & 0xFFFFu; c[8 * g + 3] = v.y >> 16;
            c[8 * g + 4] = v.z & 0xFFFFu; c[8 * g + 5] = v.z >> 16;
            c[8 * g + 6] = v.w & 0xFFFFu; c[8 * g + 7] = v.w >> 16;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) c[k] = (k < nx) ? a.codes[base + k] : 0u;
    }
    uint32_t out[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t ck = c[k];
        uint32_t v = ck & 31u;
        if (ck & kCodeNode) {
            const uint32_t d = val[ck & 0xFFu];
            v = (a.model == 1) ? static_cast<uint32_t>(flipped<true>(d, static_cast<int>((ck >> 8) & 31u), m, a.q)) : d;
        }
        out[k] = v;
    }
    if (full) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
            *reinterpret_cast<uint32_t*>(a.flip_out + base + 4 * g) =
                out[4 * g] | (out[4 * g + 1] << 8) | (out[4 * g + 2] << 16) | (out[4 * g + 3] << 24);
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (k < nx) a.flip_out[base + k] = static_cast<int8_t>(out[k]);
    }
    if (kVerify) {
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (k < nx) a.canon[base + k] = (c[k] & kCodeNode) ? key[c[k] & 0xFFu] : a.lroot[base + k];
    }
}

// After the merge: every tile-local root at the end of a border bond that
// has been linked is pointed straight at its cluster root, so that any site
// reaches the root word in at most two loads (site -> tile-local root ->
// root).  The walk halves the path on the way.
__device__ __forceinline__ void flatten_root(uint32_t* lab, uint32_t r, Control* ctl) {
    const uint32_t w = lab[r];
    if (w & kRootFlag) return;  // still a cluster root
    uint32_t x = w;
    uint32_t wx = lab[x];
    for (uint32_t n = 0; !(wx & kRootFlag); ++n) {
        if (n >= kGlobalWalkCap) {
            record_fault(ctl, kFaultGlobal);
            return;
        }
        const uint32_t w2 = lab[wx];
        if (w2 & kRootFlag) {
            x = wx;
            break;
        }
        lab[x] = w2;
        x = w2;
        wx = lab[x];
    }
    lab[r] = x;
}

// The same for a forest that only the flip reads: the linked tile-local root
// receives a copy of its cluster's root word, so that any site reaches a root
// word in at most two loads (site -> tile-local root).  Nothing else is
// written: a halving store could overwrite a copy another thread had just
// stored.  Every linked node is the end of some border bond, so every one of
// them is visited.
__device__ __forceinline__ void copy_root_word(uint32_t* lab, uint32_t r, uint32_t w, Control* ctl) {
    if (w & kRootFlag) return;  // a cluster root, or a copy already
    for (uint32_t n = 0; !(w & kRootFlag); ++n) {
        if (n >= kGlobalWalkCap) {
            record_fault(ctl, kFaultGlobal);
            return;
        }
        w = lab[w];
    }
    lab[r] = w;
}

__device__ __forceinline__ void flatten(const SweepArgs& a, const uint32_t block, const bool copies) {
    if (!a.ctl->live) return;
    // Every kernel that reads the sweep index has finished (stream order); the
    // flip only needs the mirror recorded by k_bond_local.
    if (block == 0 && threadIdx.x == 0) a.ctl->t += 1;
    const BorderBond b = border_bond(a, block * blockDim.x + threadIdx.x, 1);
    // a tile-local root that the previous lane also reaches is left to it
    // (a wave holds many distinct roots here, so a full per-wave
    // deduplication costs more than the repeated walks it saves)
    const uint32_t i = b.active ? b.i : kRootFlag, j = b.active ? b.j : kRootFlag;
    const uint32_t pi = __shfl_up(i, 1, 64), pj = __shfl_up(j, 1, 64);
    const bool first = (threadIdx.x & 63) == 0;
    const bool do_i = b.active && (first || pi != i), do_j = b.active && (first || pj != j);
    if (copies) {
        // both first loads are issued together (a lane without a walk reads
        // site 0 and discards it)
        const uint32_t wi = a.labels[do_i ? i : 0u], wj = a.labels[do_j ? j : 0u];
        if (do_i) copy_root_word(a.labels, i, wi, a.ctl);
        if (do_j) copy_root_word(a.labels, j, wj, a.ctl);
    } else {
        if (do_i) flatten_root(a.labels, i, a.ctl);
        if (do_j) flatten_root(a.labels, j, a.ctl);
    }
}

// ---------------------------------------------------------------------------
// Cluster flip.  One 64 x 64 tile per workgroup, sixteen sites per thread.
// When the lattice side is a multiple of four, thread t takes sixteen
// consecutive sites of tile row t/4 (vector loads and stores); otherwise lane
// l of wave v takes column l of tile rows 16v .. 16v+15, so that every access
// of a wave is one contiguous piece of a lattice row.  The tile's label words
// are staged in LDS, and every step of a path whose target lies in the tile
// reads LDS: an ordinary site's label word names its tile-local root, which
// is in the tile.  A tile-local root that was merged across tiles holds a
// link (after the flatten, straight to its cluster root, or a copy of the
// root word) that may leave the tile; such steps read global memory.
// ---------------------------------------------------------------------------
template <bool kVerify, bool rows4>
__device__ __forceinline__ void flip_tile(const SweepArgs& a, const int tx, const int ty, uint32_t* tl) {
    const int L = a.L;
    const uint32_t nrows = static_cast<uint32_t>(min(kTileH, L - ty * kTileH));
    const uint32_t ncols = static_cast<uint32_t>(min(kTileW, L - tx * kTileW));
    const uint32_t tile_base = __umul24(ty * kTileH, L) + static_cast<uint32_t>(tx * kTileW);
    const uint32_t t = threadIdx.x;
    const uint32_t ly = rows4 ? (t >> 2) : (t >> 6) * 16u;
    const uint32_t lx = rows4 ? (t & 3u) * 16u : (t & 63u);
    // sites k < n of the thread lie in the lattice: site k is at tile row
    // ly + k (column mapping) or column lx + k (row mapping)
    const uint32_t run = rows4 ? ncols : nrows, first = rows4 ? lx : ly;
    const bool on = rows4 ? (ly < nrows) : (lx < ncols);
    const int n = (on && first < run) ? static_cast<int>(min(16u, run - first)) : 0;
    const uint32_t step = rows4 ? 1u : static_cast<uint32_t>(L);  // lattice index step
    const uint32_t lstep = rows4 ? 1u : static_cast<uint32_t>(kTileW);
    const uint32_t base = n ? tile_base + __umul24(ly, L) + lx : 0u;
    const bool full = rows4 && n == 16;  // the row mapping's sixteen sites, 16-byte aligned words
    uint32_t x[16], w[16];
    if (full) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const uint4 v = *reinterpret_cast<const uint4*>(a.labels + base + 4 * g);
            w[4 * g] = v.x; w[4 * g + 1] = v.y; w[4 * g + 2] = v.z; w[4 * g + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) w[k] = (k < n) ? a.labels[base + k * step] : kRootFlag;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) tl[ly * kTileW + lx + k * lstep] = w[k];
    __syncthreads();
    // First step.  A target lies in the tile when its offset d from the
    // tile's first site is below nrows * L and d mod L is below the tile's
    // width; its row d / L comes from a float reciprocal corrected to the
    // exact quotient (such offsets stay below 2^22).
    const float inv_l = 1.0f / static_cast<float>(L);
    const uint32_t span = nrows * static_cast<uint32_t>(L);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        x[k] = base + k * step;
        if (!(w[k] & kRootFlag)) {
            x[k] = w[k];
            const uint32_t d = w[k] - tile_base;
            bool in_tile = d < span;
            uint32_t r = 0, c = 0;
            if (in_tile) {
                r = static_cast<uint32_t>(static_cast<float>(d) * inv_l);
                if (r * static_cast<uint32_t>(L) > d) r -= 1;
                else if (d - r * static_cast<uint32_t>(L) >= static_cast<uint32_t>(L)) r += 1;
                c = d - r * static_cast<uint32_t>(L);
                in_tile = c < ncols;
            }
            w[k] = in_tile ? tl[r * kTileW + c] : a.labels[x[k]];
        }
    }
    // Further steps (paths through merged roots), sixteen paths together.
    bool pending = true;
    for (uint32_t m = 0; pending; ++m) {
        if (m >= kGlobalWalkCap) {
            record_fault(a.ctl, kFaultFlip);
            break;
        }
        pending = false;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (!(w[k] & kRootFlag)) {
                x[k] = w[k];
                w[k] = a.labels[x[k]];
                pending = true;
            }
    }
    if (n == 0) return;
    uint32_t out[16];
    if (a.model == 0) {
#pragma unroll
        for (int k = 0; k < 16; ++k) out[k] = w[k] & 0xFFu;
    } else {
        const int m = static_cast<int>(a.ctl->mirror);
        uint32_t old[4] = {0u, 0u, 0u, 0u};  // the sixteen old spins, four to a word
        if (full && (base & 15u) == 0) {
            const uint4 v = *reinterpret_cast<const uint4*>(a.spins + base);
            old[0] = v.x; old[1] = v.y; old[2] = v.z; old[3] = v.w;
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k < n) old[k >> 2] |= static_cast<uint32_t>(static_cast<uint8_t>(a.spins[base + k * step])) << (8 * (k & 3));
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            int sp = static_cast<int>((old[k >> 2] >> (8 * (k & 3))) & 0xFFu);
            if (w[k] & 1u) {
                sp = m - sp;
                if (sp < 0) sp += a.q;
            }
            out[k] = static_cast<uint32_t>(sp);
        }
    }
    if (full) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            *reinterpret_cast<uint32_t*>(a.flip_out + base + 4 * g) =
                out[4 * g] | (out[4 * g + 1] << 8) | (out[4 * g + 2] << 16) | (out[4 * g + 3] << 24);
            if (kVerify)
                *reinterpret_cast<uint4*>(a.canon + base + 4 * g) = make_uint4(x[4 * g], x[4 * g + 1], x[4 * g + 2], x[4 * g + 3]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (k < n) {
                a.flip_out[base + k * step] = static_cast<int8_t>(out[k]);
                if (kVerify) a.canon[base + k * step] = x[k];
            }
    }
}

template <bool kVerify>
__device__ __forceinline__ void flip(const SweepArgs& a, const int tx, const int ty) {
    __shared__ uint32_t tl[kTileH * kTileW];
    if (!a.ctl->live) return;
    if ((a.L & 3) == 0)
        flip_tile<kVerify, true>(a, tx, ty, tl);
    else
        flip_tile<kVerify, false>(a, tx, ty, tl);
}

// ---------------------------------------------------------------------------
// Integer counts of the current state: n[k], the owned-bond histogram of
// (s_j - s_i) mod q, and for the clock model the correlation histograms of
// (s_{i+r} - s_i) mod q over both lattice directions at r = L/4 and L/2
// (Sec. 4).  Workgroup b takes rows b, b + nblocks, ...; thread t takes
// groups of four consecutive sites, packed one byte per site in a 32-bit word
// (the row, the row below, the right neighbours and the displaced sites), and
// four groups of a row are loaded before any is counted.  Potts q = 2 counts
// by popcounts of the packed words; q <= 8 in per-lane LDS bins; larger q by
// shared LDS atomics.  Each workgroup stores its bins to its own partial row
// (thousands of global atomics on the same few words would serialise) and
// one workgroup sums the partial rows.
// ---------------------------------------------------------------------------
constexpr int kCountThreads = 256;
constexpr int kGroupSpan = 4 * kCountThreads;  // sites of a row per step of the workgroup
constexpr int kGroups = 4;                     // steps of a row whose loads are issued together

struct Group4 {
    uint32_t w, wr, v;  // spins of four sites, of their right and lower neighbours
    uint32_t cx1, cy1, cx2, cy2;  // sites r = L/4 and L/2 to the right and below (clock model)
    int n;              // sites of the group inside the row (0..4)
};

// Four consecutive sites of the row at byte offset row, from column x on
// (columns wrap at L); n of them are wanted.
__device__ __forceinline__ uint32_t load4(const int8_t* spins, uint32_t row, int x, int L, int n, bool aligned) {
    if (aligned && n == 4 && (x & 3) == 0 && x + 3 < L) return *reinterpret_cast<const uint32_t*>(spins + row + x);
    uint32_t w = 0;
    for (int j = 0; j < n; ++j) {
        const int xj = (x + j < L) ? x + j : x + j - L;
        w |= static_cast<uint32_t>(static_cast<uint8_t>(spins[row + xj])) << (8 * j);
    }
    return w;
}

template <bool kCorr>
__device__ __forceinline__ Group4 load_group(const int8_t* spins, uint32_t here, uint32_t below, uint32_t far1,
                                             uint32_t far2, int x, int L, bool aligned, int first) {
    Group4 g{0u, 0u, 0u, 0u, 0u, 0u, 0u, max(0, min(4, L - x))};
    if (aligned && g.n == 4) {
        g.w = *reinterpret_cast<const uint32_t*>(spins + here + x);
        g.v = *reinterpret_cast<const uint32_t*>(spins + below + x);
        const uint32_t next = (x + 4 < L) ? static_cast<uint8_t>(spins[here + x + 4]) : static_cast<uint32_t>(first);
        g.wr = (g.w >> 8) | (next << 24);
    } else {
        for (int j = 0; j < g.n; ++j) {
            g.w |= static_cast<uint32_t>(static_cast<uint8_t>(spins[here + x + j])) << (8 * j);
            g.v |= static_cast<uint32_t>(static_cast<uint8_t>(spins[below + x + j])) << (8 * j);
            const uint32_t r = (x + j + 1 < L) ? static_cast<uint8_t>(spins[here + x + j + 1]) : static_cast<uint32_t>(first);
            g.wr |= r << (8 * j);
        }
    }
    if (kCorr && g.n > 0) {
        const int r1 = L / 4, r2 = L / 2;
        const int x1 = (x + r1 < L) ? x + r1 : x + r1 - L, x2 = (x + r2 < L) ? x + r2 : x + r2 - L;
        g.cx1 = load4(spins, here, x1, L, g.n, aligned);
        g.cx2 = load4(spins, here, x2, L, g.n, aligned);
        g.cy1 = load4(spins, far1, x, L, g.n, aligned);
        g.cy2 = load4(spins, far2, x, L, g.n, aligned);
    }
    return g;
}

// Calls f(group) for every group of four sites of this workgroup's rows.
template <bool kCorr, typename F>
__device__ __forceinline__ void for_groups(const SweepArgs& a, uint32_t block, uint32_t nblocks, F&& f) {
    const int L = a.L;
    const bool aligned = (L & 3) == 0;
    const int r1 = L / 4, r2 = L / 2;
    for (int y = static_cast<int>(block); y < L; y += static_cast<int>(nblocks)) {
        const uint32_t here = __umul24(y, L);
        const uint32_t below = __umul24((y + 1 == L) ? 0 : y + 1, L);
        const uint32_t far1 = kCorr ? __umul24((y + r1 < L) ? y + r1 : y + r1 - L, L) : 0u;
        const uint32_t far2 = kCorr ? __umul24((y + r2 < L) ? y + r2 : y + r2 - L, L) : 0u;
        const int first = static_cast<uint8_t>(a.spins[here]);  // right neighbour of the row's last site
        for (int xb = 0; xb < L; xb += kGroups * kGroupSpan) {
            Group4 g[kGroups];
#pragma unroll
            for (int u = 0; u < kGroups; ++u)
                g[u] = load_group<kCorr>(a.spins, here, below, far1, far2,
                                         xb + u * kGroupSpan + 4 * static_cast<int>(threadIdx.x), L, aligned, first);
#pragma unroll
            for (int u = 0; u < kGroups; ++u) f(g[u]);
        }
    }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Potts q = 2: bytes are 0 or 1, so a popcount of a packed word (or of the
// xor of two) counts ones (or unequal pairs) among its valid bytes.
__device__ __forceinline__ void count_q2(const SweepArgs& a, uint32_t block, uint32_t nblocks, uint32_t* h) {
    uint32_t sites = 0, ones = 0, diff = 0;
    for_groups<false>(a, block, nblocks, [&](const Group4& g) {
        const uint32_t m = (g.n >= 4) ? 0xFFFFFFFFu : ((1u << (8 * g.n)) - 1u);
        sites += static_cast<uint32_t>(g.n);
        ones += __popc(g.w & m);
        diff += __popc((g.w ^ g.wr) & m) + __popc((g.w ^ g.v) & m);
    });
    sites = wave_sum(sites);
    ones = wave_sum(ones);
    diff = wave_sum(diff);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&h[kRowHist + 0], sites - ones);
        atomicAdd(&h[kRowHist + 1], ones);
        atomicAdd(&h[kRowPair + 0], 2u * sites - diff);
        atomicAdd(&h[kRowPair + 1], diff);
    }
}

// q <= 8: every lane counts into bins of its own in LDS (bin b of lane l is
// word b * 64 + l of its wave's block, so no two lanes ever add to one word
// or one bank), and the workgroup folds them at the end.  Words 0-7: n[k]
// (low half); 8-15: pairs by (s_j - s_i) mod q, right neighbour in the low
// half, lower neighbour in the high half; 16-23 and 24-31: the correlation
// pairs at L/4 and L/2, x displacement low, y displacement high.  A lane
// adds at most 2^14 sites (L <= 65535 with 1024 workgroups of 256 threads),
// so 16-bit halves cannot overflow.  Differences are taken four at a time by
// byte-wise arithmetic on the packed words (no carries: every byte stays in
// 0 .. 2q - 1).
constexpr int kPrivHist = 0, kPrivPair = 8, kPrivCorr1 = 16, kPrivCorr2 = 24;
__host__ __device__ constexpr int priv_bins(bool corr) { return corr ? 32 : 16; }
constexpr int kCountWaves = kCountThreads / 64;

// (t - s) mod q in every byte of packed words t, s (bytes < q <= 8)
__device__ __forceinline__ uint32_t byte_diff_mod(uint32_t t, uint32_t s, uint32_t qq, uint32_t hi_q) {
    const uint32_t d = t + qq - s;                          // t - s + q in 1 .. 2q - 1
    const uint32_t ge = ((d + hi_q) >> 7) & 0x01010101u;    // 1 in the bytes where d >= q
    return d - ge * (qq & 0xFFu);
}

template <bool kCorr>
__device__ __forceinline__ void count_private(const SweepArgs& a, uint32_t block, uint32_t nblocks, uint32_t* h,
                                              uint32_t* bins) {
    constexpr int NB = priv_bins(kCorr);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < kCountWaves * NB * 64; k += kCountThreads) bins[k] = 0;
    __syncthreads();
    uint32_t* mine = bins + wave * NB * 64 + lane;
    const uint32_t q = static_cast<uint32_t>(a.q);
    const uint32_t qq = 0x01010101u * q, hi_q = 0x01010101u * (128u - q);
    for_groups<kCorr>(a, block, nblocks, [&](const Group4& g) {
        const uint32_t dr = byte_diff_mod(g.wr, g.w, qq, hi_q), dd = byte_diff_mod(g.v, g.w, qq, hi_q);
        uint32_t d1 = 0, e1 = 0, d2 = 0, e2 = 0;
        if (kCorr) {
            d1 = byte_diff_mod(g.cx1, g.w, qq, hi_q);
            e1 = byte_diff_mod(g.cy1, g.w, qq, hi_q);
            d2 = byte_diff_mod(g.cx2, g.w, qq, hi_q);
            e2 = byte_diff_mod(g.cy2, g.w, qq, hi_q);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j >= g.n) break;
            const int sh = 8 * j;
            atomicAdd(&mine[64 * (kPrivHist + ((g.w >> sh) & 0xFFu))], 1u);
            atomicAdd(&mine[64 * (kPrivPair + ((dr >> sh) & 0xFFu))], 1u);
            atomicAdd(&mine[64 * (kPrivPair + ((dd >> sh) & 0xFFu))], 0x10000u);
            if (kCorr) {
                atomicAdd(&mine[64 * (kPrivCorr1 + ((d1 >> sh) & 0xFFu))], 1u);
                atomicAdd(&mine[64 * (kPrivCorr1 + ((e1 >> sh) & 0xFFu))], 0x10000u);
                atomicAdd(&mine[64 * (kPrivCorr2 + ((d2 >> sh) & 0xFFu))], 1u);
                atomicAdd(&mine[64 * (kPrivCorr2 + ((e2 >> sh) & 0xFFu))], 0x10000u);
            }
        }
    });
    __syncthreads();
    // lane b of each wave adds word b over the wave's 64 lanes (both halves)
    // into the first word of the bin; then thread o < 4q adds the waves
    if (lane < static_cast<uint32_t>(NB)) {
        const uint4* row = reinterpret_cast<const uint4*>(bins + (wave * NB + lane) * 64);
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint4 v = row[k];
            sum += (v.x & 0xFFFFu) + (v.x >> 16) + (v.y & 0xFFFFu) + (v.y >> 16) + (v.z & 0xFFFFu) + (v.z >> 16) +
                   (v.w & 0xFFFFu) + (v.w >> 16);
        }
        bins[(wave * NB + lane) * 64] = sum;
    }
    __syncthreads();
    const int nout = kCorr ? 4 * static_cast<int>(q) : 2 * static_cast<int>(q);
    const int o = static_cast<int>(threadIdx.x);
    if (o < nout) {
        const int kind = o / static_cast<int>(q), d = o % static_cast<int>(q);  // hist, pairs, corr L/4, corr L/2
        uint32_t v = 0;
#pragma unroll
        for (int w = 0; w < kCountWaves; ++w) v += bins[(w * NB + 8 * kind + d) * 64];
        h[32 * kind + d] = v;  // kRowHist, kRowPair, kRowCorr1, kRowCorr2
    }
}

// q > 8: shared LDS bins and atomics.
__device__ __forceinline__ void count_lds(const SweepArgs& a, uint32_t block, uint32_t nblocks, uint32_t* h, bool corr) {
    const int q = a.q;
    auto delta = [q](uint32_t t, uint32_t s) -> int {
        const int d = static_cast<int>(t) - static_cast<int>(s);
        return d < 0 ? d + q : d;
    };
    auto body = [&](const Group4& g) {
        for (int j = 0; j < g.n; ++j) {
            const int sh = 8 * j;
            const uint32_t s = (g.w >> sh) & 0xFFu;
            atomicAdd(&h[kRowHist + s], 1u);
            atomicAdd(&h[kRowPair + delta((g.wr >> sh) & 0xFFu, s)], 1u);
            atomicAdd(&h[kRowPair + delta((g.v >> sh) & 0xFFu, s)], 1u);
            if (corr) {
                atomicAdd(&h[kRowCorr1 + delta((g.cx1 >> sh) & 0xFFu, s)], 1u);
                atomicAdd(&h[kRowCorr1 + delta((g.cy1 >> sh) & 0xFFu, s)], 1u);
                atomicAdd(&h[kRowCorr2 + delta((g.cx2 >> sh) & 0xFFu, s)], 1u);
                atomicAdd(&h[kRowCorr2 + delta((g.cy2 >> sh) & 0xFFu, s)], 1u);
            }
        }
    };
    if (corr)
        for_groups<true>(a, block, nblocks, body);
    else
        for_groups<false>(a, block, nblocks, body);
}

// Dynamic LDS of the count kernel: the per-lane bins of the q <= 8 path.
__host__ __device__ inline uint32_t count_lds_bytes(int q, int model) {
    if (model == 0 && q == 2) return 0u;
    if (q > 8) return 0u;
    return static_cast<uint32_t>(kCountWaves * priv_bins(model == 1) * 64 * 4);
}

__device__ __forceinline__ void counts(const SweepArgs& a, const uint32_t block, const uint32_t nblocks) {
    __shared__ uint32_t h[kRowWords];
    extern __shared__ uint32_t bins[];
    for (int k = threadIdx.x; k < kRowWords; k += blockDim.x) h[k] = 0;
    __syncthreads();
    const bool clock = a.model == 1;
    if (!clock && a.q == 2)
        count_q2(a, block, nblocks, h);
    else if (a.q > 8)
        count_lds(a, block, nblocks, h, clock);
    else if (clock)
        count_private<true>(a, block, nblocks, h, bins);
    else
        count_private<false>(a, block, nblocks, h, bins);
    __syncthreads();
    uint32_t* part = a.count_partial + static_cast<size_t>(block) * kRowWords;
    for (int k = threadIdx.x; k < kRowWords; k += blockDim.x) part[k] = h[k];
}

// Sum of the partial rows of the count workgroups into row[0..kRowWords):
// thread t adds partial rows t, t + blockDim, ... for every bin in use, a
// wave sum follows, and one LDS add per wave and bin.
constexpr int kCountSumThreads = 1024;

__device__ __forceinline__ void count_sum(const SweepArgs& a, int64_t* row) {
    __shared__ unsigned long long tot[kRowWords];
    for (int k = threadIdx.x; k < kRowWords; k += blockDim.x) tot[k] = 0;
    __syncthreads();
    const uint32_t nb = count_blocks(a.L);
    const int q = a.q;
    const int kinds = (a.model == 1) ? 4 : 2;  // hist, pairs (, correlations at L/4 and L/2)
    for (int k = 0; k < kinds * q; ++k) {
        const int bin = (k / q) * 32 + k % q;
        unsigned long long v = 0;
        for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) v += a.count_partial[static_cast<size_t>(b) * kRowWords + bin];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0) atomicAdd(&tot[bin], v);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kRowWords; k += blockDim.x) row[k] = static_cast<int64_t>(tot[k]);
}

// ---------------------------------------------------------------------------
// State hashes for checking long chains without dumping whole states:
// H_s = sum_i mix64((i << 8) | s_i) and H_l = sum_i mix64((i << 32) | l_i)
// mod 2^64, l_i the canonical label (smallest site index of i's cluster),
// with the SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014).
// Sums do not depend on the order of the sites, so any grid may compute them.
// Each workgroup writes its partial sums; one workgroup adds them.
// ---------------------------------------------------------------------------
constexpr int kHashThreads = 256;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ void hash_store_partial(uint64_t hs, uint64_t hl, uint64_t* part) {
    __shared__ uint64_t wsum[2][kHashThreads / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        hs += __shfl_xor(hs, off, 64);
        hl += __shfl_xor(hl, off, 64);
    }
    const int wave = static_cast<int>(threadIdx.x >> 6);
    if ((threadIdx.x & 63) == 0) {
        wsum[0][wave] = hs;
        wsum[1][wave] = hl;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint64_t v = 0;
        for (int w = 0; w < kHashThreads / 64; ++w) v += wsum[threadIdx.x][w];
        part[threadIdx.x] = v;
    }
}

// The sweep's new state and canonical labels, read from the forest after the
// border merge: every site walks to its cluster root (the root word carries
// the cluster's draw) and applies the flip the sweep decides, as k_flip does.
__device__ __forceinline__ void hash_sweep(const SweepArgs& a, uint32_t block, uint32_t nblocks) {
    if (!a.ctl->live) return;
    const uint32_t N = __umul24(a.L, a.L);
    const int m = a.model == 1 ? static_cast<int>(a.ctl->mirror) : 0;
    uint64_t hs = 0, hl = 0;
    bool broken = false;
    // (a 64-bit counter: with N close to 2^32 a 32-bit one would wrap past N)
    for (uint64_t i64 = block * kHashThreads + threadIdx.x; i64 < N; i64 += nblocks * kHashThreads) {
        const uint32_t i = static_cast<uint32_t>(i64);
        uint32_t x = i, w = a.labels[i];
        for (uint32_t n = 0; !(w & kRootFlag); ++n) {
            if (n >= kGlobalWalkCap) {
                broken = true;
                break;
            }
            x = w;
            w = a.labels[x];
        }
        int v;
        if (a.model == 0) {
            v = static_cast<int>(w & 0xFFu);
        } else {
            v = a.spins[i];
            if (w & 1u) {
                v = m - v;
                if (v < 0) v += a.q;
            }
        }
        hs += mix64((static_cast<uint64_t>(i) << 8) | static_cast<uint8_t>(v));
        hl += mix64((static_cast<uint64_t>(i) << 32) | x);
    }
    if (broken) record_fault(a.ctl, kFaultHash);
    hash_store_partial(hs, hl, a.hash_partial + 2 * static_cast<size_t>(block));
}

// Sum of the partial sums of nblocks workgroups into out[0..1].
__device__ __forceinline__ void hash_sum(const uint64_t* part, uint32_t nblocks, uint64_t* out) {
    uint64_t hs = 0, hl = 0;
    for (uint32_t b = threadIdx.x; b < nblocks; b += kHashThreads) {
        hs += part[2 * static_cast<size_t>(b)];
        hl += part[2 * static_cast<size_t>(b) + 1];
    }
    uint64_t tot[2];
    __shared__ uint64_t wsum[2][kHashThreads / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        hs += __shfl_xor(hs, off, 64);
        hl += __shfl_xor(hl, off, 64);
    }
    const int wave = static_cast<int>(threadIdx.x >> 6);
    if ((threadIdx.x & 63) == 0) {
        wsum[0][wave] = hs;
        wsum[1][wave] = hl;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        tot[threadIdx.x] = 0;
        for (int w = 0; w < kHashThreads / 64; ++w) tot[threadIdx.x] += wsum[threadIdx.x][w];
        out[threadIdx.x] = tot[threadIdx.x];
    }
}

// Per-sweep hashes from the codes, the tile-local roots and the merged node
// forest (before the next sweep overwrites them): the new state and the
// canonical labels, as hash_sweep computes them from a one-level forest.
__device__ __forceinline__ void code_hash(const SweepArgs& a, uint32_t block, uint32_t nblocks) {
    if (!a.ctl->live) return;
    const uint32_t N = __umul24(a.L, a.L);
    const int m = a.model == 1 ? static_cast<int>(a.ctl->mirror) : 0;
    uint64_t hs = 0, hl = 0;
    // (a 64-bit counter: with N close to 2^32 a 32-bit one would wrap past N)
    for (uint64_t i64 = block * kHashThreads + threadIdx.x; i64 < N; i64 += nblocks * kHashThreads) {
        const uint32_t i = static_cast<uint32_t>(i64);
        const uint32_t ck = a.codes[i];
        uint32_t v = ck & 31u, lab = a.lroot[i];
        if (ck & kCodeNode) {
            const uint32_t y = i / static_cast<uint32_t>(a.L), xx = i - y * static_cast<uint32_t>(a.L);
            const uint32_t tile = (y >> 6) * static_cast<uint32_t>(a.tiles_x) + (xx >> 6);
            uint64_t w = a.nodes[tile * kSlotsPerTile + (ck & 0xFFu)];
            for (uint32_t s = 0; !(lo32(w) & kNodeRoot); ++s) {
                if (s >= a.node_cap) {
                    record_fault(a.ctl, kFaultHash);
                    w = kNodeRoot;
                    break;
                }
                w = a.nodes[min(lo32(w), a.node_cap - 1u)];
            }
            const uint32_t d = lo32(w) & 0xFFu;
            v = (a.model == 1) ? static_cast<uint32_t>(flipped<true>(d, static_cast<int>((ck >> 8) & 31u), m, a.q)) : d;
            lab = hi32(w);
        }
        hs += mix64((static_cast<uint64_t>(i) << 8) | static_cast<uint8_t>(v));
        hl += mix64((static_cast<uint64_t>(i) << 32) | lab);
    }
    hash_store_partial(hs, hl, a.hash_partial + 2 * static_cast<size_t>(block));
}

__global__ void __launch_bounds__(kHashThreads) k_hash_sweep(SweepArgs a) { hash_sweep(a, blockIdx.x, gridDim.x); }

__global__ void __launch_bounds__(kHashThreads) k_hash_sum(SweepArgs a, uint32_t row) {
    if (!a.ctl->live) return;
    hash_sum(a.hash_partial, hash_blocks(a.L), a.hash_ring + 2 * static_cast<size_t>(row));
}

// Hashes of given arrays (H_l only when canon is given; 0 otherwise).
__global__ void __launch_bounds__(kHashThreads) k_hash_state(const int8_t* spins, const uint32_t* canon, uint32_t n,
                                                             uint64_t* part) {
    uint64_t hs = 0, hl = 0;
    for (uint64_t i64 = blockIdx.x * kHashThreads + threadIdx.x; i64 < n; i64 += gridDim.x * kHashThreads) {
        const uint32_t i = static_cast<uint32_t>(i64);
        hs += mix64((static_cast<uint64_t>(i) << 8) | static_cast<uint8_t>(spins[i]));
        if (canon) hl += mix64((static_cast<uint64_t>(i) << 32) | canon[i]);
    }
    hash_store_partial(hs, hl, part + 2 * static_cast<size_t>(blockIdx.x));
}

__global__ void __launch_bounds__(kHashThreads) k_hash_state_sum(const uint64_t* part, uint32_t nblocks, uint64_t* out) {
    hash_sum(part, nblocks, out);
}

// ---------------------------------------------------------------------------
// Entry points.  k_*: one lattice per launch.  kb_*: one launch covers every
// replica of a batch; workgroup b serves replica map[b], local block
// b - begin[replica].
// ---------------------------------------------------------------------------
// Workgroups go to the eight XCDs of the chip in turn (workgroup b to XCD
// b mod 8), and each XCD has its own L2.  Renumbering the tiles so that every
// XCD processes one contiguous run of them keeps neighbouring tiles, which
// share cache lines of the spin and label arrays, in the same L2.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t n) {
    return (n % kXcds) ? b : (b % kXcds) * (n / kXcds) + b / kXcds;
}

// kW waves per tile: 4 (16 rows each) for large lattices, 8 (8 rows each)
// where the lattice has too few tiles to fill the chip with 4-wave workgroups.
template <int kModel, int kW>
__global__ void __launch_bounds__(kW * 64) k_bond_local(SweepArgs a) {
    const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
    bond_tile<kModel, kFromSpins, kWriteLabels, kW>(a, static_cast<int>(t % a.tiles_x), static_cast<int>(t / a.tiles_x));
}

// Eight waves per SIMD (the scalar registers over the limit spill to vector
// lanes).
template <int kModel>
__global__ void __launch_bounds__(kBlock) k_bonds_only(SweepArgs a) {
    const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
    bond_tile<kModel, kFromSpins, kWriteBonds, kWaves>(a, static_cast<int>(t % a.tiles_x), static_cast<int>(t / a.tiles_x));
}

// Single lattices: the bond kernel with two-level labels, from the spins
// (a call's first sweep) or from the previous sweep's codes and node forest.
// Eight waves per SIMD: the register budget of that occupancy caps the
// scalar registers too, and the ones over the cap spill to vector lanes
// (leaving the scalar registers uncapped lowers the occupancy and costs more).
template <int kSrc, int kW>
__global__ void __launch_bounds__(kW * 64) __attribute__((amdgpu_waves_per_eu(8, 8))) k_code_bond_potts(SweepArgs a) {
    const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
    bond_tile<0, kSrc, kWriteCodes, kW>(a, static_cast<int>(t % a.tiles_x), static_cast<int>(t / a.tiles_x));
}

// The clock model's kernel keeps its tile's state in LDS, which allows seven
// workgroups per CU: seven waves per SIMD.
template <int kSrc, int kW>
__global__ void __launch_bounds__(kW * 64) __attribute__((amdgpu_waves_per_eu(7, 7))) k_code_bond_clock(SweepArgs a) {
    const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
    bond_tile<1, kSrc, kWriteCodes, kW>(a, static_cast<int>(t % a.tiles_x), static_cast<int>(t / a.tiles_x));
}

__global__ void __launch_bounds__(kMergeThreads) k_block_merge(SweepArgs a) { block_merge(a, blockIdx.x, blockIdx.y); }

// Workgroup order of the border kernels: thread g < nvb * L takes row g % L
// of vertical border g / L, the rest take the horizontal borders, 256 sites
// per workgroup.  When every workgroup lies within one border (L a multiple
// of 256) and both parts split evenly over the eight XCDs, each XCD takes one
// contiguous band of rows of the vertical borders and one contiguous run of
// the horizontal ones: the rows whose labels the bond kernel wrote on that
// XCD (tiles are numbered so that each XCD labels one contiguous run of tile
// rows), so the label loads of the walks tend to hit its L2.  The
// horizontal borders' workgroups are dispatched first: their walks are the
// longer ones (measured), and the vertical ones fill in behind them.
__device__ __forceinline__ uint32_t border_block(const SweepArgs& a, int step) {
    const uint32_t b = blockIdx.x, n = gridDim.x;
    const uint32_t L = static_cast<uint32_t>(a.L);
    if (L % 256u) return b;
    const uint32_t nvb = static_cast<uint32_t>((a.tiles_x + step - 1) / step);
    const uint32_t nhb = static_cast<uint32_t>((a.tiles_y + step - 1) / step);
    const uint32_t bands = L / 256u;
    const uint32_t nv = nvb * bands, nh = nhb * bands;
    if (n != nv + nh || nv % kXcds || nh % kXcds) return b;
    const uint32_t x = b % kXcds, i = b / kXcds, cv = nv / kXcds, ch = nh / kXcds;
    if (i >= ch) {
        const uint32_t v = x * cv + (i - ch);  // band-major: band v / nvb, border v % nvb
        return (v % nvb) * bands + v / nvb;
    }
    return nv + x * ch + i;
}

__global__ void __launch_bounds__(256) k_border_merge(SweepArgs a) {
    border_merge(a, border_block(a, a.merge_tiles) * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256) k_flatten(SweepArgs a) { flatten(a, border_block(a, 1), a.root_copies != 0); }

__global__ void __launch_bounds__(256) k_node_merge(SweepArgs a) {
    node_merge(a, border_block(a, 1) * blockDim.x + threadIdx.x);
}

template <bool kVerify>
__global__ void __launch_bounds__(256) k_code_flip(SweepArgs a) {
    const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
    code_flip<kVerify>(a, static_cast<int>(t % a.tiles_x), static_cast<int>(t / a.tiles_x));
}

__global__ void __launch_bounds__(kHashThreads) k_code_hash(SweepArgs a) { code_hash(a, blockIdx.x, gridDim.x); }

template <bool kVerify>
__global__ void __launch_bounds__(256) k_flip(SweepArgs a) {
    const uint32_t t = xcd_contiguous(blockIdx.x, gridDim.x);
    flip<kVerify>(a, static_cast<int>(t % a.tiles_x), static_cast<int>(t / a.tiles_x));
}

__global__ void __launch_bounds__(kCountThreads) k_counts(SweepArgs a) { counts(a, blockIdx.x, gridDim.x); }

__global__ void __launch_bounds__(kCountSumThreads) k_count_sum(SweepArgs a) { count_sum(a, a.count_row); }

// ---------------------------------------------------------------------------
// The paper's own labelers (Sec. 3), kept as an ablation of the union-find
// path.  Label equivalence after Hawick et al.: a scan lowers R[label] to the
// smallest label among a site's bonded neighbours (atomic minimum), an
// analysis resolves the chain of R at every site that labels itself, and a
// relabel sets label <- R[label].  After Kalentev et al.: one array, the scan
// lowers label[label] without atomics (a lost race is repaired by the next
// iteration), and the analysis resolves the chain at every site whose label
// does not label itself.  Every site starts with its own index; the iteration
// stops when a scan finds no bonded neighbour with a smaller label, and every
// site then holds the smallest index of its cluster.  Labels never exceed
// their index, so every chain walk ends.  One thread per site; workgroup
// (bx, y) takes 256 sites of row y.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool bond_bit(const uint64_t* m, int w64, int x, int y) {
    return (m[static_cast<size_t>(y) * w64 + (x >> 6)] >> (x & 63)) & 1ull;
}

__global__ void __launch_bounds__(256) k_le_init(SweepArgs a, uint32_t* R) {
    const int x = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x), y = static_cast<int>(blockIdx.y);
    if (x >= a.L) return;
    const uint32_t i = __umul24(y, a.L) + static_cast<uint32_t>(x);
    a.labels[i] = i;
    if (R) R[i] = i;
}

template <bool kHawick>
__global__ void __launch_bounds__(256) k_le_scan(SweepArgs a, uint32_t* R) {
    const int L = a.L;
    const int x = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x), y = static_cast<int>(blockIdx.y);
    if (x >= L) return;
    const uint32_t row = __umul24(y, L);
    const uint32_t l = a.labels[row + x];
    const int xl = (x == 0) ? L - 1 : x - 1, xr = (x + 1 == L) ? 0 : x + 1;
    const int yu = (y == 0) ? L - 1 : y - 1, yd = (y + 1 == L) ? 0 : y + 1;
    uint32_t m = l;
    if (bond_bit(a.bond_r, a.w64, x, y)) m = min(m, a.labels[row + xr]);
    if (bond_bit(a.bond_r, a.w64, xl, y)) m = min(m, a.labels[row + xl]);
    if (bond_bit(a.bond_d, a.w64, x, y)) m = min(m, a.labels[__umul24(yd, L) + x]);
    if (bond_bit(a.bond_d, a.w64, x, yu)) m = min(m, a.labels[__umul24(yu, L) + x]);
    if (m < l) {
        if (kHawick)
            atomicMin(&R[l], m);
        else if (m < a.labels[l])
            a.labels[l] = m;
        a.ctl->changed = 1u;
    }
}

// Hawick et al.: a site that labels itself resolves the chain of R from its index.
__global__ void __launch_bounds__(256) k_le_analysis_r(SweepArgs a, uint32_t* R) {
    const int x = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x), y = static_cast<int>(blockIdx.y);
    if (x >= a.L) return;
    const uint32_t i = __umul24(y, a.L) + static_cast<uint32_t>(x);
    if (a.labels[i] != i) return;
    uint32_t ref = R[i];
    for (uint32_t n = 0; ref != R[ref]; ++n) {
        if (n >= kGlobalWalkCap) {
            record_fault(a.ctl, kFaultGlobal);
            return;
        }
        ref = R[ref];
    }
    R[i] = ref;
}

__global__ void __launch_bounds__(256) k_le_relabel(SweepArgs a, const uint32_t* R) {
    const int x = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x), y = static_cast<int>(blockIdx.y);
    if (x >= a.L) return;
    const uint32_t i = __umul24(y, a.L) + static_cast<uint32_t>(x);
    a.labels[i] = R[a.labels[i]];
}

// Kalentev et al.: a site whose label does not label itself follows the chain.
__global__ void __launch_bounds__(256) k_le_analysis(SweepArgs a) {
    const int x = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x), y = static_cast<int>(blockIdx.y);
    if (x >= a.L) return;
    const uint32_t i = __umul24(y, a.L) + static_cast<uint32_t>(x);
    uint32_t l = a.labels[i];
    if (a.labels[l] == l) return;
    for (uint32_t n = 0; l != a.labels[l]; ++n) {
        if (n >= kGlobalWalkCap) {
            record_fault(a.ctl, kFaultGlobal);
            return;
        }
        l = a.labels[l];
    }
    a.labels[i] = l;
}

// After the last iteration: every site that labels itself (the smallest
// index of its cluster) receives its cluster's root word, so the flip reads
// labels exactly as after the union-find path.
__global__ void __launch_bounds__(256) k_le_roots(SweepArgs a) {
    const int x = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x), y = static_cast<int>(blockIdx.y);
    if (x >= a.L) return;
    const uint32_t i = __umul24(y, a.L) + static_cast<uint32_t>(x);
    if (a.labels[i] != i) return;
    uint32_t v;
    if (two_outcomes(a.model, a.q)) {
        const Words4 w = draw(i >> 7, a.ctl->t, kCluster, a.key0, a.key1);
        v = group_bit(w.w0, w.w1, w.w2, w.w3, i);
    } else {
        v = qmap(draw(i, a.ctl->t, kCluster, a.key0, a.key1).w0, static_cast<uint32_t>(a.q));
    }
    a.labels[i] = kRootFlag | v;
}

// The sweep index advances once nothing of the sweep reads it any more.
__global__ void k_le_advance(SweepArgs a) { a.ctl->t += 1; }

struct BatchMap {
    const SweepArgs* reps;  // replica table
    const uint32_t* map;    // workgroup -> replica
    const uint32_t* begin;  // replica -> its first workgroup in this launch
};

__device__ __forceinline__ uint32_t batch_replica(const BatchMap& m, uint32_t* local) {
    const uint32_t r = m.map[blockIdx.x];
    *local = blockIdx.x - m.begin[r];
    return r;
}

template <int kModel, int kW>
__global__ void __launch_bounds__(kW * 64) kb_bond_local(BatchMap m) {
    uint32_t local;
    const SweepArgs& a = m.reps[batch_replica(m, &local)];
    bond_tile<kModel, kFromSpins, kWriteLabels, kW>(a, static_cast<int>(local % a.tiles_x), static_cast<int>(local / a.tiles_x));
}

__global__ void __launch_bounds__(kMergeThreads) kb_block_merge(BatchMap m) {
    uint32_t local;
    const SweepArgs& a = m.reps[batch_replica(m, &local)];
    const int nbx = static_cast<int>(merge_blocks_x(a.tiles_x, a.merge_tiles));
    block_merge(a, static_cast<int>(local % nbx), static_cast<int>(local / nbx));
}

__global__ void __launch_bounds__(256) kb_border_merge(BatchMap m) {
    uint32_t local;
    const SweepArgs& a = m.reps[batch_replica(m, &local)];
    border_merge(a, local * blockDim.x + threadIdx.x);
}

// kCopies: root copies (a sweep whose labels only the flip reads); otherwise
// links straight to the cluster root, which a verify sweep's canonical
// labels need.
template <bool kCopies>
__global__ void __launch_bounds__(256) kb_flatten(BatchMap m) {
    uint32_t local;
    const SweepArgs& a = m.reps[batch_replica(m, &local)];
    flatten(a, local, kCopies);
}

template <bool kVerify>
__global__ void __launch_bounds__(256) kb_flip(BatchMap m) {
    uint32_t local;
    const SweepArgs& a = m.reps[batch_replica(m, &local)];
    flip<kVerify>(a, static_cast<int>(local % a.tiles_x), static_cast<int>(local / a.tiles_x));
}

__global__ void __launch_bounds__(kCountThreads) kb_counts(BatchMap m) {
    uint32_t local;
    const SweepArgs& a = m.reps[batch_replica(m, &local)];
    counts(a, local, count_blocks(a.L));
}

__global__ void __launch_bounds__(kCountSumThreads) kb_count_sum(BatchMap m, uint32_t row) {
    uint32_t local;
    const SweepArgs& a = m.reps[batch_replica(m, &local)];
    count_sum(a, a.count_row + static_cast<size_t>(row) * kRowWords);
}

__global__ void __launch_bounds__(kHashThreads) kb_hash(BatchMap m) {
    uint32_t local;
    const SweepArgs& a = m.reps[batch_replica(m, &local)];
    hash_sweep(a, local, hash_blocks(a.L));
}

__global__ void __launch_bounds__(kHashThreads) kb_hash_sum(BatchMap m, uint32_t row) {
    uint32_t local;
    const SweepArgs& a = m.reps[batch_replica(m, &local)];
    if (!a.ctl->live) return;
    hash_sum(a.hash_partial, hash_blocks(a.L), a.hash_ring + 2 * static_cast<size_t>(row));
}

}  // namespace

// Dynamic LDS of the clock bond kernels: the q x q cutoff slice.
size_t cut_bytes(int q) { return static_cast<size_t>(q) * q * sizeof(uint32_t); }

hipError_t launch_init(const SweepArgs& a, hipStream_t s) {
    const size_t N = static_cast<size_t>(a.L) * a.L;
    hipLaunchKernelGGL(k_init, dim3(static_cast<unsigned>((N + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int kW>
static void launch_bond_tiles(const SweepArgs& a, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(a.tiles_x) * static_cast<unsigned>(a.tiles_y));
    const dim3 block(kW * 64);
    if (a.model == 1)
        hipLaunchKernelGGL((k_bond_local<1, kW>), grid, block, cut_bytes(a.q), s, a);
    else
        hipLaunchKernelGGL((k_bond_local<0, kW>), grid, block, 0, s, a);
}

hipError_t launch_bond_local(const SweepArgs& a, hipStream_t s) {
    if (a.tile_waves == kWavesSmall)
        launch_bond_tiles<kWavesSmall>(a, s);
    else
        launch_bond_tiles<kWaves>(a, s);
    return hipGetLastError();
}

template <int kW>
static void launch_code_tiles(const SweepArgs& a, bool fused, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(a.tiles_x) * static_cast<unsigned>(a.tiles_y));
    const dim3 block(kW * 64);
    if (a.model == 1 && fused)
        hipLaunchKernelGGL((k_code_bond_clock<kFromCodes, kW>), grid, block, cut_bytes(a.q), s, a);
    else if (a.model == 1)
        hipLaunchKernelGGL((k_code_bond_clock<kFromSpins, kW>), grid, block, cut_bytes(a.q), s, a);
    else if (fused)
        hipLaunchKernelGGL((k_code_bond_potts<kFromCodes, kW>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_code_bond_potts<kFromSpins, kW>), grid, block, 0, s, a);
}

hipError_t launch_code_bond(const SweepArgs& a, bool fused, hipStream_t s) {
    if (a.tile_waves == kWavesSmall)
        launch_code_tiles<kWavesSmall>(a, fused, s);
    else
        launch_code_tiles<kWaves>(a, fused, s);
    return hipGetLastError();
}

hipError_t launch_node_merge(const SweepArgs& a, hipStream_t s) {
    const size_t n = (static_cast<size_t>(a.tiles_x) + a.tiles_y) * a.L;
    hipLaunchKernelGGL(k_node_merge, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_code_flip(const SweepArgs& a, bool verify, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(a.tiles_x) * static_cast<unsigned>(a.tiles_y));
    if (verify)
        hipLaunchKernelGGL(k_code_flip<true>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_code_flip<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_code_hash(const SweepArgs& a, uint32_t row, hipStream_t s) {
    hipLaunchKernelGGL(k_code_hash, dim3(hash_blocks(a.L)), dim3(kHashThreads), 0, s, a);
    hipLaunchKernelGGL(k_hash_sum, dim3(1), dim3(kHashThreads), 0, s, a, row);
    return hipGetLastError();
}

hipError_t launch_block_merge(const SweepArgs& a, hipStream_t s) {
    const int mt = a.merge_tiles;
    if (mt <= 1) return hipSuccess;
    hipLaunchKernelGGL(k_block_merge, dim3(merge_blocks_x(a.tiles_x, mt), merge_blocks_x(a.tiles_y, mt)),
                       dim3(kMergeThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_border_merge(const SweepArgs& a, hipStream_t s) {
    const unsigned nbx = static_cast<unsigned>((a.tiles_x + a.merge_tiles - 1) / a.merge_tiles);
    const unsigned nby = static_cast<unsigned>((a.tiles_y + a.merge_tiles - 1) / a.merge_tiles);
    const size_t n = (static_cast<size_t>(nbx) + nby) * a.L;
    hipLaunchKernelGGL(k_border_merge, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_flatten(const SweepArgs& a, hipStream_t s) {
    const size_t n = (static_cast<size_t>(a.tiles_x) + a.tiles_y) * a.L;
    hipLaunchKernelGGL(k_flatten, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_flip(const SweepArgs& a, bool verify, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(a.tiles_x) * static_cast<unsigned>(a.tiles_y));
    if (verify)
        hipLaunchKernelGGL(k_flip<true>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_flip<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bonds_only(const SweepArgs& a, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(a.tiles_x) * static_cast<unsigned>(a.tiles_y));
    if (a.model == 1)
        hipLaunchKernelGGL(k_bonds_only<1>, grid, dim3(kBlock), cut_bytes(a.q), s, a);
    else
        hipLaunchKernelGGL(k_bonds_only<0>, grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

static dim3 le_grid(const SweepArgs& a) { return dim3(static_cast<unsigned>((a.L + 255) / 256), static_cast<unsigned>(a.L)); }

hipError_t launch_le_init(const SweepArgs& a, uint32_t* R, hipStream_t s) {
    hipLaunchKernelGGL(k_le_init, le_grid(a), dim3(256), 0, s, a, R);
    return hipGetLastError();
}

hipError_t launch_le_iteration(const SweepArgs& a, int labeler, uint32_t* R, hipStream_t s) {
    if (labeler == kHawick) {
        hipLaunchKernelGGL(k_le_scan<true>, le_grid(a), dim3(256), 0, s, a, R);
        hipLaunchKernelGGL(k_le_analysis_r, le_grid(a), dim3(256), 0, s, a, R);
        hipLaunchKernelGGL(k_le_relabel, le_grid(a), dim3(256), 0, s, a, static_cast<const uint32_t*>(R));
    } else {
        hipLaunchKernelGGL(k_le_scan<false>, le_grid(a), dim3(256), 0, s, a, R);
        hipLaunchKernelGGL(k_le_analysis, le_grid(a), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_le_roots(const SweepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_le_roots, le_grid(a), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_le_advance, dim3(1), dim3(1), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_hash_sweep(const SweepArgs& a, uint32_t row, hipStream_t s) {
    hipLaunchKernelGGL(k_hash_sweep, dim3(hash_blocks(a.L)), dim3(kHashThreads), 0, s, a);
    hipLaunchKernelGGL(k_hash_sum, dim3(1), dim3(kHashThreads), 0, s, a, row);
    return hipGetLastError();
}

hipError_t launch_hash_state(const int8_t* spins, const uint32_t* canon, uint32_t n, uint64_t* part_and_out,
                             hipStream_t s) {
    // part_and_out: [blocks][2] partial sums, then the two results
    const uint32_t nb = hash_state_blocks(n);
    hipLaunchKernelGGL(k_hash_state, dim3(nb), dim3(kHashThreads), 0, s, spins, canon, n, part_and_out);
    hipLaunchKernelGGL(k_hash_state_sum, dim3(1), dim3(kHashThreads), 0, s, static_cast<const uint64_t*>(part_and_out),
                       nb, part_and_out + 2 * static_cast<size_t>(nb));
    return hipGetLastError();
}

hipError_t launch_counts(const SweepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_counts, dim3(count_blocks(a.L)), dim3(kCountThreads), count_lds_bytes(a.q, a.model), s, a);
    hipLaunchKernelGGL(k_count_sum, dim3(1), dim3(kCountSumThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace swmc

namespace swmc {

hipError_t launch_batch(BatchKernel k, const BatchLaunch& l, hipStream_t s, uint32_t row) {
    if (l.blocks == 0) return hipSuccess;
    const BatchMap m{l.reps, l.map, l.begin};
    const dim3 grid(l.blocks);
    switch (k) {
        case kBKBondPotts:
            if (l.waves == kWavesSmall)
                hipLaunchKernelGGL((kb_bond_local<0, kWavesSmall>), grid, dim3(kWavesSmall * 64), 0, s, m);
            else
                hipLaunchKernelGGL((kb_bond_local<0, kWaves>), grid, dim3(kWaves * 64), 0, s, m);
            break;
        case kBKBondClock:
            if (l.waves == kWavesSmall)
                hipLaunchKernelGGL((kb_bond_local<1, kWavesSmall>), grid, dim3(kWavesSmall * 64), cut_bytes(32), s, m);
            else
                hipLaunchKernelGGL((kb_bond_local<1, kWaves>), grid, dim3(kWaves * 64), cut_bytes(32), s, m);
            break;
        case kBKBlockMerge: hipLaunchKernelGGL(kb_block_merge, grid, dim3(kMergeThreads), 0, s, m); break;
        case kBKBorderMerge: hipLaunchKernelGGL(kb_border_merge, grid, dim3(256), 0, s, m); break;
        case kBKFlatten: hipLaunchKernelGGL(kb_flatten<false>, grid, dim3(256), 0, s, m); break;
        case kBKFlattenCopies: hipLaunchKernelGGL(kb_flatten<true>, grid, dim3(256), 0, s, m); break;
        case kBKFlip: hipLaunchKernelGGL(kb_flip<false>, grid, dim3(256), 0, s, m); break;
        case kBKFlipVerify: hipLaunchKernelGGL(kb_flip<true>, grid, dim3(256), 0, s, m); break;
        case kBKCounts: hipLaunchKernelGGL(kb_counts, grid, dim3(kCountThreads), count_lds_bytes(3, 1), s, m); break;
        case kBKCountSum: hipLaunchKernelGGL(kb_count_sum, grid, dim3(kCountSumThreads), 0, s, m, row); break;
        case kBKHash: hipLaunchKernelGGL(kb_hash, grid, dim3(kHashThreads), 0, s, m); break;
        case kBKHashSum: hipLaunchKernelGGL(kb_hash_sum, grid, dim3(kHashThreads), 0, s, m, row); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace swmc
