// Internal declarations shared by the HIP kernels and the host runtime of
// libswmc.  Nothing here crosses the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swmc {

// Tile of the bond + local-labeling kernel: 64 columns (one per lane of a
// wave64) by kTileH rows; a workgroup of 4 waves, each wave owning
// kTileH / 4 consecutive rows.
constexpr int kTileW = 64;
constexpr int kTileH = 64;
constexpr int kWaves = 4;
constexpr int kBlock = kWaves * 64;
// Lattices with fewer tiles than kSmallTiles split each tile over
// kWavesSmall waves of 8 rows instead, for more waves per CU.
constexpr int kWavesSmall = 8;
constexpr int kSmallTiles = 3072;
// Merge schedule (a per-context parameter, see the autotuner): 1 runs one
// device-wide border kernel; 2 or 4 first join the inner borders of blocks of
// that many tiles per side inside one workgroup (in LDS).
constexpr int kMergeTiles = 4;
// Threads of a first-level merge workgroup.
constexpr int kMergeThreads = 1024;

// Random-number purposes (third counter word of a Philox draw).
constexpr uint32_t kBondHi = 0;
constexpr uint32_t kBondLo = 1;
constexpr uint32_t kCluster = 2;
constexpr uint32_t kMirror = 3;
constexpr uint32_t kInit = 4;

// Root marker in the label array: a word with this bit set belongs to a
// cluster root and carries the cluster's draw (Potts: new value; clock: the
// reflection bit) in its low bits; any other word is the index of a site of
// the same cluster with a smaller index.
constexpr uint32_t kRootFlag = 0x80000000u;

constexpr int kRing = 1024;      // per-sweep count rows kept on the device

// Step bounds of the forest walks.  Every link points to a smaller index, so
// a correct forest ends every walk in fewer steps than it has nodes; a walk
// that takes more has met a broken forest, records a fault bit in the
// control block and stops, so a kernel never loops on it.
constexpr uint32_t kLdsWalkCap = kTileW * kTileH;       // a tile forest in LDS (4096 nodes)
constexpr uint32_t kGlobalWalkCap = 1u << 22;           // the global forest
enum FaultBits : uint32_t { kFaultLds = 1u, kFaultGlobal = 2u, kFaultFlip = 4u, kFaultHash = 8u };

// Two-level labels of single lattices.  Per site, a 16-bit code: a site
// whose tile-local component stays off the tile's perimeter holds its new
// value (bit 15 clear); any other site holds kCodeNode | slot (bits 0-7),
// plus (clock model) its old value in bits 8-12.  The components that reach
// a tile's perimeter (at most 252 per tile) are the nodes of a global forest:
// node tile * kSlotsPerTile + slot is a 64-bit word whose high half is the
// component's smallest site index (its key) and whose low half is either
// kNodeRoot | draw (a cluster root) or the index of a node with a smaller key.
constexpr uint32_t kSlotsPerTile = 256;
constexpr uint32_t kCodeNode = 0x8000u;
constexpr uint32_t kNodeRoot = 0x80000000u;
// Largest side of a single lattice (site indices stay below 2^32); batches,
// the server, the static entry point and the label-equivalence labelers keep
// root flags in 32-bit label words and stop at kMaxSideFlagged.
constexpr int kMaxSide = 65535;
constexpr int kMaxSideFlagged = 46340;

// Per-tile border record written by the bond kernel.  Edge e of border_roots:
// 0 right column, 1 bottom row, 2 left column, 3 top row (the last valid
// column / row of a ragged tile).  Masks: bit = row (columns) or column (rows).
enum BorderMask {
    kRightR = 0,   // right bonds of the right column (they leave the tile)
    kRightD = 1,   // down bonds of the right column
    kLeftD = 2,    // down bonds of the left column
    kBottomD = 3,  // down bonds of the bottom row (they leave the tile)
    kBottomR = 4,  // right bonds of the bottom row
    kTopR = 5,     // right bonds of the top row
    kBorderMasks = 8
};
// int64 per count row: hist[32], pair_hist[32], and for the clock model the
// correlation histograms at r = L/4 and L/2 (Sec. 4)
constexpr int kRowWords = 128;
constexpr int kRowHist = 0, kRowPair = 32, kRowCorr1 = 64, kRowCorr2 = 96;

// Device control block at the start of the arena.
struct Control {
    uint64_t t;       // sweep index of the current state
    uint64_t target;  // sweeps stop once t reaches this (all ones: never)
    uint32_t mirror;  // clock model: mirror index of the sweep in progress
    uint32_t live;    // the sweep in progress runs (t < target when it started)
    uint32_t changed; // label-equivalence labelers: a scan found a smaller label
    uint32_t fault;   // nonzero: a forest walk exceeded its step bound (kFault* bits); the
                      // kernel that saw it gave up its walks, the host reports SW_EDEVICE
    uint32_t pad[8];
};
static_assert(sizeof(Control) == 64, "control block is one 64-byte line");

struct SweepArgs {
    int8_t* spins;        // [N] the state the bond kernel reads (and the fused kernel writes)
    int8_t* flip_out;     // [N] where k_flip writes the new state (usually spins)
    uint64_t* bond_r;     // [L][w64]: bit x%64 of word x/64 = right bond of (x,y)
    uint64_t* bond_d;     // [L][w64]: down bonds
    uint32_t* labels;     // [N] union-find forest with root words (kRootFlag)
    uint32_t* canon;      // [N] canonical labels (verify mode)
    const uint32_t* table;// cutoff table (Potts q*q; clock q^3)
    Control* ctl;
    int64_t* count_row;   // destination row of the count kernel (or null)
    uint32_t* count_partial;  // [count_blocks(L)][kRowWords]: each count workgroup's bins
    uint32_t* border_roots;   // [tiles][4][64]: tile-local root (site index) of each edge site
    uint64_t* border_bonds;   // [tiles][kBorderMasks]: the bond bits the border joins read
    // two-level labels (single lattices; the previous sweep's arrays are read
    // by the fused kernel)
    uint16_t* codes;              // [N] per-site codes of this sweep
    const uint16_t* codes_prev;   // [N] the previous sweep's
    uint64_t* nodes;              // [tiles][kSlotsPerTile] this sweep's node forest
    const uint64_t* nodes_prev;
    uint32_t* nslots;             // [tiles] nodes per tile
    const uint32_t* nslots_prev;
    uint8_t* border_slots;        // [tiles][4][64] slot of each perimeter site (edges as border_roots)
    uint32_t* lroot;              // [N] or null: tile-local root (site index) of every site
    int8_t* spins_out;            // or null: the fused kernel also stores the state it computed
    uint32_t node_cap;            // nodes of the forest: a walk longer than this met a broken forest
    uint64_t* hash_ring;      // [kRing][2]: per-sweep state hashes (spins, canonical labels)
    uint64_t* hash_partial;   // [hash_blocks(L)][2]: each hash workgroup's sums
    int L, q, model, w64;
    int tiles_x, tiles_y;
    int tile_waves;       // waves per bond-kernel workgroup: kWaves or kWavesSmall (single
                          // lattices; batched launches always use kWaves)
    int merge_tiles;      // tiles per side of a first-level merge block (1: no block level)
    int root_copies;      // single lattices: k_flatten stores the cluster's root word (not a link) at every linked
                          // tile-local root: the labels then lead to a root word in at most two
                          // loads, but no longer name the root site (off in verify mode);
                          // batched launches pick the flatten kernel per sweep instead
    uint32_t key0, key1;
};

// Launch wrappers (defined in sw_kernels.hip).
hipError_t launch_init(const SweepArgs& a, hipStream_t s);
hipError_t launch_bond_local(const SweepArgs& a, hipStream_t s);
// Two-level labels: the bond kernel writing codes and nodes (fused: from the
// previous sweep's codes and node forest instead of spins), the merge of the
// node forests across tile borders (also advances the sweep index), the last
// sweep's flip into flip_out (and canonical labels into canon when verify),
// and the per-sweep hashes read from codes, lroot and the merged forest.
hipError_t launch_code_bond(const SweepArgs& a, bool fused, hipStream_t s);
hipError_t launch_node_merge(const SweepArgs& a, hipStream_t s);
hipError_t launch_code_flip(const SweepArgs& a, bool verify, hipStream_t s);
hipError_t launch_code_hash(const SweepArgs& a, uint32_t row, hipStream_t s);
hipError_t launch_block_merge(const SweepArgs& a, hipStream_t s);
hipError_t launch_border_merge(const SweepArgs& a, hipStream_t s);
hipError_t launch_flatten(const SweepArgs& a, hipStream_t s);
hipError_t launch_flip(const SweepArgs& a, bool verify, hipStream_t s);
hipError_t launch_counts(const SweepArgs& a, hipStream_t s);
// Per-sweep state hashes, run after the border merge of a sweep (before the
// flatten): the new state (the flip this sweep decides) and its canonical
// labels, summed into hash_ring[row] (which must hold zeros).
hipError_t launch_hash_sweep(const SweepArgs& a, uint32_t row, hipStream_t s);
// Hashes of given arrays: spins[n] and, if canon is not null, canon[n].
// part_and_out holds kHashPartWords words: the partial sums of up to 1024
// workgroups, then the two results (at 2 * blocks, 2 * blocks + 1 with
// blocks = hash_state_blocks(n)).
hipError_t launch_hash_state(const int8_t* spins, const uint32_t* canon, uint32_t n, uint64_t* out, hipStream_t s);
constexpr size_t kHashPartWords = 2 * 1024 + 2;
__host__ __device__ inline uint32_t hash_state_blocks(uint64_t n) {
    const uint64_t want = (n + 1023) / 1024;
    return want == 0 ? 1u : (want < 1024 ? static_cast<uint32_t>(want) : 1024u);
}
__host__ __device__ inline uint32_t hash_blocks(int L) {
    const uint64_t n = (static_cast<uint64_t>(L) * L + 1023) / 1024;
    return static_cast<uint32_t>(n < 1024 ? n : 1024);
}
// The paper's labelers (Sec. 3) as an ablation: bonds only, then label
// equivalence iterations, then root words at the sites that label themselves.
enum Labeler { kUnionFind = 0, kHawick = 1, kKalentev = 2 };
hipError_t launch_bonds_only(const SweepArgs& a, hipStream_t s);
hipError_t launch_le_init(const SweepArgs& a, uint32_t* R, hipStream_t s);
// one iteration: scan (+ analysis, + relabel for Hawick et al.)
hipError_t launch_le_iteration(const SweepArgs& a, int labeler, uint32_t* R, hipStream_t s);
hipError_t launch_le_roots(const SweepArgs& a, hipStream_t s);

// Workgroups of each launch for one lattice.
__host__ __device__ inline uint32_t count_blocks(int L) {
    const uint64_t n = (static_cast<uint64_t>(L) * L + 255) / 256;
    return static_cast<uint32_t>(n < 1024 ? n : 1024);
}
__host__ __device__ inline uint32_t merge_blocks_x(int tiles_x, int mt) {
    return mt > 0 ? static_cast<uint32_t>((tiles_x + mt - 1) / mt) : 0u;
}

// Batched launches: one launch covers the workgroups of every replica.
enum BatchKernel {
    kBKBondPotts, kBKBondClock, kBKBlockMerge, kBKBorderMerge, kBKFlatten, kBKFlattenCopies, kBKFlip, kBKFlipVerify,
    kBKCounts, kBKCountSum, kBKHash, kBKHashSum, kNumBatchKernels
};
struct BatchLaunch {
    const SweepArgs* reps;  // device replica table
    const uint32_t* map;    // device: workgroup -> replica
    const uint32_t* begin;  // device: replica -> first workgroup of this launch
    uint32_t blocks;        // workgroups of the launch
    int waves;              // bond kernels: waves per tile (kWaves or kWavesSmall)
};
hipError_t launch_batch(BatchKernel k, const BatchLaunch& l, hipStream_t s, uint32_t row);

enum KernelId {
    kKBondLocal, kKBlockMerge, kKBorderMerge, kKFlatten, kKFlip, kKCounts, kKFlipBond,
    kKBondsOnly, kKLeIteration, kKLeRoots, kKHash,
    kKCodeBond, kKCodeFlipBond, kKNodeMerge, kKCodeFlip, kNumKernels
};
extern const char* const kKernelNames[kNumKernels];

}  // namespace swmc
