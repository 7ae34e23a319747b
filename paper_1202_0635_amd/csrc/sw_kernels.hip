// HIP kernels of the Swendsen-Wang sweep for gfx950 (wave64, LDS union-find).
//
// One sweep = k_bond_local -> k_border_merge -> k_flip (Sec. 2 steps (1)-(3);
// the GPU organisation of Sec. 3 is replaced by a non-iterative union-find):
//   k_bond_local   per 64 x kTileH tile: FK bonds from Philox draws, row runs by
//                  wave ballots, vertical unions in an LDS forest, tile-local
//                  roots written to the global label forest; every tile-local
//                  root draws its cluster value now (a root that later loses
//                  the merge simply never gets read).
//   k_border_merge one thread per bond that leaves a tile or wraps around the
//                  torus: lock-free union of the two global roots, the larger
//                  index linked under the smaller by compare-and-swap.
//   k_flip         each site follows its forest path to the root word and
//                  takes the root's value (Potts) or reflection (clock).
#include "sw_device.hpp"
#include "sw_internal.hpp"

namespace swmc {

const char* const kKernelNames[kNumKernels] = {"k_bond_local", "k_border_merge", "k_flip", "k_counts"};

namespace {

__device__ __forceinline__ uint32_t lds_load(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x in the tile forest (parents always have smaller indices).
__device__ __forceinline__ uint32_t lds_find(uint32_t* P, uint32_t x) {
    uint32_t p = lds_load(&P[x]);
    while (p != x) {
        x = p;
        p = lds_load(&P[x]);
    }
    return x;
}

// Join the sets of a and b: the larger root is lowered to the smaller with an
// LDS atomic min; if that root had meanwhile been linked elsewhere, its old
// parent still has to be joined, so the loop continues with it.
__device__ __forceinline__ void lds_union(uint32_t* P, uint32_t a, uint32_t b) {
    while (true) {
        a = lds_find(P, a);
        b = lds_find(P, b);
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

// Root of x in the global forest; *word receives the root word.
__device__ __forceinline__ uint32_t g_find(const uint32_t* lab, uint32_t x, uint32_t* word) {
    uint32_t w = g_load(&lab[x]);
    while (!(w & kRootFlag)) {
        x = w;
        w = g_load(&lab[x]);
    }
    *word = w;
    return x;
}

__device__ void g_union(uint32_t* lab, uint32_t a, uint32_t b) {
    uint32_t wa, wb;
    a = g_find(lab, a, &wa);
    b = g_find(lab, b, &wb);
    while (a != b) {
        if (a > b) {
            uint32_t tmp = a;
            a = b;
            b = tmp;
            tmp = wa;
            wa = wb;
            wb = tmp;
        }
        // link root b under the smaller root a, if b is still a root
        uint32_t expected = wb;
        if (__hip_atomic_compare_exchange_strong(&lab[b], &expected, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        b = g_find(lab, b, &wb);
        a = g_find(lab, a, &wa);
    }
}

__device__ __forceinline__ int mirror_of(uint64_t t, int q, uint32_t k0, uint32_t k1) {
    return static_cast<int>(qmap(draw(0u, t, kMirror, k0, k1).w0, static_cast<uint32_t>(q)));
}

__device__ __forceinline__ uint32_t bond_bit(const uint64_t* bonds, int w64, int x, int y) {
    return static_cast<uint32_t>(bonds[static_cast<size_t>(y) * w64 + (x >> 6)] >> (x & 63)) & 1u;
}

// ---------------------------------------------------------------------------
// Random start: s_i = qmap(draw(i, 0, init)).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_init(SweepArgs a) {
    const size_t N = static_cast<size_t>(a.L) * a.L;
    const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const Words4 w = draw(static_cast<uint32_t>(i), 0, kInit, a.key0, a.key1);
    a.spins[i] = static_cast<int8_t>(qmap(w.w0, static_cast<uint32_t>(a.q)));
}

// ---------------------------------------------------------------------------
// Bonds + tile-local labeling.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_bond_local(SweepArgs a) {
    constexpr int RPW = kTileH / kWaves;  // rows per wave
    __shared__ uint32_t P[kTileH * kTileW];
    __shared__ uint64_t in_r[kTileH];
    __shared__ uint64_t in_d[kTileH];
    __shared__ uint32_t cut[32 * 32];
    __shared__ uint32_t roots[kWaves][RPW * kTileW];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int L = a.L, q = a.q;
    const int tx = blockIdx.x, ty = blockIdx.y;
    const int x0 = tx * kTileW, y0 = ty * kTileH;
    const int x = x0 + lane;
    const bool col_ok = x < L;
    const int xr = (x + 1 == L) ? 0 : x + 1;
    const int nvalid = min(kTileW, L - x0);
    // lanes whose right bond stays inside the tile (not the last column, no wrap)
    const uint64_t in_tile_r = (nvalid >= 64) ? (~0ull >> 1) : ((1ull << (nvalid - 1)) - 1ull);
    const uint64_t t = a.ctl->t;
    const uint32_t k0 = a.key0, k1 = a.key1;

    // Cutoff slice of this sweep: Potts C[a][b]; clock C[m][a][b] for the mirror m.
    const int m = (a.model == 1) ? mirror_of(t, q, k0, k1) : 0;
    const uint32_t* src = a.table + static_cast<size_t>(m) * q * q;
    for (int k = threadIdx.x; k < q * q; k += kBlock) cut[k] = src[k];
    __syncthreads();

    // Phase 1: bonds of the wave's rows, in groups of four rows per draw.
    for (int g = 0; g < RPW / 4; ++g) {
        const int ly0 = wave * RPW + g * 4;
        const int yb = y0 + ly0;  // multiple of 4
        Words4 hi = {0, 0, 0, 0};
        if (col_ok && yb < L)
            hi = draw(static_cast<uint32_t>((yb >> 2) * L + x), t, kBondHi, k0, k1);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int ly = ly0 + k;
            const int y = yb + k;
            const bool ok = col_ok && (y < L);
            bool br = false, bd = false;
            if (ok) {
                const int yd = (y + 1 == L) ? 0 : y + 1;
                const int s = a.spins[static_cast<size_t>(y) * L + x];
                const int sr = a.spins[static_cast<size_t>(y) * L + xr];
                const int sd = a.spins[static_cast<size_t>(yd) * L + x];
                const uint32_t cr = cut[s * q + sr];
                const uint32_t cd = cut[s * q + sd];
                const uint32_t w = (k == 0) ? hi.w0 : (k == 1) ? hi.w1 : (k == 2) ? hi.w2 : hi.w3;
                const uint32_t ur = w >> 16, ud = w & 0xFFFFu;
                br = ur < (cr >> 16);
                bd = ud < (cd >> 16);
                const bool tie_r = (ur == (cr >> 16)) && (cr & 0xFFFFu);
                const bool tie_d = (ud == (cd >> 16)) && (cd & 0xFFFFu);
                if (tie_r || tie_d) {
                    // low halves of the two uniforms, drawn only when needed
                    const uint32_t lo = draw(static_cast<uint32_t>(static_cast<size_t>(y) * L + x), t, kBondLo, k0, k1).w0;
                    br = br || (tie_r && (lo >> 16) < (cr & 0xFFFFu));
                    bd = bd || (tie_d && (lo & 0xFFFFu) < (cd & 0xFFFFu));
                }
            }
            const uint64_t mr = __ballot(br);
            const uint64_t md = __ballot(bd);
            if (lane == 0 && y < L) {
                a.bond_r[static_cast<size_t>(y) * a.w64 + tx] = mr;
                a.bond_d[static_cast<size_t>(y) * a.w64 + tx] = md;
            }
            const uint64_t ir = mr & in_tile_r;
            const uint64_t id = (ly + 1 < kTileH && y + 1 < L) ? md : 0ull;
            if (lane == 0) {
                in_r[ly] = ir;
                in_d[ly] = id;
            }
            // run start: the highest lane j <= lane with no in-tile bond from j-1 to j
            const uint64_t brk = ~(ir << 1);
            const int start = 63 - __clzll(brk & (~0ull >> (63 - lane)));
            P[ly * kTileW + lane] = static_cast<uint32_t>(ly * kTileW + start);
        }
    }
    __syncthreads();

    // Phase 2: vertical unions inside the tile.  A bond is skipped when the
    // lane to its left carries a vertical bond between the same two runs.
    for (int r = 0; r < RPW; ++r) {
        const int ly = wave * RPW + r;
        if (ly + 1 >= kTileH) break;
        const uint64_t d = in_d[ly];
        if (!((d >> lane) & 1ull)) continue;
        if (lane > 0 && ((d >> (lane - 1)) & 1ull) && ((in_r[ly] >> (lane - 1)) & 1ull) &&
            ((in_r[ly + 1] >> (lane - 1)) & 1ull))
            continue;
        lds_union(P, static_cast<uint32_t>(ly * kTileW + lane), static_cast<uint32_t>((ly + 1) * kTileW + lane));
    }
    __syncthreads();

    // Phase 3: tile-local roots -> global label forest.
    uint32_t nroots = 0;
    for (int r = 0; r < RPW; ++r) {
        const int ly = wave * RPW + r;
        const int y = y0 + ly;
        const bool ok = col_ok && (y < L);
        const uint32_t self = static_cast<uint32_t>(ly * kTileW + lane);
        const uint32_t root = ok ? lds_find(P, self) : self;
        const bool is_root = ok && (root == self);
        if (ok && !is_root) {
            const uint32_t g = static_cast<uint32_t>((y0 + static_cast<int>(root >> 6)) * L + x0 + static_cast<int>(root & 63));
            a.labels[static_cast<size_t>(y) * L + x] = g;
        }
        const uint64_t rm = __ballot(is_root);
        if (is_root) {
            const uint32_t pos = nroots + static_cast<uint32_t>(__popcll(rm & ((1ull << lane) - 1ull)));
            roots[wave][pos] = static_cast<uint32_t>(y * L + x);
        }
        nroots += static_cast<uint32_t>(__popcll(rm));
    }
    __syncthreads();
    // Every tile-local root draws its cluster's value (Sec. 3: a new value is
    // assigned to every label; here only to labels that are roots).
    for (uint32_t j = lane; j < nroots; j += 64) {
        const uint32_t i = roots[wave][j];
        const uint32_t w = draw(i, t, kCluster, k0, k1).w0;
        const uint32_t v = (a.model == 0) ? qmap(w, static_cast<uint32_t>(q)) : (w >> 31);
        a.labels[i] = kRootFlag | v;
    }
}

// ---------------------------------------------------------------------------
// Union across tile borders and the periodic wrap.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_border_merge(SweepArgs a) {
    const int L = a.L;
    const size_t nv = static_cast<size_t>(a.tiles_x) * L;
    const size_t nh = static_cast<size_t>(a.tiles_y) * L;
    const size_t gid = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid < nv) {
        // right edge of tile column tx, row y
        const int tx = static_cast<int>(gid / L);
        const int y = static_cast<int>(gid % L);
        const int xe = min((tx + 1) * kTileW, L) - 1;
        const int xr = (xe + 1 == L) ? 0 : xe + 1;
        if (!bond_bit(a.bond_r, a.w64, xe, y)) return;
        // redundant if row y-1 of the same tile row already joins the same two sets
        if ((y % kTileH) != 0 && bond_bit(a.bond_r, a.w64, xe, y - 1) && bond_bit(a.bond_d, a.w64, xe, y - 1) &&
            bond_bit(a.bond_d, a.w64, xr, y - 1))
            return;
        g_union(a.labels, static_cast<uint32_t>(y * L + xe), static_cast<uint32_t>(y * L + xr));
    } else if (gid < nv + nh) {
        const size_t h = gid - nv;
        const int ty = static_cast<int>(h / L);
        const int x = static_cast<int>(h % L);
        const int ye = min((ty + 1) * kTileH, L) - 1;
        const int yd = (ye + 1 == L) ? 0 : ye + 1;
        if (!bond_bit(a.bond_d, a.w64, x, ye)) return;
        if ((x % kTileW) != 0 && bond_bit(a.bond_d, a.w64, x - 1, ye) && bond_bit(a.bond_r, a.w64, x - 1, ye) &&
            bond_bit(a.bond_r, a.w64, x - 1, yd))
            return;
        g_union(a.labels, static_cast<uint32_t>(ye * L + x), static_cast<uint32_t>(yd * L + x));
    }
}

// ---------------------------------------------------------------------------
// Cluster flip; the last workgroup advances the sweep index.
// ---------------------------------------------------------------------------
template <bool kVerify>
__global__ void __launch_bounds__(256) k_flip(SweepArgs a) {
    const size_t N = static_cast<size_t>(a.L) * a.L;
    const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t t = a.ctl->t;
    if (i < N) {
        uint32_t x = static_cast<uint32_t>(i);
        uint32_t w = a.labels[i];
        while (!(w & kRootFlag)) {
            x = w;
            w = a.labels[x];
        }
        const uint32_t v = w & 0xFFu;
        if (a.model == 0) {
            a.spins[i] = static_cast<int8_t>(v);
        } else if (v) {
            const int m = mirror_of(t, a.q, a.key0, a.key1);
            int s = m - a.spins[i];
            if (s < 0) s += a.q;
            a.spins[i] = static_cast<int8_t>(s);
        }
        if (kVerify) a.canon[i] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t nblocks = gridDim.x;
        const uint32_t prev = atomicAdd(&a.ctl->done, 1u);
        if (prev == nblocks - 1) {
            a.ctl->done = 0;
            a.ctl->t = t + 1;
        }
    }
}

// ---------------------------------------------------------------------------
// Integer counts of the current state: n[k] and the owned-bond histogram of
// (s_j - s_i) mod q, accumulated into one int64 row.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_counts(SweepArgs a) {
    __shared__ uint32_t h[kRowWords];
    for (int k = threadIdx.x; k < kRowWords; k += blockDim.x) h[k] = 0;
    __syncthreads();
    const int L = a.L, q = a.q;
    const size_t N = static_cast<size_t>(L) * L;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < N;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const int y = static_cast<int>(i / L), x = static_cast<int>(i % L);
        const int s = a.spins[i];
        const int sr = a.spins[static_cast<size_t>(y) * L + ((x + 1 == L) ? 0 : x + 1)];
        const int sd = a.spins[static_cast<size_t>((y + 1 == L) ? 0 : y + 1) * L + x];
        int dr = sr - s, dd = sd - s;
        if (dr < 0) dr += q;
        if (dd < 0) dd += q;
        atomicAdd(&h[s], 1u);
        atomicAdd(&h[32 + dr], 1u);
        atomicAdd(&h[32 + dd], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kRowWords; k += blockDim.x)
        if (h[k]) atomicAdd(reinterpret_cast<unsigned long long*>(&a.count_row[k]), static_cast<unsigned long long>(h[k]));
}

}  // namespace

hipError_t launch_init(const SweepArgs& a, hipStream_t s) {
    const size_t N = static_cast<size_t>(a.L) * a.L;
    hipLaunchKernelGGL(k_init, dim3(static_cast<unsigned>((N + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bond_local(const SweepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_bond_local, dim3(a.tiles_x, a.tiles_y), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_border_merge(const SweepArgs& a, hipStream_t s) {
    const size_t n = (static_cast<size_t>(a.tiles_x) + a.tiles_y) * a.L;
    hipLaunchKernelGGL(k_border_merge, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_flip(const SweepArgs& a, bool verify, hipStream_t s) {
    const size_t N = static_cast<size_t>(a.L) * a.L;
    const dim3 grid(static_cast<unsigned>((N + 255) / 256));
    if (verify)
        hipLaunchKernelGGL(k_flip<true>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_flip<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_counts(const SweepArgs& a, hipStream_t s) {
    const size_t N = static_cast<size_t>(a.L) * a.L;
    size_t blocks = (N + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_counts, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace swmc
