// HIP kernels of the Swendsen-Wang sweep for gfx950 (wave64, LDS union-find).
//
// One sweep = k_bond_local -> k_border_merge -> k_flatten -> k_flip (Sec. 2
// steps (1)-(3);
// the GPU organisation of Sec. 3 is replaced by a non-iterative union-find):
//   k_bond_local   per 64 x kTileH tile: FK bonds from Philox draws, row runs by
//                  wave ballots, vertical unions in an LDS forest, tile-local
//                  roots written to the global label forest; every tile-local
//                  root draws its cluster value now (a root that later loses
//                  the merge simply never gets read).
//   k_border_merge one thread per bond that leaves a tile or wraps around the
//                  torus: lock-free union of the two global roots, the larger
//                  index linked under the smaller by compare-and-swap.
//   k_flatten      points every linked tile-local root straight at its root.
//   k_flip         each site follows its (now at most three-step) path to the
//                  root word and takes the root's value (Potts) or
//                  reflection (clock).
#include "sw_device.hpp"
#include "sw_internal.hpp"

namespace swmc {

const char* const kKernelNames[kNumKernels] = {"k_bond_local", "k_border_merge", "k_flatten", "k_flip", "k_counts"};

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

__device__ __forceinline__ void g_store(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x in the global forest; *word receives the root word.  Path
// halving: a visited non-root is pointed at its grandparent.  Only non-root
// words are rewritten and only with an ancestor's index, so a concurrent
// compare-and-swap (which targets root words) is never disturbed.
__device__ __forceinline__ uint32_t g_find(uint32_t* lab, uint32_t x, uint32_t* word) {
    uint32_t w = g_load(&lab[x]);
    while (!(w & kRootFlag)) {
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
// Bonds + tile-local labeling.  Lane = column, wave = kTileH/4 consecutive
// rows; each spin is loaded once (its right neighbour comes from the next
// lane, its lower neighbour from the next row held in registers).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_bond_local(SweepArgs a) {
    constexpr int RPW = kTileH / kWaves;  // rows per wave
    __shared__ uint32_t P[kTileH * kTileW];  // tile forest; afterwards each wave's root list
    __shared__ uint64_t in_r[kTileH];
    __shared__ uint64_t in_d[kTileH];
    __shared__ uint32_t cut[32 * 32];

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
    const bool clock = a.model == 1;

    // Cutoffs of this sweep: Potts needs only the equal-spin cutoff; the clock
    // model reads the q x q slice of its mirror m from LDS.
    const uint32_t c_eq = a.table[0];
    if (clock) {
        const int m = mirror_of(t, q, k0, k1);
        const uint32_t* src = a.table + static_cast<size_t>(m) * q * q;
        for (int k = threadIdx.x; k < q * q; k += kBlock) cut[k] = src[k];
        if (tx == 0 && ty == 0 && threadIdx.x == 0) a.ctl->mirror = static_cast<uint32_t>(m);
    }
    __syncthreads();

    const int ly_base = wave * RPW;
    const int y_base = y0 + ly_base;
    int sreg[RPW + 1];
#pragma unroll
    for (int r = 0; r <= RPW; ++r) {
        const int yr = y_base + r;  // yr == L is row 0 (the periodic neighbour of row L-1)
        sreg[r] = (col_ok && yr <= L) ? a.spins[static_cast<size_t>(yr == L ? 0 : yr) * L + x] : 0;
    }
    const bool edge_lane = (lane == nvalid - 1);

    // Phase 1: bonds of the wave's rows, four rows per draw.
#pragma unroll
    for (int g = 0; g < RPW / 4; ++g) {
        const int ly0 = ly_base + g * 4;
        const int yb = y0 + ly0;  // multiple of 4
        Words4 hi = {0, 0, 0, 0};
        if (col_ok && yb < L) hi = draw(static_cast<uint32_t>((yb >> 2) * L + x), t, kBondHi, k0, k1);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = g * 4 + k;
            const int ly = ly0 + k;
            const int y = yb + k;
            const bool ok = col_ok && (y < L);
            const int s = sreg[r];
            const int sd = sreg[r + 1];
            int sr = __shfl_down(s, 1, 64);
            if (ok && edge_lane) sr = a.spins[static_cast<size_t>(y) * L + xr];
            bool br = false, bd = false;
            if (ok) {
                uint32_t cr, cd;
                if (clock) {
                    cr = cut[s * q + sr];
                    cd = cut[s * q + sd];
                } else {
                    cr = (s == sr) ? c_eq : 0u;
                    cd = (s == sd) ? c_eq : 0u;
                }
                const uint32_t w = (k == 0) ? hi.w0 : (k == 1) ? hi.w1 : (k == 2) ? hi.w2 : hi.w3;
                const uint32_t ur = w >> 16, ud = w & 0xFFFFu;
                br = ur < (cr >> 16);
                bd = ud < (cd >> 16);
                const bool tie_r = (ur == (cr >> 16)) && (cr & 0xFFFFu);
                const bool tie_d = (ud == (cd >> 16)) && (cd & 0xFFFFu);
                if (tie_r || tie_d) {
                    // low halves of the two uniforms, drawn only when the high halves tie
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
        const int ly = ly_base + r;
        if (ly + 1 >= kTileH) break;
        const uint64_t d = in_d[ly];
        if (!((d >> lane) & 1ull)) continue;
        if (lane > 0 && ((d >> (lane - 1)) & 1ull) && ((in_r[ly] >> (lane - 1)) & 1ull) &&
            ((in_r[ly + 1] >> (lane - 1)) & 1ull))
            continue;
        lds_union(P, static_cast<uint32_t>(ly * kTileW + lane), static_cast<uint32_t>((ly + 1) * kTileW + lane));
    }
    __syncthreads();

    // Phase 3: tile-local roots.
    uint32_t rootreg[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const uint32_t self = static_cast<uint32_t>((ly_base + r) * kTileW + lane);
        rootreg[r] = (col_ok && y_base + r < L) ? lds_find(P, self) : self;
    }
    __syncthreads();
    uint32_t* list = P + ly_base * kTileW;  // this wave's slice of P holds its root list
    uint32_t nroots = 0;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int y = y_base + r;
        const bool ok = col_ok && (y < L);
        const uint32_t self = static_cast<uint32_t>((ly_base + r) * kTileW + lane);
        const uint32_t root = rootreg[r];
        const bool is_root = ok && (root == self);
        if (ok && !is_root)
            a.labels[static_cast<size_t>(y) * L + x] =
                static_cast<uint32_t>((y0 + static_cast<int>(root >> 6)) * L + x0 + static_cast<int>(root & 63));
        const uint64_t rm = __ballot(is_root);
        if (is_root) list[nroots + static_cast<uint32_t>(__popcll(rm & ((1ull << lane) - 1ull)))] =
            static_cast<uint32_t>(y * L + x);
        nroots += static_cast<uint32_t>(__popcll(rm));
    }
    __syncthreads();
    // Every tile-local root draws its cluster's value (Sec. 3 assigns a new
    // value to every label index; here only roots draw, one lane per root).
    for (uint32_t j = lane; j < nroots; j += 64) {
        const uint32_t i = list[j];
        const uint32_t w = draw(i, t, kCluster, k0, k1).w0;
        const uint32_t v = clock ? (w >> 31) : qmap(w, static_cast<uint32_t>(q));
        a.labels[i] = kRootFlag | v;
    }
}

// ---------------------------------------------------------------------------
// Bonds that leave a tile (or wrap around the torus).  Thread g < nv: right
// edge of tile column g / L, row g % L; otherwise bottom edge of a tile row.
// The bond is skipped when the neighbouring bond along the same border joins
// the same two tile-local sets (both its ends are tile-internal neighbours).
// ---------------------------------------------------------------------------
struct BorderBond {
    bool active;
    uint32_t i, j;
};

__device__ __forceinline__ BorderBond border_bond(const SweepArgs& a, size_t gid) {
    const int L = a.L;
    const size_t nv = static_cast<size_t>(a.tiles_x) * L;
    const size_t nh = static_cast<size_t>(a.tiles_y) * L;
    BorderBond b{false, 0u, 0u};
    if (gid < nv) {
        const int tx = static_cast<int>(gid / L);
        const int y = static_cast<int>(gid % L);
        const int xe = min((tx + 1) * kTileW, L) - 1;
        const int xr = (xe + 1 == L) ? 0 : xe + 1;
        if (!bond_bit(a.bond_r, a.w64, xe, y)) return b;
        if ((y % kTileH) != 0 && bond_bit(a.bond_r, a.w64, xe, y - 1) && bond_bit(a.bond_d, a.w64, xe, y - 1) &&
            bond_bit(a.bond_d, a.w64, xr, y - 1))
            return b;
        b = {true, static_cast<uint32_t>(y * L + xe), static_cast<uint32_t>(y * L + xr)};
    } else if (gid < nv + nh) {
        const size_t h = gid - nv;
        const int ty = static_cast<int>(h / L);
        const int x = static_cast<int>(h % L);
        const int ye = min((ty + 1) * kTileH, L) - 1;
        const int yd = (ye + 1 == L) ? 0 : ye + 1;
        if (!bond_bit(a.bond_d, a.w64, x, ye)) return b;
        if ((x % kTileW) != 0 && bond_bit(a.bond_d, a.w64, x - 1, ye) && bond_bit(a.bond_r, a.w64, x - 1, ye) &&
            bond_bit(a.bond_r, a.w64, x - 1, yd))
            return b;
        b = {true, static_cast<uint32_t>(ye * L + x), static_cast<uint32_t>(yd * L + x)};
    }
    return b;
}

__global__ void __launch_bounds__(256) k_border_merge(SweepArgs a) {
    const BorderBond b = border_bond(a, static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x);
    if (b.active) g_union(a.labels, b.i, b.j);
}

// After the merge: every linked tile-local root at the end of a border bond
// is pointed straight at its cluster root, so that any site reaches the root
// word in at most three loads (site -> tile-local root -> root).
__device__ __forceinline__ void flatten_from(uint32_t* lab, uint32_t e) {
    uint32_t w = lab[e];
    uint32_t r = e;
    if (!(w & kRootFlag)) {
        r = w;
        w = lab[r];
    }
    if (w & kRootFlag) return;  // the tile-local root is still a cluster root
    uint32_t x = w;             // walk to the root, halving the path on the way
    uint32_t wx = lab[x];
    while (!(wx & kRootFlag)) {
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

__global__ void __launch_bounds__(256) k_flatten(SweepArgs a) {
    // Every kernel that reads the sweep index has finished (stream order); the
    // flip only needs the mirror recorded by k_bond_local.
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->t += 1;
    const BorderBond b = border_bond(a, static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x);
    if (!b.active) return;
    flatten_from(a.labels, b.i);
    flatten_from(a.labels, b.j);
}

// ---------------------------------------------------------------------------
// Cluster flip, four sites per thread.
// ---------------------------------------------------------------------------
template <bool kVerify>
__global__ void __launch_bounds__(256) k_flip(SweepArgs a) {
    const size_t N = static_cast<size_t>(a.L) * a.L;
    const size_t base = (static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x) * 4;
    const bool clock = a.model == 1;
    if (base < N) {
        const int n = (N - base >= 4) ? 4 : static_cast<int>(N - base);
        uint32_t x[4], w[4];
        if (n == 4) {
            const uint4 v = *reinterpret_cast<const uint4*>(a.labels + base);
            w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        } else {
            for (int k = 0; k < 4; ++k) w[k] = (k < n) ? a.labels[base + k] : kRootFlag;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = static_cast<uint32_t>(base + k);
        // follow the four paths together (independent loads in flight)
        while (!((w[0] & w[1] & w[2] & w[3]) & kRootFlag)) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (!(w[k] & kRootFlag)) {
                    x[k] = w[k];
                    w[k] = a.labels[x[k]];
                }
        }
        uint32_t out[4];
        if (!clock) {
#pragma unroll
            for (int k = 0; k < 4; ++k) out[k] = w[k] & 0xFFu;
        } else {
            const int m = static_cast<int>(a.ctl->mirror);
            for (int k = 0; k < 4; ++k) {
                int s = (k < n) ? a.spins[base + k] : 0;
                if (w[k] & 1u) {
                    s = m - s;
                    if (s < 0) s += a.q;
                }
                out[k] = static_cast<uint32_t>(s);
            }
        }
        if (n == 4) {
            *reinterpret_cast<uint32_t*>(a.spins + base) = out[0] | (out[1] << 8) | (out[2] << 16) | (out[3] << 24);
            if (kVerify) *reinterpret_cast<uint4*>(a.canon + base) = make_uint4(x[0], x[1], x[2], x[3]);
        } else {
            for (int k = 0; k < n; ++k) {
                a.spins[base + k] = static_cast<int8_t>(out[k]);
                if (kVerify) a.canon[base + k] = x[k];
            }
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

hipError_t launch_flatten(const SweepArgs& a, hipStream_t s) {
    const size_t n = (static_cast<size_t>(a.tiles_x) + a.tiles_y) * a.L;
    hipLaunchKernelGGL(k_flatten, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_flip(const SweepArgs& a, bool verify, hipStream_t s) {
    const size_t N = static_cast<size_t>(a.L) * a.L;
    const dim3 grid(static_cast<unsigned>((N + 1023) / 1024));
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
