// sw_sweep_static: Swendsen-Wang sweeps of one lattice with no device
// allocation, for callers that cannot allocate (code under HIP graph
// capture, serving loops, harnesses that forbid hipMalloc).
//
// The state is the caller's device spin array; every intermediate array of
// the sweep (label forest, bond masks, border records, control block) lives
// in one file-scope device buffer of fixed size, `scratch`, which each GPU
// holds until the process ends.  The kernels are the ones sw_sweep runs for
// the first sweep of a call: bonds and tile labeling, the device-wide border
// merge (merge schedule 1), the flatten and the flip into the spin array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sw.h"
#include "sw_host.hpp"
#include "sw_internal.hpp"

using namespace swmc;
using namespace swmc::host;

namespace {

// Largest lattice side the buffer is sized for.
constexpr int kStaticMaxL = 1024;
constexpr size_t kUp = 256;
constexpr size_t up_c(size_t v) { return (v + kUp - 1) / kUp * kUp; }
constexpr size_t tiles_of(size_t L) { return ((L + kTileW - 1) / kTileW) * ((L + kTileH - 1) / kTileH); }

// Offsets of the parts of the buffer for a lattice of side L.
struct StaticLayout {
    size_t ctl, labels, bond_r, bond_d, border_roots, border_bonds, total;
};
constexpr StaticLayout static_layout(size_t L) {
    StaticLayout s{};
    const size_t N = L * L, w64 = (L + 63) / 64, tiles = tiles_of(L);
    size_t o = 0;
    s.ctl = o; o += up_c(sizeof(Control));
    s.labels = o; o += up_c(N * 4);
    s.bond_r = o; o += up_c(L * w64 * 8);
    s.bond_d = o; o += up_c(L * w64 * 8);
    s.border_roots = o; o += up_c(tiles * 4 * kTileW * 4);
    s.border_bonds = o; o += up_c(tiles * kBorderMasks * 8);
    s.total = o;
    return s;
}
constexpr size_t kScratchBytes = static_layout(kStaticMaxL).total;
static_assert(kScratchBytes == SW_STATIC_SCRATCH_BYTES, "sw.h states the buffer size");

// One copy per GPU.  In host code this name is a host-side stand-in, never a
// device address: host code uses the address hipGetSymbolAddress returned.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void* g_scratch[kMaxDevices] = {};
hipError_t g_status[kMaxDevices] = {};

// The buffer's device address on the current device (looked up once per device).
hipError_t scratch_address(int dev, char** out) {
    std::call_once(g_once[dev], [dev] {
        void* ptr = nullptr;
        g_status[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch[dev] = ptr;
    });
    *out = static_cast<char*>(g_scratch[dev]);
    if (g_status[dev] != hipSuccess) return g_status[dev];
    return *out ? hipSuccess : hipErrorInvalidSymbol;
}

// A fresh control block at sweep index t (no sweep target, no fault): the
// buffer keeps whatever the previous call left there.
__global__ void k_static_control(Control* ctl, uint64_t t) {
    ctl->t = t;
    ctl->target = ~0ull;
    ctl->mirror = 0u;
    ctl->live = 1u;
    ctl->changed = 0u;
    ctl->fault = 0u;
}

__global__ void k_static_fault(const Control* ctl, uint32_t* out) { *out = ctl->fault; }

}  // namespace

extern "C" int sw_sweep_static(const sw_lattice* p, int8_t* spins, uint64_t t, int32_t nsweeps,
                               const uint32_t* table, int32_t* labels, uint32_t* fault, void* stream) {
    std::string why;
    if (!lattice_ok(p, &why)) return fail(SW_EINVAL, "%s", why.c_str());
    if (p->L > kStaticMaxL)
        return fail(SW_EINVAL, "sw_sweep_static: L = %d exceeds the static buffer's maximum %d", p->L, kStaticMaxL);
    if (!spins || !table) return fail(SW_EINVAL, "sw_sweep_static: spins and table must be device pointers");
    // the flip moves spins and labels sixteen bytes at a time
    if (reinterpret_cast<uintptr_t>(spins) % 16 || reinterpret_cast<uintptr_t>(labels) % 16 ||
        reinterpret_cast<uintptr_t>(table) % 4)
        return fail(SW_EINVAL, "sw_sweep_static: spins and labels must be 16-byte aligned, table 4-byte aligned");
    if (nsweeps < 0) return fail(SW_EINVAL, "nsweeps must be >= 0");
    if (labels && nsweeps == 0) return fail(SW_EINVAL, "sw_sweep_static: labels need at least one sweep");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SW_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(SW_EDEVICE, "device index %d beyond %d", dev, kMaxDevices);
    char* base = nullptr;
    e = scratch_address(dev, &base);
    if (e != hipSuccess) return fail(SW_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    const hipStream_t s = static_cast<hipStream_t>(stream);

    const StaticLayout lay = static_layout(static_cast<size_t>(p->L));
    SweepArgs a{};
    a.spins = spins;
    a.flip_out = spins;
    a.labels = reinterpret_cast<uint32_t*>(base + lay.labels);
    a.canon = reinterpret_cast<uint32_t*>(labels);
    a.bond_r = reinterpret_cast<uint64_t*>(base + lay.bond_r);
    a.bond_d = reinterpret_cast<uint64_t*>(base + lay.bond_d);
    a.border_roots = reinterpret_cast<uint32_t*>(base + lay.border_roots);
    a.border_bonds = reinterpret_cast<uint64_t*>(base + lay.border_bonds);
    a.ctl = reinterpret_cast<Control*>(base + lay.ctl);
    a.table = table;
    a.L = p->L;
    a.q = p->q;
    a.model = p->model;
    a.w64 = (p->L + 63) / 64;
    a.tiles_x = (p->L + kTileW - 1) / kTileW;
    a.tiles_y = (p->L + kTileH - 1) / kTileH;
    a.tile_waves = (a.tiles_x * a.tiles_y < kSmallTiles) ? kWavesSmall : kWaves;
    a.merge_tiles = 1;
    a.key0 = static_cast<uint32_t>(p->seed);
    a.key1 = static_cast<uint32_t>(p->seed >> 32);

    hipLaunchKernelGGL(k_static_control, dim3(1), dim3(1), 0, s, a.ctl, t);
    e = hipGetLastError();
    for (int32_t k = 0; k < nsweeps && e == hipSuccess; ++k) {
        const bool verify = labels && k == nsweeps - 1;
        e = launch_bond_local(a, s);
        if (e == hipSuccess) e = launch_border_merge(a, s);
        a.root_copies = verify ? 0 : 1;
        if (e == hipSuccess) e = launch_flatten(a, s);
        if (e == hipSuccess) e = launch_flip(a, verify, s);
    }
    if (e == hipSuccess && fault) {
        hipLaunchKernelGGL(k_static_fault, dim3(1), dim3(1), 0, s, static_cast<const Control*>(a.ctl), fault);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return fail(SW_EDEVICE, "sw_sweep_static: %s", hipGetErrorString(e));
    return SW_OK;
}
