// Device-side building blocks of the sweep: the counter-based generator and
// the uniform-to-state map.  Written for gfx950 from the published definitions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swmc {

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 products; the 64-bit products map to v_mad_u64_u32, and the key
// schedule depends only on the seed, so it stays in scalar registers.
__device__ __forceinline__ Words4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(pa >> 32) ^ c3 ^ k1;
        c1 = static_cast<uint32_t>(pb);
        c3 = static_cast<uint32_t>(pa);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// One draw of the sweep's stream: counter (c0, t mod 2^32, purpose, t >> 32).
__device__ __forceinline__ Words4 draw(uint32_t c0, uint64_t t, uint32_t purpose, uint32_t k0,
                                       uint32_t k1) {
    return philox10(c0, static_cast<uint32_t>(t), purpose, static_cast<uint32_t>(t >> 32), k0, k1);
}

// Uniform 32-bit word -> {0..q-1} by a multiply-shift.
__device__ __forceinline__ uint32_t qmap(uint32_t w, uint32_t q) {
    return static_cast<uint32_t>((static_cast<uint64_t>(w) * q) >> 32);
}

}  // namespace swmc
