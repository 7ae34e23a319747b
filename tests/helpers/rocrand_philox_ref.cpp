// Test helper: evaluates Philox4x32-10 through rocRAND's own engine, so the
// oracle's generator can be checked against an implementation it shares no
// code with.  rocRAND's engine keys Philox with the 64-bit seed (low word
// first); seed(seed, subsequence, offset) puts the subsequence in counter
// words 2..3 and offset/4 in words 0..1.  Host-only; needs no GPU.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>

extern "C" void rr_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const unsigned long long seed = (unsigned long long)key[0] | ((unsigned long long)key[1] << 32);
    const unsigned long long subsequence = (unsigned long long)ctr[2] | ((unsigned long long)ctr[3] << 32);
    const unsigned long long block = (unsigned long long)ctr[0] | ((unsigned long long)ctr[1] << 32);
    rocrand_device::philox4x32_10_engine eng(seed, subsequence, 0);
    // Advance to the requested 128-bit block; offset counts 32-bit outputs, so
    // the block count is added in pieces that keep block*4 within 64 bits.
    unsigned long long remaining = block;
    while (remaining != 0) {
        const unsigned long long piece = remaining < (1ull << 61) ? remaining : (1ull << 61);
        eng.discard(piece * 4ull);
        remaining -= piece;
    }
    uint4 r = eng.next4();
    out[0] = r.x; out[1] = r.y; out[2] = r.z; out[3] = r.w;
}
