// Independent Philox4x32-10 implementation for pinning the oracle: drives
// rocRAND's philox4x32_10 engine through its public seed / subsequence /
// offset interface.  Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin and
// prints the four output words (hex) of the block with that counter and key.
//
// Mapping (rocRAND engine semantics): key = (lo32(seed), hi32(seed));
// the subsequence fills counter words 2..3 and offset/4 fills words 0..1.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        rocrand_device::philox4x32_10_engine e(seed, sub, 0ULL);
        // advance the block counter by whole blocks (4 words each): c0 blocks,
        // then c1 * 2^32 blocks in four quarter steps so no offset overflows
        e.discard((unsigned long long)c0 * 4ULL);
        for (int q = 0; q < 4; ++q) e.discard((unsigned long long)c1 << 32);
        uint4 r = e.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
