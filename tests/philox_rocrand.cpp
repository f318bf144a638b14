// Host-side Philox4x32-10 outputs from rocRAND's engine, used as an
// independent check of the oracle's generator.  Reads "c0 c1 c2 c3 k0 k1"
// lines on stdin and prints the four output words.  rocRAND's engine state
// (seed, subsequence, offset) maps to key = (seed_lo, seed_hi),
// counter = (offset/4 as words 0-1, subsequence as words 2-3).
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main()
{
    unsigned int c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        rocrand_device::philox4x32_10_engine eng(seed, sub, 0);
        // advance the counter by c0 + c1*2^32 blocks of four outputs
        eng.discard(4ull * c0);
        for (int i = 0; i < 4; i++) eng.discard((unsigned long long)c1 << 32);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
