// Reference Philox4x32-10 words from rocRAND's header-only engine (host side).
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) on stdin and prints the four
// output words for counter (c0..c3) and key (k0, k1).  The engine is seeded
// with seed = k0 | k1 << 32, subsequence = c2 | c3 << 32 and offset
// 4 * (c0 | c1 << 32), which places its counter at (c0, c1, c2, c3).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long sub = c2 | (c3 << 32);
        unsigned long long off = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine eng(seed, sub, off);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
