// Host program that evaluates rocRAND's Philox4x32-10 engine (an independent implementation,
// compiled from the installed open-source header) on counters read from stdin.
// Input lines: seed c0 c1 c2 c3 (decimal).  Output lines: four uint32 words (decimal).
// rocRAND's engine maps (seed, subsequence, offset) to key = (lo32 seed, hi32 seed) and
// counter = (lo32(offset/4), hi32(offset/4), lo32(subsequence), hi32(subsequence)).
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        unsigned long long offset = 4ull * (c0 | (c1 << 32));
        unsigned long long sub = c2 | (c3 << 32);
        rocrand_device::philox4x32_10_engine eng(seed, sub, offset);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
