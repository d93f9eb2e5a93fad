// Prints Philox4x32-10 output words computed by rocRAND's own engine, run on the
// host CPU, for counters and keys read from stdin ("c0 c1 c2 c3 k0 k1" per line).
// The engine is positioned so that its next block is exactly philox(counter, key):
// key = the seed's two words; counter words 2,3 = the subsequence; words 0,1 =
// the number of 4-word blocks skipped (skipped in four equal parts plus a
// remainder, so that the skip count in words never overflows 64 bits).
// Used by the tests to pin the oracle's generator to a library.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (static_cast<unsigned long long>(k1) << 32) | k0;
        unsigned long long subsequence = (static_cast<unsigned long long>(c3) << 32) | c2;
        unsigned long long blocks = (static_cast<unsigned long long>(c1) << 32) | c0;
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, 0ull);
        for (int part = 0; part < 4; ++part)
            eng.discard((blocks / 4ull) * 4ull);
        eng.discard((blocks % 4ull) * 4ull);
        uint4 w = eng.next4();
        std::printf("%u %u %u %u\n", w.x, w.y, w.z, w.w);
    }
    return 0;
}
