// Independent Philox4x32-10 pin: rocRAND's engine (header-only source),
// run on the host. Reads lines "c0 c1 c2 c3 k0 k1" and prints 4 words.
// The engine's counter is set through its public seeding interface:
// key = seed, counter = (offset/4 low, high, subsequence low, high).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
        unsigned long long offset = (((unsigned long long)c1 << 32) | c0) * 4ull;
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        unsigned a = eng(), b = eng(), c = eng(), d = eng();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
