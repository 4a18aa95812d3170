// Host-side cross-check of the oracle's Philox4x32-10 block function against
// rocRAND's open-source philox4x32_10 engine.  Reads lines "c0 c1 c2 c3 k0 k1"
// (c1 < 2^30) and prints the engine's first four outputs for that state:
// seed = k0 | k1 << 32, subsequence = c2 | c3 << 32, offset = 4 (c0 | c1 << 32)
// puts the engine's counter at exactly (c0, c1, c2, c3).
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, offset, &st);
        unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
