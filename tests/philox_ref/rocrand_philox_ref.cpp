// Test-only host program: prints Philox4x32-10 outputs computed by ROCm's
// open-source rocrand device/host header, for counters and keys read from stdin
// (one "c0 c1 c2 c3 k0 k1" line each). Used to cross-check the oracle's own
// Philox implementation; nothing in the library or the oracle includes it.
#include <cstdio>
#include <cstdint>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subsequence = ((unsigned long long)c3 << 32) | c2;
        unsigned long long offset = 4ull * (((unsigned long long)c1 << 32) | c0);
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
        unsigned a = eng(), b = eng(), c = eng(), d = eng();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
