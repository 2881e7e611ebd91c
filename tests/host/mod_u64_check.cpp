// Host check of the exact 64-bit remainder used by the initialization draws:
// compares mod_u64 with the integer % on edge cases and pseudo-random inputs.
#include <cstdio>
#include <cstdint>

#include "cq_internal.h"

static uint64_t next(uint64_t& s)  // splitmix64 as a plain input generator
{
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int main()
{
    long bad = 0, n = 0;
    auto check = [&](uint64_t r, uint64_t T) {
        ++n;
        if (cq::mod_u64(r, T) != r % T) {
            if (bad < 5) std::printf("mismatch r=%llu T=%llu\n", (unsigned long long)r, (unsigned long long)T);
            ++bad;
        }
    };
    const uint64_t edge_r[] = {0ull, 1ull, 2ull, 0xFFFFFFFFull, 0x100000000ull, (1ull << 53) - 1, 1ull << 53,
                               (1ull << 53) + 1, (1ull << 63) - 1, 1ull << 63, ~0ull - 1, ~0ull};
    for (uint64_t T = 1; T < 5000; ++T)
        for (uint64_t r : edge_r) {
            check(r, T);
            check(0ull - T, T);
        }
    uint64_t s = 12345;
    for (int k = 0; k < 4000000; ++k) {
        const uint64_t r = next(s);
        const int bits = 1 + int(next(s) % 64);
        uint64_t T = next(s) >> (64 - bits);
        if (T == 0) T = 1;
        check(r, T);
        check(0ull - T, T);
        check(r, (T >> 1) + 1);
    }
    std::printf("%ld checks, %ld mismatches\n", n, bad);
    return bad == 0 ? 0 : 1;
}
