// Host build of the device arithmetic header: the sum form of the lazy Shoup
// product (remainder a w + h (2^64 - q)) against the subtraction form and
// against a w mod q, for every modulus given on the command line, on edge
// operands and SplitMix64 samples.  Prints "ok <count>" or the first failure.
#include "modarith.hpp"
#include <cstdio>
#include <cstdlib>

static uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static bool check(uint64_t a, uint64_t w, uint64_t q) {
    const uint64_t wp = (uint64_t)(((u128)w << 64) / q);
    const uint64_t r = mul_shoup_lazy4(a, w, wp, q);
    const uint64_t rn = mul_shoup_lazy4n(a, w, wp, 0 - q);
    const uint64_t want = (uint64_t)(((u128)a * w) % q);
    if (r != rn || rn >= 4 * q || rn % q != want) {
        printf("fail q=%llu a=%llu w=%llu r=%llu rn=%llu want=%llu\n", (unsigned long long)q,
               (unsigned long long)a, (unsigned long long)w, (unsigned long long)r, (unsigned long long)rn,
               (unsigned long long)want);
        return false;
    }
    return true;
}

int main(int argc, char **argv) {
    uint64_t seed = 12201, count = 0;
    for (int i = 1; i < argc; i++) {
        const uint64_t q = strtoull(argv[i], nullptr, 10);
        const uint64_t edge_a[] = {0, 1, q - 1, q, 4 * q - 1, 8 * q - 1, ~0ull, 1ull << 63};
        const uint64_t edge_w[] = {0, 1, 2, q / 2, q - 1};
        for (uint64_t a : edge_a)
            for (uint64_t w : edge_w) {
                if (!check(a, w, q)) return 1;
                count++;
            }
        for (int j = 0; j < 200000; j++) {
            const uint64_t a = splitmix(seed), w = splitmix(seed) % q;
            if (!check(a, w, q)) return 1;
            count++;
        }
    }
    printf("ok %llu\n", (unsigned long long)count);
    return 0;
}
