// Known-answer generator for the Philox pin: reads lines "c0 c1 c2 c3 k0 k1"
// from stdin and prints the four output words of rocRAND's Philox4x32-10
// engine for that counter and key (a library implementation of the SC'11
// generator, used here only to check the oracle's own implementation).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned int c[4], k[2];
    while (std::scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
        unsigned long long subseq = ((unsigned long long)c[3] << 32) | c[2];
        // The engine takes its counter as (subsequence, offset in words); set
        // counter word 0 through the offset and add word 1 in four steps so
        // that no 64-bit offset overflows.
        rocrand_device::philox4x32_10_engine eng(seed, subseq, 4ull * c[0]);
        for (int i = 0; i < 4; i++) eng.discard((unsigned long long)c[1] << 32);
        unsigned int a = eng(), b = eng(), d = eng(), e = eng();
        std::printf("%u %u %u %u\n", a, b, d, e);
    }
    return 0;
}
