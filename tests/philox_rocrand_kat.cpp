// Known-answer generator for the Philox4x32-10 pin: evaluates rocRAND's
// host-callable philox4x32_10_engine (an implementation written by another
// project) on (counter, key) pairs read from stdin, one
// "c0 c1 c2 c3 k0 k1" line each, and prints the four output words.
// The engine's counter is (offset/4 split over words 0-1, subsequence split
// over words 2-3), its key the 64-bit seed, so with offset = 4*(c0 | c1<<32)
// and subsequence = c2 | c3<<32 its first block is Philox(counter, key).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
