// Host-only helper for the oracle's Philox pin: reads lines
// "key0 key1 c0 c1 c2 c3" (hex) on stdin and prints rocRAND's
// Philox4x32-10 output words for that key and counter, using rocRAND's own
// engine (an implementation independent of the oracle).  rocRAND's engine
// keys on the 64-bit seed, puts the 64-bit subsequence in counter words 2-3
// and the offset / 4 in counter words 0-1.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long off = (((unsigned long long)c1 << 32) | c0) * 4ull;
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
        std::printf("%08x %08x %08x %08x\n", a, b, c, d);
    }
    return 0;
}
