// Host-only probe: prints rocRAND's Philox4x32-10 output for given
// (key, counter) pairs, as an implementation independent of the oracle's.
// rocRAND's engine(seed, subsequence, offset) starts from counter
// (0, 0, lo32(subsequence), hi32(subsequence)) and adds offset/4 to the
// 64-bit (word1:word0) half, with key = (lo32(seed), hi32(seed)).
// Input lines: key0 key1 c0 c1 c2 c3 (hex).  Output: four hex words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long off = (((unsigned long long)c1 << 32) | c0) * 4ULL;
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
        std::printf("%08x %08x %08x %08x\n", a, b, c, d);
    }
    return 0;
}
