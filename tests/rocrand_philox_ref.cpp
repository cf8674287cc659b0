// Host-only reference: evaluates Philox4x32-10 with rocRAND's header-only engine, an
// implementation independent of the oracle's.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal)
// from stdin and prints "o0 o1 o2 o3" per line.  rocRAND's engine maps (seed, subsequence,
// offset) to key = (seed lo, seed hi) and counter = (offset/4 lo, offset/4 hi, subsequence lo,
// subsequence hi); the offset is advanced in pieces to avoid overflowing 4 * offset.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const unsigned long long seed = k0 | (static_cast<unsigned long long>(k1) << 32);
        const unsigned long long sub = c2 | (static_cast<unsigned long long>(c3) << 32);
        const unsigned long long off = c0 | (static_cast<unsigned long long>(c1) << 32);
        rocrand_device::philox4x32_10_engine e(seed, sub, 0);
        const unsigned long long q = off >> 2, r = off & 3;
        for (int i = 0; i < 4; ++i) e.discard(4 * q);
        if (r) e.discard(4 * r);
        const uint4 o = e.next4();
        std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
