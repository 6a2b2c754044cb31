// Prints Philox4x32-10 blocks computed by rocRAND's engine, one line per
// (key0 key1 ctr0 ctr1 ctr2 ctr3) line read from stdin.  Used only by the
// CPU tests, to pin the oracle's own Philox against an independent library.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        // the engine's (seed, subsequence, offset) places the key in the two
        // key words, the subsequence in counter words 2-3 and offset / 4 in
        // counter words 0-1 (offset counts 32-bit outputs)
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%08x %08x %08x %08x\n", a, b, c, d);
    }
    return 0;
}
