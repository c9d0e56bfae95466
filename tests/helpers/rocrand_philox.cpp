// Prints rocRAND's Philox4x32-10 block for (key, counter) pairs read from
// stdin, one "k0 k1 c0 c1 c2 c3" line each (hex).  rocRAND keys the engine
// with the 64-bit seed and starts the counter at (offset/4, subsequence),
// so counter (c0,c1,c2,c3) is reached with subsequence = c2 | c3 << 32 and
// offset = 4 * (c0 | c1 << 32).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        uint4 r = e.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
