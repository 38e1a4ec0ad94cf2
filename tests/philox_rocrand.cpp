// Prints rocRAND's Philox4x32-10 block for (key, counter) pairs read from
// stdin, one "seed x y z w" line each (x, y, z, w = counter words, y < 2^30).
// rocRAND is an independent implementation of the same published generator;
// tests use this program to pin the oracle's and the literal reference's
// Philox.  Host-only: no GPU is touched.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned long long seed;
    unsigned int x, y, z, w;
    while (std::scanf("%llu %u %u %u %u", &seed, &x, &y, &z, &w) == 5) {
        // rocRAND's engine places the skip-ahead offset (in 32-bit outputs,
        // four per block) in counter words 0-1 and the subsequence in 2-3.
        unsigned long long offset = 4ull * ((unsigned long long)y << 32 | x);
        unsigned long long subsequence = (unsigned long long)w << 32 | z;
        rocrand_device::philox4x32_10_engine e(seed, subsequence, offset);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
