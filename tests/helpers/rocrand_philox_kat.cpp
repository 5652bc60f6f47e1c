// Test helper: prints rocRAND's Philox4x32-10 block for counters read from
// stdin ("c0 c1 c2 c3 seed" per line, decimal), using only the library's
// public engine API.  rocRAND is an independent implementation of the
// published generator, so agreement pins the oracle's Philox.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long c0, c1, c2, c3, seed;
    while (std::scanf("%llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &seed) == 5) {
        // counter = (x, y, z, w): subsequence advances (z, w), offset/4 advances (x, y)
        unsigned long long subsequence = c2 | (c3 << 32);
        unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, subsequence, offset);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
