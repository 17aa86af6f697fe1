// Reference Philox4x32-10 outputs from rocRAND's host-callable engine (a library
// routine), used to pin the oracle's own Philox.  Reads lines
// "k0 k1 c0 c1 c2 c3" (decimal) from stdin and prints the four output words.
// rocRAND's engine(seed, subsequence, offset) starts at key = seed and counter
// (offset/4 low, offset/4 high, subsequence low, subsequence high).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long subsequence = c2 | (c3 << 32);
        unsigned long long offset = 4ULL * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, subsequence, offset);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
