// Reference Philox4x32-10 outputs from rocRAND's engine (host side), used to pin
// the oracle's Philox.  Reads lines "k0 k1 c0 c1 c2 c3" (decimal) on stdin and
// prints the four output words.  Counter words (c0, c1) are the engine's
// offset / 4 and (c2, c3) its subsequence; key = seed.
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main()
{
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = (k1 << 32) | k0;
        unsigned long long sub = (c3 << 32) | c2;
        unsigned long long off = 4ull * ((c1 << 32) | c0);
        rocrand_state_philox4x32_10 st(seed, sub, off);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
