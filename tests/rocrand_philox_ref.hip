// Host-only reference for the Philox4x32-10 pin: prints rocRAND's
// philox4x32_10 output for counters (c, i, 0, 0) and key (seed_lo, seed_hi),
// reached through rocRAND's public skip-ahead API: the counter is advanced by
// X = i*2^32 + c positions of four words, taken as two skips of 2X words each
// so that no offset overflows 64 bits for any i < 2^31.
// Reads "seed i c" triples from stdin, writes four words per line.
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main()
{
    unsigned long long seed, i, c;
    while (std::scanf("%llu %llu %llu", &seed, &i, &c) == 3) {
        rocrand_state_philox4x32_10 st;
        const unsigned long long X = (i << 32) + c;
        rocrand_init(seed, 0ull, 2ull * X, &st);
        skipahead(2ull * X, &st);
        uint4 w = rocrand4(&st);
        std::printf("%u %u %u %u\n", w.x, w.y, w.z, w.w);
    }
    return 0;
}
