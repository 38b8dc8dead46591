// Host-only helper for the oracle's Philox pin: evaluates rocRAND's
// independent Philox4x32-10 engine (open-source header) on the host.
// stdin: lines "k0 k1 c0 c1 c2 c3"; stdout: the four output words.
// rocRAND's engine seeded with (seed = k1:k0, subsequence = c3:c2,
// offset = 4 * (c1:c0)) starts exactly at counter (c0, c1, c2, c3).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
        unsigned long long offset = 4ull * (((unsigned long long)c1 << 32) | c0);
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, offset, &st);
        unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
