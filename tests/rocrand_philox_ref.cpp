// Reference Philox4x32-10 outputs from rocRAND (a library routine, used only
// to pin the oracle's own Philox).  Reads lines "c0 c1 c2 c3 k0 k1" and
// prints the four output words of Philox4x32-10(counter, key).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        // counter words 2,3 come from the subsequence, word 0 from the offset
        rocrand_init(seed, sub, 4ull * c0, &st);
        // word 1: each skip of 2^34 numbers adds 2^32 counter values, i.e. +1 to word 1
        unsigned long long rem = c1;
        while (rem) {
            unsigned long long piece = rem < (1ull << 29) ? rem : (1ull << 29);
            skipahead(piece << 34, &st);
            rem -= piece;
        }
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
