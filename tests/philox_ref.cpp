// Reference Philox4x32-10 outputs from the rocRAND library's host-callable engine, used
// to pin the oracle's independent implementation.  Reads lines "c0 c1 c2 c3 k0 k1" on
// stdin and prints the four output words of each.  The engine takes the key from the
// 64-bit seed, the low counter words from offset/4 and the high ones from the
// subsequence number.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned int c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long offset = (((unsigned long long)c1 << 32) | c0) * 4ull;
        unsigned long long subsequence = ((unsigned long long)c3 << 32) | c2;
        rocrand_device::philox4x32_10_engine e(seed, subsequence, 0ull);
        e.discard(offset);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
