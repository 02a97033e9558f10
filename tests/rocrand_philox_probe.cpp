// Black-box Philox4x32-10 outputs from rocRAND's host-callable engine, used to
// pin the oracle's independent implementation.  Reads lines
// "seed c0 c1 c2 c3" and prints the four 32-bit words of the block with key
// (seed lo, seed hi) and counter (c0, c1, c2, c3).  The engine's counter is
// reached through its (subsequence, offset) seeding: subsequence fills
// counter words 2-3, offset/4 fills words 0-1 (c1 must stay below 2^30).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
    unsigned long long seed;
    unsigned c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, subseq, off);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
