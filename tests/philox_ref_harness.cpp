// Known-answer harness for the oracle's Philox4x32-10: prints the block that
// ROCm's rocRAND engine (an independent implementation, used here only as a
// reference) produces for a 64-bit key and the counter (c0 c1 c2 c3), given as
// two 64-bit halves.  Reads "key c01 c23" lines from stdin.
#include <cstdio>
#include <cstdlib>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long key, c01, c23;
    while (std::scanf("%llu %llu %llu", &key, &c01, &c23) == 3) {
        // The engine's counter is (offset/4 as 64 bits, subsequence as 64 bits).
        rocrand_device::philox4x32_10_engine e(key, c23, c01 * 4ull);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
