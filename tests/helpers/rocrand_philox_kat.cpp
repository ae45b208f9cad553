// Independent Philox4x32-10 reference for the oracle's generator: rocRAND's
// header-only engine, run on the host.  For each line "seed subsequence
// offset" on stdin it prints the next four 32-bit words of the engine.  The
// engine's counter is (offset / 4 as 64 bits, subsequence as 64 bits) and its
// key is the seed split into two 32-bit halves.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
