// Test helper: prints rocRAND's Philox4x32-10 block for (seed, subsequence,
// offset) triples read from stdin. rocRAND's engine is an implementation
// written independently of this project; it pins the oracle's generator.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        uint4 v = e.next4();
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
