// Independent Philox4x32-10 reference for the oracle's pin test: runs
// rocRAND's open-source philox4x32_10 engine on the host CPU.
// Input lines: c0 c1 c2 c3 seed   (c1 < 2^30 so that the engine's counter
// offset 4*(c0 | c1<<32) fits in 64 bits).  Output: the four words of the
// block at counter (c0, c1, c2, c3) with key (seed lo, seed hi).
// rocRAND seeds key = seed, counter.zw = subsequence, counter.xy = offset/4.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3;
    unsigned long long seed;
    while (std::scanf("%u %u %u %u %llu", &c0, &c1, &c2, &c3, &seed) == 5) {
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
