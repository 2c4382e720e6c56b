// Host-side reference for the oracle's Philox4x32-10: evaluates rocRAND's
// philox4x32_10 engine (an independent implementation of Salmon et al.,
// SC'11) on the host.  Reads lines "k0 k1 c0 c1 c2 c3" (decimal uint32) and
// prints the four output words.  rocrand_init(seed, subsequence, offset)
// places seed in the key, subsequence in counter words 2-3 and offset / 4 in
// counter words 0-1, so offset = 4 * (c0 + 2^32 c1) selects counter c.
#include <cstdio>
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_kernel.h>

int main() {
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(k0 | (k1 << 32), c2 | (c3 << 32), 4ull * (c0 | (c1 << 32)), &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
