// Reference Philox4x32-10 outputs from rocRAND's own engine (header source),
// used only to pin the oracle's generator.  Reads lines "k0 k1 c0 c1 c2 c3"
// and prints the four output words of the block with that key and counter.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main() {
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        // seed -> key (low, high); subsequence -> counter words 2, 3;
        // offset / 4 -> counter words 0, 1 (applied in four steps so the
        // 64-bit offset argument never overflows).
        rocrand_device::philox4x32_10_engine e(k0 | (k1 << 32), c2 | (c3 << 32), 4ull * c0);
        for (int i = 0; i < 4; ++i) e.discard(c1 << 32);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
