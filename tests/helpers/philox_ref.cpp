// Independent Philox4x32-10 reference for the oracle's pin tests: the rocRAND
// host/device engine (a third-party implementation), driven on the CPU.
// stdin: lines "c0 c1 c2 c3 k0 k1" (decimal); stdout: "o0 o1 o2 o3".
// rocRAND's engine with seed s, subsequence t and offset 4*b evaluates the
// Philox bijection at counter (b lo, b hi, t lo, t hi) under key (s lo, s hi).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long sub = c2 | (c3 << 32);
        unsigned long long off = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned o0 = e(), o1 = e(), o2 = e(), o3 = e();
        std::printf("%u %u %u %u\n", o0, o1, o2, o3);
    }
    return 0;
}
