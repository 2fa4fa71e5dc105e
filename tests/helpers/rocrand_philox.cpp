// Test helper: prints Philox4x32-10 blocks computed by rocRAND's host/device
// engine, used only to cross-check the oracle's own Philox implementation.
// Input lines: "seed c0 c1 c2 c3" (decimal).  Output lines: "w0 w1 w2 w3".
// rocRAND's engine keys on the 64-bit seed; its 128-bit counter is reached
// with discard_subsequence (upper 64 bits) and discard (4 numbers per block).
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main() {
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        unsigned long long lo = c0 | (c1 << 32);
        unsigned long long hi = c2 | (c3 << 32);
        rocrand_device::philox4x32_10_engine eng(seed, hi, 0ull);
        // discard(4*lo) would overflow for large lo; advance in two halves
        eng.discard(2ull * lo);
        eng.discard(2ull * lo);
        unsigned w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
