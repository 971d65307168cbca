// Independent reference for the oracle's Philox4x32-10: rocRAND's engine, evaluated on
// the host.  The engine is positioned at counter (x, y, z, w) with key (lo, hi) by
// seeding with the 64-bit key, subsequence (w:z) and offset 4*(y:x); its next four
// outputs are then the four words of Philox(counter, key).
// Reads lines "key_lo key_hi c0 c1 c2 c3" (decimal) on stdin, prints four words each.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdint>

int main()
{
    unsigned long long klo, khi, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &klo, &khi, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = (khi << 32) | klo;
        unsigned long long subsequence = (c3 << 32) | c2;
        unsigned long long offset = ((c1 << 32) | c0) * 4ull;
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
        unsigned int w0 = eng.next(), w1 = eng.next(), w2 = eng.next(), w3 = eng.next();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
