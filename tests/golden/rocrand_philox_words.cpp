// Prints Philox4x32-10 words computed by rocRAND's own engine (host side),
// used as an external reference for the oracle's generator.  Input lines on
// stdin: "c0 c1 c2 c3 k0 k1" (hex); output lines: four hex words.
// rocRAND's engine maps seed -> key (lo, hi), subsequence -> counter words
// 2..3 and offset/4 -> counter words 0..1, so a counter/key pair is reached
// by seeding with the key, skipping to subsequence (c2, c3) and offset
// 4 * (c0, c1).
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long off = 4ull * (((unsigned long long)c1 << 32) | c0);
        rocrand_device::philox4x32_10_engine eng(seed, sub, off);
        unsigned w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
        std::printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
    }
    return 0;
}
