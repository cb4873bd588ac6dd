// Reference Philox4x32-10 outputs from rocRAND's engine, used by the tests to
// pin the oracle's own Philox.  Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin
// and prints the four output words of that counter block under that key.
// The engine's state is (counter, key) with key = (seed lo, seed hi); seeding
// with subsequence (c2 | c3 << 32) and offset 4 * (c0 | c1 << 32) places the
// counter at (c0, c1, c2, c3), so its next four outputs are that block.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        const unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        const unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        unsigned a = eng(), b = eng(), c = eng(), d = eng();
        std::printf("%08x %08x %08x %08x\n", a, b, c, d);
    }
    return 0;
}
