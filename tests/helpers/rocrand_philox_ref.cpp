// Reference Philox4x32-10 outputs from rocRAND's own header implementation, run
// on the host. Used only by the test that pins the oracle's Philox: the two
// implementations are independent, so agreement on many (key, counter) pairs
// checks the round function, the multipliers, the key schedule and the word
// order together.
//
// stdin : lines "k0 k1 c0 c1 c2 c3" (hex words), with c1 < 2^30
// stdout: lines "x0 x1 x2 x3" (hex words) = Philox4x32-10(key, counter)
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main()
{
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        const unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        const unsigned long long subsequence = ((unsigned long long)c3 << 32) | c2;
        const unsigned long long offset = 4ull * (((unsigned long long)c1 << 32) | c0);
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subsequence, offset, &st);
        unsigned x0 = rocrand(&st), x1 = rocrand(&st), x2 = rocrand(&st), x3 = rocrand(&st);
        std::printf("%08x %08x %08x %08x\n", x0, x1, x2, x3);
    }
    return 0;
}
