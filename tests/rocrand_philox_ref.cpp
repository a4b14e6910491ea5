// Host program: Philox4x32-10 words from rocRAND's own generator (its
// header-only engine compiled for the host).  Used by the CPU test that pins
// the oracle's Philox.  Reads "c0 c1 c2 c3 k0 k1" lines (hex) from stdin and
// prints the four output words of that counter block.
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main()
{
    unsigned c[4], k[2];
    while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
        unsigned long long subsequence = ((unsigned long long)c[3] << 32) | c[2];
        unsigned long long offset = 4ull * (((unsigned long long)c[1] << 32) | c[0]);
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subsequence, offset, &st);
        unsigned w0 = rocrand(&st), w1 = rocrand(&st), w2 = rocrand(&st), w3 = rocrand(&st);
        std::printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
    }
    return 0;
}
