// Independent Philox4x32-10 reference for the oracle's pin: runs the
// header-only rocRAND engine on the host.  Reads lines "c0 c1 c2 c3 k0 k1"
// (hex) and prints the four output words of Philox4x32-10(counter, key).
// rocRAND's engine takes the key as a 64-bit seed (low word = key word 0) and
// builds the 128-bit counter from a 64-bit subsequence (words 2, 3) and a
// 64-bit offset counted in single outputs (four per counter step, words 0, 1).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long step = (unsigned long long)c0 | ((unsigned long long)(c1 & 0x3fffffffu) << 32);
        rocrand_device::philox4x32_10_engine e(seed, subseq, 4ull * step);
        // discard(2^62 outputs) advances the counter by 2^60, i.e. word 1 by 2^28
        for (unsigned k = 0; k < 4u * (c1 >> 30); ++k)
            e.discard(1ull << 62);
        uint4 r = e.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
