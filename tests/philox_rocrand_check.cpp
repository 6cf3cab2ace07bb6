// Host program for the oracle's generator pin: evaluates Philox4x32-10 with
// rocRAND's open-source implementation (an implementation independent of
// the oracle) and prints the four output words for every
// (counter, key) line read from stdin.  Built and run by the CPU tests.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct Exposed : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    Exposed e;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c; c.x = c0; c.y = c1; c.z = c2; c.w = c3;
        uint2 k; k.x = k0; k.y = k1;
        uint4 r = e.block(c, k);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
