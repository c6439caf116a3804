// Independent Philox4x32-10 for pinning the oracle: the host-callable
// ten-round block function of rocRAND's philox4x32_10 engine (source header shipped with
// ROCm).  Reads lines "c0 c1 c2 c3 k0 k1" (decimal) and prints the four
// output words of each block.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

// ten_rounds() is a protected member; a derived class exposes it.
struct philox_probe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    philox_probe eng;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 ctr{c0, c1, c2, c3};
        uint2 key{k0, k1};
        uint4 o = eng.block(ctr, key);
        std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
