// Prints rocRAND's Philox4x32-10 block function for (counter, key) tuples
// given on the command line: c0 c1 c2 c3 k0 k1 [...].  Host-only; used to
// pin the oracle's Philox against an independent implementation.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>
#include <cstdlib>

struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main(int argc, char** argv)
{
    Probe p;
    for (int a = 1; a + 5 < argc + 1; a += 6) {
        uint4 c = { (unsigned)strtoul(argv[a], 0, 0), (unsigned)strtoul(argv[a + 1], 0, 0),
                    (unsigned)strtoul(argv[a + 2], 0, 0), (unsigned)strtoul(argv[a + 3], 0, 0) };
        uint2 k = { (unsigned)strtoul(argv[a + 4], 0, 0), (unsigned)strtoul(argv[a + 5], 0, 0) };
        uint4 o = p.block(c, k);
        std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
