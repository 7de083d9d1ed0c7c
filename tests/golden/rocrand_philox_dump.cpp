// Host-only helper for the oracle's RNG test: prints Philox4x32-10 outputs of
// rocRAND's engine (an independent implementation of the published
// generator) for counter/key pairs read from stdin, one per line as 6 hex words.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct exposed : rocrand_device::philox4x32_10_engine {
    static uint4 rounds(uint4 c, uint2 k)
    {
        exposed e;
        return e.ten_rounds(c, k);
    }
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = exposed::rounds(make_uint4(c0, c1, c2, c3), make_uint2(k0, k1));
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
