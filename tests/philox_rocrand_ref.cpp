// Reference Philox4x32-10 blocks from rocRAND (test-only): reads lines
// "c0 c1 c2 c3 k0 k1" and prints the four output words of rocRAND's
// philox4x32_10 engine for that counter and key. The library is run, not
// copied: it is an independent implementation to pin the oracle against.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

// ten_rounds is a protected member of the engine; a derived class exposes it.
struct Engine : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    Engine eng;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 ctr;
        ctr.x = c0; ctr.y = c1; ctr.z = c2; ctr.w = c3;
        uint2 key;
        key.x = k0; key.y = k1;
        const uint4 r = eng.ten_rounds(ctr, key);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
