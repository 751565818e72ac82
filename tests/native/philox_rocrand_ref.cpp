// Independent Philox4x32-10 for pinning the oracle's generator: rocRAND's
// header implementation, run on the host (no GPU call is made).
// stdin: lines "c0 c1 c2 c3 k0 k1" (decimal u32); stdout: four words per line.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct PhiloxProbe : rocrand_device::philox4x32_10_engine {
    uint4 apply(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    PhiloxProbe p;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c = make_uint4(c0, c1, c2, c3);
        uint2 k = make_uint2(k0, k1);
        uint4 r = p.apply(c, k);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
